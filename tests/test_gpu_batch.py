"""GPU parity of the batched persistent voter: every task of a mixed batch is
identical to the oracle and to ftv_vote on the same task, under every schedule
the autotuner may pick, and across graph replays."""
import ctypes

import numpy as np
import pytest

import oracle
from test_gpu_vote import U, _replicas

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu):
    c = gpu.Context(0)
    yield c
    c.close()


def _tol_pair(ftv, dtype, rng):
    if np.dtype(dtype).kind == "i":
        return oracle.exact(), ftv.exact()
    c = rng.integers(0, 4)
    if c == 0:
        return oracle.rel(1e-3), ftv.rel(1e-3)
    if c == 1:
        return oracle.exact(), ftv.exact()
    m = 4 if dtype == np.float32 else 2
    return oracle.ulp(m), ftv.ulp(m)


def make_batch(ftv, rng, ntasks, max_elems, ks=(2, 3, 4, 5, 6, 7)):
    import torch
    dev = torch.device("cuda:0")
    tasks = []
    for i in range(ntasks):
        dtype = [np.float32, np.float64, np.int32, np.int64][rng.integers(0, 4)]
        k = int(rng.choice(ks))
        n = int(np.exp(rng.uniform(0, np.log(max_elems)))) if rng.random() > 0.05 else int(rng.integers(0, 5))
        reps = _replicas(rng, dtype, k, n)
        tol_o, tol_f = _tol_pair(ftv, dtype, rng)
        t_reps = [torch.from_numpy(r).to(dev) for r in reps]
        cons = torch.empty(max(n, 1), dtype=t_reps[0].dtype, device=dev)
        mask = torch.empty(max(n, 1), dtype=torch.uint8, device=dev)
        tasks.append(dict(reps=reps, t_reps=t_reps, tol_o=tol_o, tol_f=tol_f, cons=cons, mask=mask, n=n, k=k))
    stats = ftv.stats_tensor(dev, len(tasks))
    descs = []
    for i, t in enumerate(tasks):
        d = ftv.make_desc(t["t_reps"], t["tol_f"], t["cons"], t["mask"], None, n=t["n"])
        d.stats = stats.data_ptr() + i * ctypes.sizeof(ftv.Stats)
        descs.append(d)
    return tasks, descs, stats


def outputs(ftv, tasks, stats):
    import torch
    torch.cuda.synchronize()
    out = []
    for i, t in enumerate(tasks):
        out.append((t["cons"][:t["n"]].cpu().numpy().copy(), t["mask"][:t["n"]].cpu().numpy().copy(),
                    ftv.read_stats(stats, i)))
    return out


def same(a, b):
    for (c1, m1, s1), (c2, m2, s2) in zip(a, b):
        u = U[c1.dtype]
        if not (np.array_equal(c1.view(u), c2.view(u)) and np.array_equal(m1, m2)):
            return False
        if any(not np.array_equal(s1[key], s2[key]) for key in s1):
            return False
    return True


def check_oracle(tasks, got):
    for i, (t, (c, m, s)) in enumerate(zip(tasks, got)):
        ref = oracle.vote(t["reps"], t["tol_o"])
        u = U[ref.consensus.dtype]
        assert np.array_equal(c.view(u), ref.consensus.view(u)), f"task {i} consensus"
        assert np.array_equal(m, ref.mask), f"task {i} mask"
        k = t["k"]
        assert np.array_equal(s["pair"][:k, :k], ref.pair), f"task {i} pair"
        assert np.array_equal(s["disagree"][:k], ref.disagree), f"task {i} disagree"
        assert s["no_majority"] == ref.no_majority and s["n"] == t["n"], f"task {i}"
        assert (s["verdict"], s["winner"]) == (ref.verdict, ref.winner), f"task {i} verdict"


def test_mixed_batch_matches_oracle_and_per_task(gpu, ctx):
    rng = np.random.default_rng(2024)
    print("case: mixed batch of 300 tasks, up to 40000 elements", flush=True)
    tasks, descs, stats = make_batch(gpu, rng, 300, 40000)
    gpu.vote_batch(ctx, descs)
    got = outputs(gpu, tasks, stats)
    check_oracle(tasks, got)
    # per-task launches on the same tasks give the same bits
    for d in descs:
        gpu.load().ftv_vote(ctx.handle, ctypes.byref(d), None)
    assert same(outputs(gpu, tasks, stats), got)


def test_every_schedule_gives_identical_results(gpu, ctx):
    rng = np.random.default_rng(7)
    tasks, descs, stats = make_batch(gpu, rng, 120, 200000, ks=(2, 3, 5))
    gpu.vote_batch(ctx, descs)
    ref = outputs(gpu, tasks, stats)
    check_oracle(tasks, ref)
    for tv in (256, 1024, 4096, 65536):
        for block in (256, 512):
            for gm in (1, 3, 8):
                for order in (0, 1, 2, 3):
                    cfg = gpu.BatchCfg(tv, block, gm, order, (tv + order) % 2, 0)
                    print(f"case: schedule tile={tv} block={block} grid={gm} order={order}", flush=True)
                    ctx.set_batch_config(cfg)
                    gpu.vote_batch(ctx, descs)
                    assert same(outputs(gpu, tasks, stats), ref), (tv, block, gm, order)
    best = gpu.tune_batch(ctx, descs, iters=2)
    assert same(outputs(gpu, tasks, stats), ref)
    assert best.block in (256, 512)


def test_graph_replays_and_batch_changes(gpu, ctx):
    """Replay the captured graph many times with different tables, with eager
    work in between; every replay must match the oracle."""
    import torch
    rng = np.random.default_rng(99)
    batches = [make_batch(gpu, rng, n, 30000) for n in (50, 5, 200)]
    refs = []
    for tasks, descs, stats in batches:
        gpu.vote_batch(ctx, descs)
        got = outputs(gpu, tasks, stats)
        check_oracle(tasks, got)
        refs.append(got)
    for rep in range(4):
        for (tasks, descs, stats), ref in zip(batches, refs):
            stats.zero_()
            for t in tasks:
                t["cons"].zero_()
                t["mask"].fill_(0xEE)
            gpu.vote_batch(ctx, descs)
            _ = torch.ones(1000, device="cuda").sum().item()
            assert same(outputs(gpu, tasks, stats), ref), rep


def test_batch_alignment_is_checked(gpu, ctx):
    import torch
    x = torch.zeros(64, dtype=torch.float32, device="cuda")
    st = gpu.stats_tensor("cuda")
    d = gpu.make_desc([x[1:], x[1:], x[1:]], gpu.ulp(1), None, None, st)
    with pytest.raises(gpu.FtvError) as e:
        gpu.vote_batch(ctx, [d])
    assert e.value.code == gpu.E_ALIGN


def test_tune_cache_roundtrip(gpu, ctx, tmp_path, monkeypatch):
    """The autotuner stores its choice as JSON and reuses it on a cache hit;
    the cached schedule gives the same results."""
    import json
    rng = np.random.default_rng(44)
    tasks, descs, stats = make_batch(gpu, rng, 40, 50000, ks=(2, 3, 5))
    path = tmp_path / "tune.json"
    monkeypatch.setenv("FTV_TUNE_CACHE", str(path))
    best = gpu.tune_batch(ctx, descs, iters=1)
    ref = outputs(gpu, tasks, stats)
    check_oracle(tasks, ref)
    doc = json.loads(path.read_text())
    assert len(doc) == 1
    (key, val), = doc.items()
    assert val == [best.tile_vecs, best.block, best.grid_mult, best.order, best.nt_stores]
    # a different schedule in the cache file is picked up as is
    path.write_text(json.dumps({key: [1024, 512, 2, 2, 0]}))
    again = gpu.tune_batch(ctx, descs, iters=1)
    assert (again.tile_vecs, again.block, again.grid_mult, again.order, again.nt_stores) == (1024, 512, 2, 2, 0)
    assert same(outputs(gpu, tasks, stats), ref)


def test_batch_planted_nonzero_argmin_winners(gpu, ctx):
    """Tasks whose winner is a non-zero argmin of the disagree counts
    (ELEMENT_MAJORITY and UNRESOLVED), mixed with ordinary tasks in one batch:
    identical to the oracle."""
    import torch
    import synth
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(515)
    tasks, _, _ = make_batch(gpu, rng, 40, 30000, ks=(2, 3, 5))
    cases = []
    for dtype in ("f32", "f64", "i32", "i64"):
        for per in ([40, 10, 30], [40, 10, 30, 10, 50], [40, 10, 30, 10, 50, 60, 70]):
            for nomaj in (0, 2):
                cases.append((dtype, per, nomaj))
    for j, (dtype, per, nomaj) in enumerate(cases):
        n = 50000 + 1237 * j
        _, reps = synth.planted_set(dtype, n, per, nomaj, seed=synth.SEED_BASE + 100 + j)
        if dtype[0] == "i":
            tol_o, tol_f = oracle.exact(), gpu.exact()
        else:
            tol_o, tol_f = oracle.ulp(4), gpu.ulp(4)
        t_reps = [torch.from_numpy(r).to(dev) for r in reps]
        tasks.append(dict(reps=reps, t_reps=t_reps, tol_o=tol_o, tol_f=tol_f,
                          cons=torch.empty(n, dtype=t_reps[0].dtype, device=dev),
                          mask=torch.empty(n, dtype=torch.uint8, device=dev), n=n, k=len(per)))
    stats = gpu.stats_tensor(dev, len(tasks))
    descs = []
    for i, t in enumerate(tasks):
        d = gpu.make_desc(t["t_reps"], t["tol_f"], t["cons"], t["mask"], None, n=t["n"])
        d.stats = stats.data_ptr() + i * ctypes.sizeof(gpu.Stats)
        descs.append(d)
    print(f"case: batch of {len(tasks)} tasks with {len(cases)} planted non-zero winners", flush=True)
    gpu.vote_batch(ctx, descs)
    got = outputs(gpu, tasks, stats)
    check_oracle(tasks, got)
    nz = sum(1 for (_, _, s) in got[-len(cases):] if s["winner"] != 0 and s["verdict"] >= 2)
    assert nz == len(cases)
