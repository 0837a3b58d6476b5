"""GPU parity: ftv_vote (through the C ABI) against the CPU oracle, bit for bit.

Consensus bits, mask bytes, the k x k mismatch counts, the disagreement and
no-majority counts, the verdict and the winner must all be identical.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

U = {np.dtype(np.float32): np.uint32, np.dtype(np.float64): np.uint64,
     np.dtype(np.int32): np.uint32, np.dtype(np.int64): np.uint64}


def _tols(ftv, dtype):
    if np.dtype(dtype).kind == "i":
        return [(oracle.exact(), ftv.exact())]
    return [(oracle.exact(), ftv.exact()), (oracle.ulp(0), ftv.ulp(0)), (oracle.ulp(4), ftv.ulp(4)),
            (oracle.ulp(2 ** 40), ftv.ulp(2 ** 40)), (oracle.rel(1e-3), ftv.rel(1e-3)),
            (oracle.rel(1e-3, 1e-30), ftv.rel(1e-3, 1e-30))]


def _replicas(rng, dtype, k, n):
    dtype = np.dtype(dtype)
    if dtype.kind == "i":
        info = np.iinfo(dtype)
        base = rng.integers(info.min, info.max, n, dtype=dtype, endpoint=True)
        reps = []
        for r in range(k):
            x = base.copy()
            idx = rng.choice(n, n // 10, replace=False) if n else np.zeros(0, int)
            x.view(U[dtype])[idx] ^= (np.ones(idx.size, U[dtype]) << rng.integers(0, 8 * dtype.itemsize, idx.size).astype(U[dtype]))
            reps.append(x)
        return reps
    base = rng.standard_normal(n).astype(dtype)
    sp = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 1e-45 if dtype == np.float32 else 5e-324,
                   -1e-40 if dtype == np.float32 else -1e-310], dtype=dtype)
    if n:
        idx = rng.choice(n, min(n, max(1, n // 50)), replace=False)
        base[idx] = sp[rng.integers(0, sp.size, idx.size)]
    reps = []
    for r in range(k):
        x = base.copy()
        synth.ulp_noise(x, 1234, r, round(0.3 * (1 << 24)), 6)
        if n:
            idx = rng.choice(n, max(1, n // 20), replace=False)
            x[idx] = rng.standard_normal(idx.size).astype(dtype) * (1 + 1e-3 * rng.standard_normal(idx.size))
            idx2 = rng.choice(n, max(1, n // 200), replace=False)
            x[idx2] = sp[rng.integers(0, sp.size, idx2.size)]
        reps.append(x)
    return reps


def _run(ftv, ctx, reps, tol_f, offset=0, want_cons=True, want_mask=True):
    import torch
    dev = torch.device("cuda:0")
    if offset:
        ts = []
        for r in reps:
            buf = torch.empty(r.size + offset, dtype=torch.from_numpy(r[:0]).dtype, device=dev)
            buf[offset:] = torch.from_numpy(r).to(dev)
            ts.append(buf[offset:])
    else:
        ts = [torch.from_numpy(r).to(dev) for r in reps]
    cons, mask, st = ftv.vote(ctx, ts, tol_f, want_consensus=want_cons, want_mask=want_mask)
    torch.cuda.synchronize()
    return (cons.cpu().numpy() if cons is not None else None,
            mask.cpu().numpy() if mask is not None else None, ftv.read_stats(st))


def _check(got, ref, k, where=""):
    cons, mask, s = got
    if cons is not None:
        u = U[ref.consensus.dtype]
        bad = np.nonzero(cons.view(u) != ref.consensus.view(u))[0]
        assert bad.size == 0, f"{where}: consensus differs at {bad[:8]}"
    if mask is not None:
        bad = np.nonzero(mask != ref.mask)[0]
        assert bad.size == 0, f"{where}: mask differs at {bad[:8]}"
    assert np.array_equal(s["pair"][:k, :k], ref.pair), where
    assert not s["pair"][k:, :].any() and not s["pair"][:, k:].any(), where
    assert np.array_equal(s["disagree"][:k], ref.disagree), where
    assert s["no_majority"] == ref.no_majority, where
    assert s["n"] == ref.mask.size, where
    assert (s["verdict"], s["winner"]) == (ref.verdict, ref.winner), where


@pytest.fixture(scope="module")
def ctx(gpu):
    c = gpu.Context(0)
    yield c
    c.close()


def test_small_task_set(gpu, ctx):
    print("case: small task set, n=2^20 k=3 fp32 ULP4", flush=True)
    reps = synth.small_task_set()
    ref = oracle.vote(reps, oracle.ulp(4))
    _check(_run(gpu, ctx, reps, gpu.ulp(4)), ref, 3, "small_task_set")
    assert ref.verdict == oracle.TASK_MAJORITY and ref.disagree[2] > 0


@pytest.mark.parametrize("dtype", [np.float32, np.float64, np.int32, np.int64])
def test_dtype_tol_k_matrix(gpu, ctx, dtype):
    rng = np.random.default_rng(100 + np.dtype(dtype).itemsize)
    n = 10003   # several workgroups of tiles and a ragged tail
    for k in range(2, 8):
        reps = _replicas(rng, dtype, k, n)
        for tol_o, tol_f in _tols(gpu, dtype):
            where = f"{np.dtype(dtype).name} k={k} tol={tol_o}"
            print("case:", where, flush=True)
            ref = oracle.vote(reps, tol_o)
            _check(_run(gpu, ctx, reps, tol_f), ref, k, where)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 7, 255, 256, 257, 2047, 2048, 2049, 4095, 65537])
def test_edge_sizes(gpu, ctx, n):
    rng = np.random.default_rng(n)
    for dtype, k in ((np.float32, 3), (np.float64, 5), (np.int32, 2)):
        reps = _replicas(rng, dtype, k, n)
        tol_o, tol_f = _tols(gpu, dtype)[-1 if np.dtype(dtype).kind == "f" else 0]
        print(f"case: n={n} {np.dtype(dtype).name} k={k}", flush=True)
        _check(_run(gpu, ctx, reps, tol_f), oracle.vote(reps, tol_o), k, f"n={n}")


@pytest.mark.parametrize("offset", [1, 2, 3])
def test_unaligned_scalar_path(gpu, ctx, offset):
    rng = np.random.default_rng(7 + offset)
    for dtype, k in ((np.float32, 3), (np.float64, 3), (np.int32, 4), (np.float32, 7)):
        reps = _replicas(rng, dtype, k, 3001)
        tol_o, tol_f = _tols(gpu, dtype)[2 if np.dtype(dtype).kind == "f" else 0]
        print(f"case: offset={offset} {np.dtype(dtype).name} k={k}", flush=True)
        _check(_run(gpu, ctx, reps, tol_f, offset=offset), oracle.vote(reps, tol_o), k, "unaligned")


def test_optional_outputs(gpu, ctx):
    rng = np.random.default_rng(11)
    reps = _replicas(rng, np.float32, 3, 5000)
    ref = oracle.vote(reps, oracle.ulp(4))
    for wc, wm in ((False, True), (True, False), (False, False)):
        print(f"case: consensus={wc} mask={wm}", flush=True)
        _check(_run(gpu, ctx, reps, gpu.ulp(4), want_cons=wc, want_mask=wm), ref, 3, "optional")


@pytest.mark.parametrize("dtype,k", [(np.float32, 2), (np.float32, 3), (np.float32, 5), (np.float32, 7),
                                     (np.float64, 2), (np.float64, 5), (np.float64, 7)])
def test_full_steps_and_optional_outputs(gpu, ctx, dtype, k):
    """Many full tiles of each launch shape, a partial tile and a ragged tail,
    under ULP and REL, with every combination of the optional outputs (a
    missing output's stores go to a zero-size buffer resource)."""
    rng = np.random.default_rng(500 + k)
    n = 200003
    reps = _replicas(rng, dtype, k, n)
    m = 4 if dtype == np.float32 else 2
    for tol_o, tol_f in ((oracle.ulp(m), gpu.ulp(m)), (oracle.rel(1e-3), gpu.rel(1e-3))):
        ref = oracle.vote(reps, tol_o)
        for wc, wm in ((True, True), (False, True), (True, False), (False, False)):
            where = f"{np.dtype(dtype).name} k={k} tol={tol_o} consensus={wc} mask={wm}"
            print("case:", where, flush=True)
            _check(_run(gpu, ctx, reps, tol_f, want_cons=wc, want_mask=wm), ref, k, where)


@pytest.mark.parametrize("dtype,k,tile_elems,exact", [(np.float32, 2, 4096, False), (np.float32, 3, 4096, False),
                                                      (np.int32, 2, 4096, True), (np.float64, 4, 1024, False),
                                                      (np.float64, 7, 512, False)])
def test_xcd_tile_order_many_rounds(gpu, ctx, dtype, k, tile_elems, exact):
    """The launch shapes that hand out a round's tiles XCD by XCD, with the
    full grid of one workgroup per CU, two and a half grid-stride rounds, a
    partial tile and a ragged tail: every element is voted once."""
    rng = np.random.default_rng(700 + k)
    n = 5 * 128 * tile_elems + tile_elems // 2 + 3
    reps = _replicas(rng, dtype, k, n)
    m = 4 if dtype == np.float32 else 2
    tols = [(oracle.exact(), gpu.exact())] if exact else [(oracle.ulp(m), gpu.ulp(m)), (oracle.rel(1e-3), gpu.rel(1e-3))]
    for tol_o, tol_f in tols:
        where = f"xcd order {np.dtype(dtype).name} k={k} n={n} tol={tol_o}"
        print("case:", where, flush=True)
        _check(_run(gpu, ctx, reps, tol_f), oracle.vote(reps, tol_o), k, where)


def test_repeat_is_deterministic(gpu, ctx):
    reps = synth.small_task_set(n=300001)
    a = _run(gpu, ctx, reps, gpu.ulp(4))
    b = _run(gpu, ctx, reps, gpu.ulp(4))
    assert np.array_equal(a[0].view(np.uint32), b[0].view(np.uint32)) and np.array_equal(a[1], b[1])
    assert all(np.array_equal(a[2][key], b[2][key]) for key in a[2])


def test_invalid_arguments_are_errors(gpu, ctx):
    import torch
    x = torch.zeros(16, dtype=torch.int32, device="cuda")
    with pytest.raises(gpu.FtvError) as e:
        gpu.vote(ctx, [x, x, x], gpu.ulp(2))
    assert e.value.code == gpu.E_DTYPE
    with pytest.raises(gpu.FtvError) as e:
        gpu.vote(ctx, [x], gpu.exact())
    assert e.value.code == gpu.E_K
    with pytest.raises(gpu.FtvError) as e:
        gpu.vote(ctx, [x, x, x], gpu.Tol(7, 0, 0, 0.0, 0.0))
    assert e.value.code == gpu.E_INVALID
    # a replica pointer that is not element-aligned is rejected before any launch
    import ctypes
    st = gpu.stats_tensor("cuda")
    d = gpu.make_desc([x, x, x], gpu.exact(), stats=st)
    d.replicas[1] = x.data_ptr() + 1
    rc = gpu.load().ftv_vote(ctx.handle, ctypes.byref(d), None)
    assert rc == gpu.E_ALIGN
    f = torch.zeros(16, dtype=torch.float32, device="cuda")
    with pytest.raises(gpu.FtvError) as e:
        gpu.vote(ctx, [f, f, f], gpu.rel(float("nan")))
    assert e.value.code == gpu.E_INVALID


def test_large_task_recipe_host_generated(gpu, ctx):
    for dtype, tol in (("f32", 4), ("f64", 2)):
        n = 1 << 20
        print(f"case: large-task recipe {dtype} n=2^20", flush=True)
        reps = synth.large_task_set(n, dtype, flip_rate=2e-5)
        ref = oracle.vote(reps, oracle.ulp(tol))
        _check(_run(gpu, ctx, reps, gpu.ulp(tol)), ref, 3, f"large_task_set {dtype}")
        assert ref.disagree[2] > 0 and ref.disagree[0] == 0 and ref.disagree[1] == 0


def test_device_generator_matches_host_generator(gpu):
    import torch
    import synth.device as sd
    for dtype, dist in (("f32", synth.UNIFORM), ("f64", synth.UNIFORM), ("f32", synth.NORMAL),
                        ("f64", synth.NORMAL), ("i32", synth.INTFULL), ("i64", synth.INTFULL)):
        td = {"f32": torch.float32, "f64": torch.float64, "i32": torch.int32, "i64": torch.int64}[dtype]
        t = torch.empty(50001, dtype=td, device="cuda")
        sd.fill(t, dtype, dist, 77, 5, offset=123)
        host = synth.values(dtype, dist, 77, 5, 50001, offset=123)
        got = t.cpu().numpy()
        assert np.array_equal(got.view(U[got.dtype]), host.view(U[host.dtype])), (dtype, dist)
    for dtype in ("f32", "f64"):
        host = synth.values(dtype, synth.NORMAL, 3, 0, 40000)
        t = torch.from_numpy(host.copy()).cuda()
        sd.ulp_noise(t, dtype, 3, 1, round(0.3 * (1 << 24)), 3)
        synth.ulp_noise(host, 3, 1, round(0.3 * (1 << 24)), 3)
        assert np.array_equal(t.cpu().numpy().view(U[host.dtype]), host.view(U[host.dtype]))
    a = sd.large_task_set(1 << 16, "f32")
    b = synth.large_task_set(1 << 16, "f32")
    for x, y in zip(a, b):
        assert np.array_equal(x.cpu().numpy().view(np.uint32), y.view(np.uint32))


@pytest.mark.parametrize("dtype,side,tol", [("f32", 16384, 4), ("f64", 8192, 2)])
def test_large_task_full_size(gpu, ctx, dtype, side, tol):
    """The full single-large-task workload, in the launch configuration the
    benchmark times, checked element by element against the oracle."""
    import torch
    import synth.device as sd
    n = side * side
    print(f"case: large task full size {dtype} {side}x{side}", flush=True)
    reps_d = sd.large_task_set(n, dtype)
    cons, mask, st = gpu.vote(ctx, reps_d, gpu.ulp(tol))
    torch.cuda.synchronize()
    s = gpu.read_stats(st)
    reps = [r.cpu().numpy() for r in reps_d]
    del reps_d
    ref = oracle.vote(reps, oracle.ulp(tol))
    _check((cons.cpu().numpy(), mask.cpu().numpy(), s), ref, 3, f"large_task_set full {dtype}")
    assert s["verdict"] == gpu.TASK_MAJORITY and s["winner"] == 0


@pytest.mark.parametrize("dtype", ["f32", "f64", "i32", "i64"])
def test_planted_nonzero_argmin_winner(gpu, ctx, dtype):
    """Every replica faulty somewhere (no TASK_MAJORITY), disagree counts with
    their minimum at replica 1 (tied with 3 for k >= 4): the winner of
    ELEMENT_MAJORITY and of UNRESOLVED (nomaj > 0) is a non-zero argmin.  n is
    ragged and spans many tiles of every launch shape."""
    n = 200003
    for per in ([40, 10, 30], [40, 10, 30, 10, 50], [40, 10, 30, 10, 50, 60, 70]):
        for nomaj in (0, 3):
            print(f"case: planted winner {dtype} k={len(per)} nomaj={nomaj}", flush=True)
            _, reps = synth.planted_set(dtype, n, per, nomaj)
            pairs = _tols(gpu, np.dtype(synth._np[dtype]))
            tol_o, tol_f = pairs[0] if dtype[0] == "i" else pairs[2]
            ref = oracle.vote(reps, tol_o)
            assert ref.winner != 0
            assert ref.verdict == (oracle.UNRESOLVED if nomaj else oracle.ELEMENT_MAJORITY)
            _check(_run(gpu, ctx, reps, tol_f), ref, len(per), f"planted {dtype} {per} {nomaj}")


def test_two_streams_share_a_context(gpu, ctx):
    """Votes issued alternately on two streams with one context, never
    synchronised in between: each stream counts in its own accumulators, so
    every stats record equals the oracle's (never counts of the other stream)."""
    import torch
    dev = torch.device("cuda:0")
    sets = []
    for j in range(2):
        _, reps = synth.planted_set("f32", 300001 + 17 * j, [40 + 7 * j, 10, 30 + j], 2 * j,
                                    seed=synth.SEED_BASE + 300 + j)
        sets.append((reps, oracle.vote(reps, oracle.ulp(4))))
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    t_reps = [[torch.from_numpy(r).to(dev) for r in reps] for reps, _ in sets]
    torch.cuda.synchronize()
    outs = [[gpu.stats_tensor(dev) for _ in range(8)] for _ in range(2)]
    print("case: two streams, one context, 8 interleaved votes each", flush=True)
    for i in range(8):
        for j in range(2):
            with torch.cuda.stream(streams[j]):
                gpu.vote(ctx, t_reps[j], gpu.ulp(4), stats=outs[j][i], want_consensus=False,
                         want_mask=False, stream=streams[j])
    torch.cuda.synchronize()
    for j in range(2):
        ref = sets[j][1]
        for i in range(8):
            s = gpu.read_stats(outs[j][i])
            assert np.array_equal(s["pair"][:3, :3], ref.pair), (j, i)
            assert np.array_equal(s["disagree"][:3], ref.disagree), (j, i)
            assert s["no_majority"] == ref.no_majority and (s["verdict"], s["winner"]) == (ref.verdict, ref.winner)


def _corrupted_set(rng, dtype, k, n):
    """k replicas: a base, rounding noise (+-1..3 ULP on 30% of the elements)
    on replica 1, replica 2 replaced by unrelated values; the rest copies of
    the base or of replica 1.  Most elements then hold three different bit
    patterns, the case the in-place general vote and the fix-up pass decide."""
    dtype = np.dtype(dtype)
    base = rng.standard_normal(n).astype(dtype)
    noisy = base.copy()
    synth.ulp_noise(noisy, 4321, 1, round(0.3 * (1 << 24)), 3)
    garbage = (rng.standard_normal(n) * 1e3).astype(dtype)
    reps = [base, noisy, garbage]
    for r in range(3, k):
        reps.append((base if r % 2 else noisy).copy())
    return reps[:k]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_corrupted_replica_with_rounding_noise(gpu, ctx, dtype):
    """Per-task launches (general vote in place) and one batched launch
    (k >= 4 through the fix-up pass) against the oracle, k = 3..7."""
    import ctypes
    import torch
    rng = np.random.default_rng(515 + np.dtype(dtype).itemsize)
    dev = torch.device("cuda:0")
    tasks = []
    for k in (3, 4, 5, 6, 7):
        reps = _corrupted_set(rng, dtype, k, 100003)
        for tol_o, tol_f in ((oracle.ulp(4), gpu.ulp(4)), (oracle.exact(), gpu.exact()),
                             (oracle.rel(1e-3), gpu.rel(1e-3))):
            where = f"corrupted {np.dtype(dtype).name} k={k} tol={tol_o}"
            print("case:", where, flush=True)
            ref = oracle.vote(reps, tol_o)
            _check(_run(gpu, ctx, reps, tol_f), ref, k, where)
            tasks.append((where, reps, tol_o, tol_f, ref))
    # the same tasks in one batched launch
    outs = []
    stats = gpu.stats_tensor(dev, len(tasks))
    descs = []
    for i, (where, reps, tol_o, tol_f, ref) in enumerate(tasks):
        t = [torch.from_numpy(r).to(dev) for r in reps]
        cons = torch.empty(reps[0].size, dtype=t[0].dtype, device=dev)
        mask = torch.empty(reps[0].size, dtype=torch.uint8, device=dev)
        d = gpu.make_desc(t, tol_f, cons, mask, None)
        d.stats = stats.data_ptr() + i * ctypes.sizeof(gpu.Stats)
        descs.append(d)
        outs.append((t, cons, mask))
    print(f"case: one batch of {len(descs)} corrupted-replica tasks", flush=True)
    gpu.vote_batch(ctx, descs)
    torch.cuda.synchronize()
    for i, (where, reps, tol_o, tol_f, ref) in enumerate(tasks):
        _, cons, mask = outs[i]
        _check((cons.cpu().numpy(), mask.cpu().numpy(), gpu.read_stats(stats, i)), ref, len(reps),
               "batched " + where)
