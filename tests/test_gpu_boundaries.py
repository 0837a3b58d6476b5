"""GPU parity at the edges of the tolerance decisions (Sec. IV-D: integers
bit-wise, floating point within a tolerance), bit for bit against the oracle.

The replica sets (edge_sets.boundary_set) put every element on a decision
edge: ULP steps around m across zero, denormals, +-max, +-inf and the NaN
keys, relative distances at the delta, ties, and sets with a random strict
majority per element.  The same sets go through the per-task vote, the
batched launch and the block vote's element-vote fallback.
"""
import ctypes

import numpy as np
import pytest

import oracle
from edge_sets import U, boundary_set

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu):
    c = gpu.Context(0)
    yield c
    c.close()


def _tols(ftv, dtype, m, delta):
    return [(oracle.ulp(m), ftv.ulp(m)), (oracle.exact(), ftv.exact()), (oracle.rel(delta), ftv.rel(delta)),
            (oracle.rel(delta, float(np.finfo(dtype).smallest_normal) * 4), ftv.rel(delta, float(np.finfo(dtype).smallest_normal) * 4))]


def _cases(ftv, dtype, seed):
    rng = np.random.default_rng(seed)
    n = 30011
    for k in (2, 3, 4, 5, 6, 7):
        for m, delta, anchored in ((1, 1e-3, False), (4, 1e-6, False), (1000, 1e-3, False), (4, 1e-3, True)):
            reps = boundary_set(rng, dtype, k, n, m, delta, anchored)
            for tol_o, tol_f in _tols(ftv, dtype, m, delta):
                yield (f"{np.dtype(dtype).name} k={k} m={m} delta={delta} anchored={anchored} tol={tol_o}",
                       reps, tol_o, tol_f)


def _compare(where, k, cons, mask, s, ref):
    u = U[ref.consensus.dtype]
    bad = np.nonzero(cons.view(u) != ref.consensus.view(u))[0]
    assert bad.size == 0, f"{where}: consensus differs at {bad[:8]}"
    bad = np.nonzero(mask != ref.mask)[0]
    assert bad.size == 0, f"{where}: mask differs at {bad[:8]}"
    assert np.array_equal(s["pair"][:k, :k], ref.pair), where
    assert np.array_equal(s["disagree"][:k], ref.disagree), where
    assert s["no_majority"] == ref.no_majority, where
    assert (s["verdict"], s["winner"]) == (ref.verdict, ref.winner), where


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_tolerance_edges_per_task(gpu, ctx, dtype):
    import torch
    nomaj, verdicts = 0, set()
    for where, reps, tol_o, tol_f in _cases(gpu, dtype, 31 + np.dtype(dtype).itemsize):
        print("case:", where, flush=True)
        t = [torch.from_numpy(r).cuda() for r in reps]
        cons, mask, st = gpu.vote(ctx, t, tol_f)
        torch.cuda.synchronize()
        ref = oracle.vote(reps, tol_o)
        _compare(where, len(reps), cons.cpu().numpy(), mask.cpu().numpy(), gpu.read_stats(st), ref)
        nomaj += ref.no_majority
        verdicts.add(ref.verdict)
    assert nomaj > 0   # the sets do reach elements without a majority
    assert verdicts >= {oracle.ELEMENT_MAJORITY, oracle.UNRESOLVED}


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_tolerance_edges_batched(gpu, ctx, dtype):
    import torch
    dev = torch.device("cuda:0")
    tasks = []
    for where, reps, tol_o, tol_f in _cases(gpu, dtype, 57 + np.dtype(dtype).itemsize):
        t = [torch.from_numpy(r).to(dev) for r in reps]
        cons = torch.empty(reps[0].size, dtype=t[0].dtype, device=dev)
        mask = torch.empty(reps[0].size, dtype=torch.uint8, device=dev)
        tasks.append((where, reps, tol_o, tol_f, t, cons, mask))
    stats = gpu.stats_tensor(dev, len(tasks))
    descs = []
    for i, (_, _, _, tol_f, t, cons, mask) in enumerate(tasks):
        d = gpu.make_desc(t, tol_f, cons, mask, None)
        d.stats = stats.data_ptr() + i * ctypes.sizeof(gpu.Stats)
        descs.append(d)
    print(f"case: one batch of {len(descs)} edge tasks ({np.dtype(dtype).name})", flush=True)
    gpu.vote_batch(ctx, descs)
    torch.cuda.synchronize()
    for i, (where, reps, tol_o, _, _, cons, mask) in enumerate(tasks):
        _compare("batched " + where, len(reps), cons.cpu().numpy(), mask.cpu().numpy(), gpu.read_stats(stats, i),
                 oracle.vote(reps, tol_o))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_tolerance_edges_block_fallback(gpu, ctx, dtype):
    """Nearly every 4 KiB block of these sets lacks a fingerprint majority, so
    the block vote decides them with its element-vote fallback."""
    import torch
    rng = np.random.default_rng(71 + np.dtype(dtype).itemsize)
    for k in (2, 3, 5, 7):
        m, delta = (4, 1e-3) if k % 2 else (1, 1e-6)
        reps = boundary_set(rng, dtype, k, 20011, m, delta)
        for tol_o, tol_f in _tols(gpu, dtype, m, delta):
            where = f"blocks {np.dtype(dtype).name} k={k} tol={tol_o}"
            print("case:", where, flush=True)
            t = [torch.from_numpy(r).cuda() for r in reps]
            out = gpu.vote_blocks(ctx, t, tol_f, 4096)
            torch.cuda.synchronize()
            ref = oracle.vote_blocks(reps, tol_o, 4096)
            u = U[np.dtype(dtype)]
            assert np.array_equal(out["blockmap"].cpu().numpy(), ref.blockmap), where
            assert np.array_equal(out["consensus"].cpu().numpy().view(u), ref.consensus.view(u)), where
            assert np.array_equal(out["mask"].cpu().numpy(), ref.mask), where
            s = gpu.read_block_stats(out["bstats"])
            assert (s["fallback_blocks"], s["unresolved_elems"], s["verdict"], s["winner"]) == \
                (ref.fallback_blocks, ref.unresolved_elems, ref.verdict, ref.winner), where
            assert ref.fallback_blocks > 0, where
