"""GPU parity at the edges of the tolerance decisions (Sec. IV-D: integers
bit-wise, floating point within a tolerance), bit for bit against the oracle.

Every element of these replica sets is built to sit on a decision edge: the
replicas of an element lie 0, 1, m-1, m, m+1 or 2m+1 ordered-key steps from
a base value (m = the ULP tolerance), so that each pair is just inside or
just outside the tolerance, with base values at +-0, the denormal range, the
smallest normal, +-max, +-inf and NaNs, where the steps cross zero, leave the
finite range or enter the NaN keys; or at relative distances of a fraction
(just below 1, 1, just above 1) of the relative delta; or split into two
equal-sized groups (ties, no strict majority).  The same sets go through the
per-task vote, the batched launch and the block vote's element-vote fallback.
"""
import ctypes

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

U = {np.dtype(np.float32): np.uint32, np.dtype(np.float64): np.uint64}


@pytest.fixture(scope="module")
def ctx(gpu):
    c = gpu.Context(0)
    yield c
    c.close()


def _step_keys(x: np.ndarray, d: np.ndarray) -> np.ndarray:
    """x moved by d steps of the IEEE totalOrder key (saturating at both
    ends of the key range), computed on the bits."""
    u = U[x.dtype]
    nb = 8 * x.itemsize
    sign = u(1) << u(nb - 1)
    top = np.iinfo(u).max
    bits = x.view(u)
    key = np.where(bits & sign, ~bits, bits | sign).astype(u)
    dd = np.abs(d).astype(u)
    up = np.where(key <= top - dd, key + dd, top)
    down = np.where(key >= dd, key - dd, u(0))
    key2 = np.where(d >= 0, up, down).astype(u)
    out = np.where(key2 & sign, key2 & ~sign, ~key2).astype(u)
    return out.view(x.dtype)


def _specials(dtype):
    f = np.finfo(dtype)
    u = U[np.dtype(dtype)]
    nan_payload = np.array([(u(0x7fc00123) if dtype == np.float32 else u(0x7ff8000000000123))], dtype=u).view(dtype)[0]
    return np.array([0.0, -0.0, f.smallest_subnormal, -f.smallest_subnormal, f.smallest_normal - f.smallest_subnormal,
                     f.smallest_normal, -f.smallest_normal, 1.0, -1.0, f.max, -f.max, np.inf, -np.inf, np.nan,
                     -np.nan, nan_payload], dtype=dtype)


def boundary_set(rng, dtype, k, n, m, delta, anchored=False):
    """k replicas of n elements on the edges of a ULP tolerance m and of a
    relative tolerance delta (see the module docstring).  Anchored: for each
    element a random k//2 + 1 of the replicas hold the base value itself and
    there are no tie splits, so every element has a strict majority and only
    the other replicas sit on the edges."""
    dtype = np.dtype(dtype)
    sp = _specials(dtype)
    # 0, 1: ULP edges, 2: relative edges, 3: tie split (in every other set)
    kind = rng.integers(0, 4 if rng.random() < 0.5 and not anchored else 3, n)
    base = (rng.standard_normal(n) * 10.0 ** rng.integers(-20, 21, n)).astype(dtype)
    at_special = rng.random(n) < 0.35
    base[at_special] = sp[rng.integers(0, sp.size, int(at_special.sum()))]
    offs = np.array([0, 1, -1, m - 1, -(m - 1), m, -m, m + 1, -(m + 1), 2 * m + 1, -(2 * m + 1)], dtype=np.int64)
    reps = []
    # relative edges: base * (1 + s * delta * f), f just below 1, 1, just above 1, in fp64 then rounded
    fr = np.array([0.0, 0.5, 1.0 - 2.0 ** -30, 1.0, 1.0 + 2.0 ** -30, 2.0])
    b64 = base.astype(np.float64)
    other = _step_keys(base, np.full(n, m + 1 + int(rng.integers(0, 3)), dtype=np.int64))
    split = rng.random(n) < 0.5
    rank = np.argsort(np.argsort(rng.random((k, n)), axis=0), axis=0)   # per element, a random order of replicas
    for r in range(k):
        d = offs[rng.integers(0, offs.size, n)]
        x = _step_keys(base, d)
        s = np.where(rng.random(n) < 0.5, -1.0, 1.0)
        with np.errstate(over="ignore", invalid="ignore"):
            rel = (b64 * (1.0 + s * delta * fr[rng.integers(0, fr.size, n)])).astype(dtype)
        x = np.where(kind == 2, rel, x)
        # tie split: the first half of the replicas hold base, the rest `other`
        # (or the halves swapped), so no value has a strict majority for even k
        first = r < k // 2
        x = np.where(kind == 3, np.where(first ^ split, base, other), x)
        if anchored:
            x = np.where(rank[r] <= k // 2, base, x)
        reps.append(np.ascontiguousarray(x.astype(dtype)))
    return reps


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
