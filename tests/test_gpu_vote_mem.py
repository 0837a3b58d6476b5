"""GPU parity of ftv_vote_mem: replicas in host memory (pageable or pinned)
and in device memory, streamed to the device in pieces; every result equals
the oracle's and ftv_vote's on device copies of the same replicas, bit for
bit."""
import numpy as np
import pytest

import oracle
from test_gpu_vote import U, _replicas

pytestmark = pytest.mark.gpu

MIB = 1 << 20


@pytest.fixture(scope="module")
def ctx(gpu):
    c = gpu.Context(0)
    yield c
    c.close()


def _place(reps, where):
    import torch
    out = []
    for r, w in zip(reps, where):
        t = torch.from_numpy(r)
        if w == "dev":
            t = t.cuda()
        elif w == "pin":
            t = t.pin_memory()
        out.append(t)
    return out


def _same(a, b):
    u = U[a.dtype]
    return np.array_equal(a.view(u), b.view(u))


@pytest.mark.parametrize("dtype,k,where,chunk,n", [
    (np.float32, 3, ("dev", "host", "dev"), MIB, 3 * (MIB // 4) + 12345),
    (np.float32, 2, ("host", "dev"), MIB, MIB // 4),
    (np.float64, 5, ("pin", "dev", "dev", "host", "dev"), MIB, 2 * (MIB // 8) + 5),
    (np.int32, 3, ("host", "host", "host"), 2 * MIB, 5 * (MIB // 2) + 1),
    (np.int64, 7, ("dev", "pin", "dev", "dev", "host", "dev", "dev"), MIB, 300001),
])
def test_mixed_memories_match_oracle_and_device_vote(gpu, ctx, dtype, k, where, chunk, n):
    import torch
    rng = np.random.default_rng(900 + k)
    reps = _replicas(rng, dtype, k, n)
    kinds = [(oracle.exact(), gpu.exact())] if np.dtype(dtype).kind == "i" else \
        [(oracle.ulp(4), gpu.ulp(4)), (oracle.rel(1e-3), gpu.rel(1e-3))]
    for tol_o, tol_f in kinds:
        print(f"case: {np.dtype(dtype).name} k={k} {where} chunk={chunk} n={n} tol={tol_o}", flush=True)
        ref = oracle.vote(reps, tol_o)
        cons, mask, st = gpu.vote_mem(ctx, _place(reps, where), tol_f, chunk_bytes=chunk)
        torch.cuda.synchronize()
        s = gpu.read_stats(st)
        assert _same(cons.cpu().numpy(), ref.consensus)
        assert np.array_equal(mask.cpu().numpy(), ref.mask)
        assert np.array_equal(s["pair"][:k, :k], ref.pair)
        assert np.array_equal(s["disagree"][:k], ref.disagree)
        assert (s["no_majority"], s["verdict"], s["winner"], s["n"]) == \
            (ref.no_majority, ref.verdict, ref.winner, n)
        c2, m2, st2 = gpu.vote(ctx, _place(reps, ["dev"] * k), tol_f)
        torch.cuda.synchronize()
        assert torch.equal(cons.view(torch.uint8), c2.view(torch.uint8)) and torch.equal(mask, m2)
        assert torch.equal(st.cpu(), st2.cpu())


def test_reuse_empty_and_errors(gpu, ctx):
    import torch
    rng = np.random.default_rng(77)
    big = _replicas(rng, np.float32, 3, 4 * (MIB // 4) + 3)
    small = _replicas(rng, np.float32, 3, 1000)
    print("case: a large call, a device-only call, then a small one (staging reused)", flush=True)
    for reps in (big, small):
        ref = oracle.vote(reps, oracle.ulp(4))
        cons, mask, st = gpu.vote_mem(ctx, _place(reps, ("host", "dev", "dev")), gpu.ulp(4), chunk_bytes=MIB)
        c2, m2, st2 = gpu.vote(ctx, _place(reps, ("dev", "dev", "dev")), gpu.ulp(4))
        torch.cuda.synchronize()
        assert _same(cons.cpu().numpy(), ref.consensus) and np.array_equal(mask.cpu().numpy(), ref.mask)
        assert gpu.read_stats(st)["verdict"] == ref.verdict
        assert torch.equal(st.cpu(), st2.cpu())
    print("case: n = 0 with a host replica", flush=True)
    e = [torch.zeros(0, dtype=torch.float32), torch.zeros(0, dtype=torch.float32).cuda(),
         torch.zeros(0, dtype=torch.float32).cuda()]
    _, _, st = gpu.vote_mem(ctx, e, gpu.ulp(4))
    torch.cuda.synchronize()
    assert gpu.read_stats(st)["verdict"] == gpu.UNANIMOUS and gpu.read_stats(st)["n"] == 0
    print("case: invalid chunk size", flush=True)
    reps = _place(small, ("host", "dev", "dev"))
    with pytest.raises(RuntimeError):
        gpu.vote_mem(ctx, reps, gpu.ulp(4), chunk_bytes=4096)


def test_pinned_slices_read_in_place(gpu, ctx):
    """Pinned host replicas are read by the vote kernel in place: replicas that
    are slices of one pinned allocation, at element and 16-byte offsets (the
    scalar and the vector path), equal the oracle and the all-device vote."""
    import torch
    rng = np.random.default_rng(77)
    n = 200003
    reps = _replicas(rng, np.float32, 3, n)
    for off in (0, 1, 4):   # elements: 1 leaves the replicas 4-byte aligned only
        pool = torch.empty(3 * (n + 8), dtype=torch.float32).pin_memory()
        ts = []
        for r in range(3):
            base = r * (n + 8) + off
            pool[base:base + n] = torch.from_numpy(reps[r])
            ts.append(pool[base:base + n])
        ts[1] = torch.from_numpy(reps[1]).cuda()     # one replica on the device
        print(f"case: pinned slices of one allocation, offset {off}", flush=True)
        ref = oracle.vote(reps, oracle.ulp(4))
        cons, mask, st = gpu.vote_mem(ctx, ts, gpu.ulp(4), chunk_bytes=MIB)
        torch.cuda.synchronize()
        s = gpu.read_stats(st)
        assert _same(cons.cpu().numpy(), ref.consensus)
        assert np.array_equal(mask.cpu().numpy(), ref.mask)
        assert np.array_equal(s["pair"][:3, :3], ref.pair) and np.array_equal(s["disagree"][:3], ref.disagree)
        assert (s["no_majority"], s["verdict"], s["winner"]) == (ref.no_majority, ref.verdict, ref.winner)
