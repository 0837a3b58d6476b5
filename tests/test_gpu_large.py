"""GPU: element counts past 2^31 and 2^32, so that every kernel's 64-bit
indexing is exercised: one k = 3 int32 task of 2^32 + 2^20 + 3 elements per
replica (16 GiB each, a ragged vector tail), through ftv_vote, as a task of a
batch, and through the block path.  The replicas are identical apart from
faults planted at the index boundaries, so the whole result is known outside
small windows around them: there the consensus equals replica 0 and the masks
and block map are zero; inside, the oracle recomputes every element.  The
stats of the whole task equal the oracle's over the windows laid end to end,
since every element outside them is unanimous and adds nothing to a count."""
import ctypes

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

N = (1 << 32) + (1 << 20) + 3
P1 = [(1 << 31) - 1, 1 << 31, (1 << 32) - 1, 1 << 32, N - 1]      # replica 1 differs
P2 = [0, (1 << 31) + 5, (1 << 32) + 1, N - 2]                      # replica 2 differs
PB = [(1 << 32) + 16391]                                           # all three differ
W = 256
PER = 65536 // 4                                                    # int32 per 64 KiB block


@pytest.fixture(scope="module")
def ctx(gpu):
    c = gpu.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def big(gpu):
    import torch
    import synth
    import synth.device as sd
    print(f"case: generating 3 int32 replicas of {N} elements", flush=True)
    reps = [torch.empty(N, dtype=torch.int32, device="cuda") for _ in range(3)]
    for r in reps:
        sd.fill(r, "i32", synth.INTFULL, 14052912 + 32, 0)
    for p in P1:
        reps[1][p:p + 1].bitwise_xor_(1 << (p % 31))
    for p in P2:
        reps[2][p:p + 1].bitwise_xor_(1 << ((p + 7) % 31))
    for p in PB:
        reps[1][p:p + 1].bitwise_xor_(1 << 3)
        reps[2][p:p + 1].bitwise_xor_(1 << 5)
    torch.cuda.synchronize()
    yield reps
    del reps
    torch.cuda.empty_cache()


def _windows():
    iv = sorted((max(0, p - W), min(N, p + W + 1)) for p in P1 + P2 + PB)
    out = []
    for a, b in iv:
        if out and a <= out[-1][1]:
            out[-1] = (out[-1][0], max(out[-1][1], b))
        else:
            out.append((a, b))
    return out


def _nonzero(t):
    """Positions of the non-zero elements, found in chunks (torch's own nonzero
    is limited to fewer than 2^32 elements)."""
    step = 1 << 30
    return np.concatenate([t[o:o + step].nonzero().flatten().cpu().numpy() + o
                           for o in range(0, t.numel(), step)] + [np.zeros(0, np.int64)])


def _inside(pos, spans):
    return all(any(a <= int(p) < b for a, b in spans) for p in pos)


def _check_whole(gpu, reps, cons, mask, s, tol=None):
    import torch
    tol = tol or oracle.exact()
    wins = _windows()
    host = [[r[a:b].cpu().numpy() for r in reps] for a, b in wins]
    off = _nonzero(cons.view(torch.int32) != reps[0].view(torch.int32))  # bit patterns
    assert _inside(off, wins)
    assert _inside(_nonzero(mask), wins)
    for (a, b), h in zip(wins, host):
        ref = oracle.vote(h, tol)
        assert np.array_equal(cons[a:b].cpu().numpy().view(np.uint32), ref.consensus.view(np.uint32)), (a, b)
        assert np.array_equal(mask[a:b].cpu().numpy(), ref.mask), (a, b)
    ref = oracle.vote([np.concatenate([h[r] for h in host]) for r in range(3)], tol)
    assert s["n"] == N
    assert np.array_equal(s["pair"][:3, :3], ref.pair)
    assert np.array_equal(s["disagree"][:3], ref.disagree)
    assert (s["no_majority"], s["verdict"], s["winner"]) == (ref.no_majority, ref.verdict, ref.winner)
    if tol.kind == oracle.exact().kind:
        assert s["no_majority"] == len(PB) and s["verdict"] == gpu.UNRESOLVED
    torch.cuda.empty_cache()


def test_vote_past_2_pow_32(gpu, ctx, big):
    import torch
    print("case: ftv_vote, 2^32 + 2^20 + 3 int32", flush=True)
    cons, mask, st = gpu.vote(ctx, big, gpu.exact())
    torch.cuda.synchronize()
    _check_whole(gpu, big, cons, mask, gpu.read_stats(st))


def test_vote_fp32_ulp_past_2_pow_32(gpu, ctx, big):
    """The same bits as fp32 under a 4-ULP tolerance: the launch shape with
    branch-free full steps (NaN bit patterns included)."""
    import torch
    print("case: ftv_vote fp32 ULP 4, 2^32 + 2^20 + 3 elements", flush=True)
    f = [r.view(torch.float32) for r in big]
    cons, mask, st = gpu.vote(ctx, f, gpu.ulp(4))
    torch.cuda.synchronize()
    _check_whole(gpu, f, cons, mask, gpu.read_stats(st), oracle.ulp(4))


def test_batch_task_past_2_pow_32(gpu, ctx, big):
    import torch
    print("case: ftv_vote_batch, the large task among small ones", flush=True)
    cons = torch.empty_like(big[0])
    mask = torch.empty(N, dtype=torch.uint8, device="cuda")
    stats = gpu.stats_tensor(torch.device("cuda:0"), 4)
    small = [torch.arange(n, dtype=torch.int32, device="cuda") for n in (0, 5, 4099)]
    outs = [(torch.empty(max(n, 1), dtype=torch.int32, device="cuda"),
             torch.empty(max(n, 1), dtype=torch.uint8, device="cuda")) for n in (0, 5, 4099)]
    descs = [gpu.make_desc(big, gpu.exact(), cons, mask, None, n=N)]
    for t, (c, m) in zip(small, outs):
        descs.append(gpu.make_desc([t, t, t], gpu.exact(), c, m, None, n=t.numel()))
    for i, d in enumerate(descs):
        d.stats = stats.data_ptr() + i * ctypes.sizeof(gpu.Stats)
    gpu.vote_batch(ctx, descs)
    torch.cuda.synchronize()
    _check_whole(gpu, big, cons, mask, gpu.read_stats(stats, 0))
    for i, (t, (c, m)) in enumerate(zip(small, outs)):
        n = t.numel()
        assert torch.equal(c[:n], t) and not m[:n].any().item()
        assert gpu.read_stats(stats, i + 1)["verdict"] == gpu.UNANIMOUS


def test_block_vote_past_2_pow_32(gpu, ctx, big):
    import torch
    print("case: ftv_vote_blocks, 64 KiB blocks over 16 GiB replicas", flush=True)
    out = gpu.vote_blocks(ctx, big, gpu.exact(), 65536)
    torch.cuda.synchronize()
    nblocks = (N * 4 + 65535) // 65536
    hit = sorted({p // PER for p in P1 + P2 + PB})
    spans = [(b * PER, min(N, (b + 1) * PER)) for b in hit]
    host = [[r[a:b].cpu().numpy() for r in big] for a, b in spans]
    # the affected blocks laid end to end; the partial last block stays last
    ref = oracle.vote_blocks([np.concatenate([h[r] for h in host]) for r in range(3)], oracle.exact(), 65536)
    s = gpu.read_block_stats(out["bstats"])
    assert s["blocks"] == nblocks
    assert (s["disagree_blocks"], s["fallback_blocks"], s["unresolved_elems"]) == \
        (ref.disagree_blocks, ref.fallback_blocks, ref.unresolved_elems)
    assert np.array_equal(s["replica_blocks"][:3], ref.replica_blocks)
    assert (s["verdict"], s["winner"]) == (ref.verdict, ref.winner)
    both = {p // PER for p in P1 + PB} & {p // PER for p in P2 + PB}
    assert s["fallback_blocks"] == len(both) and s["unresolved_elems"] == len(PB)
    bm = out["blockmap"]
    assert _nonzero(bm).tolist() == hit
    assert np.array_equal(bm[hit].cpu().numpy(), ref.blockmap)
    cons, mask = out["consensus"], out["mask"]
    assert _inside(_nonzero(cons != big[0]), spans)
    assert _inside(_nonzero(mask), spans)
    o = 0
    for (a, b) in spans:
        assert np.array_equal(cons[a:b].cpu().numpy(), ref.consensus[o:o + b - a]), (a, b)
        assert np.array_equal(mask[a:b].cpu().numpy(), ref.mask[o:o + b - a]), (a, b)
        o += b - a
    fps = out["fps"].view(3, nblocks)
    for j, b in enumerate(hit):
        assert np.array_equal(fps[:, b].contiguous().cpu().numpy().view(np.uint64), ref.fps[:, j]), b
    for b in (0, 131071, 131072, 262143, 262144, nblocks - 1):
        a = b * PER
        want = [oracle.fingerprint(r[a:min(N, a + PER)].cpu().numpy())[0] for r in big]
        assert fps[:, b].contiguous().cpu().numpy().view(np.uint64).tolist() == want, b
    del out, cons, mask
    torch.cuda.empty_cache()
