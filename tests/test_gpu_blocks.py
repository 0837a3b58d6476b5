"""GPU parity of block fingerprints and the fused block vote with consensus
restore, against the oracle, bit for bit."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu):
    c = gpu.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("bb", [4096, 8192, 16384, 32768, 65536])
def test_fingerprint_parity(gpu, ctx, bb):
    import torch
    rng = np.random.default_rng(bb)
    for nbytes in (1, 7, 8, 63, 64, 100, 4095, 4096, 4097, 65536, 3 * 65536 + 13, (1 << 20) + 24):
        raw = rng.integers(0, 256, nbytes, dtype=np.uint8)
        t = torch.from_numpy(raw).cuda()
        print(f"case: fingerprint nbytes={nbytes} block={bb}", flush=True)
        fp = gpu.fingerprint(ctx, t, bb)
        torch.cuda.synchronize()
        got = fp.cpu().numpy().view(np.uint64)
        assert np.array_equal(got, oracle.fingerprint(raw, bb)), nbytes


def _block_case(gpu, reps, tol_o, tol_f, bb, want_fps=True, want_mask=True):
    import torch
    t = [torch.from_numpy(r).cuda() for r in reps]
    out = gpu.vote_blocks(ctx_holder[0], t, tol_f, bb, want_fps=want_fps, want_mask=want_mask)
    torch.cuda.synchronize()
    ref = oracle.vote_blocks(reps, tol_o, bb)
    k = len(reps)
    u = np.uint32 if reps[0].itemsize == 4 else np.uint64
    if want_fps:
        assert np.array_equal(out["fps"].cpu().numpy().view(np.uint64).reshape(k, -1), ref.fps)
    assert np.array_equal(out["blockmap"].cpu().numpy(), ref.blockmap)
    assert np.array_equal(out["consensus"].cpu().numpy().view(u), ref.consensus.view(u))
    if want_mask:
        assert np.array_equal(out["mask"].cpu().numpy(), ref.mask)
    s = gpu.read_block_stats(out["bstats"])
    assert (s["blocks"], s["disagree_blocks"], s["fallback_blocks"], s["unresolved_elems"]) == \
        (ref.blocks, ref.disagree_blocks, ref.fallback_blocks, ref.unresolved_elems)
    assert np.array_equal(s["replica_blocks"][:k], ref.replica_blocks)
    assert (s["verdict"], s["winner"]) == (ref.verdict, ref.winner)
    return ref


ctx_holder = []


@pytest.fixture(autouse=True)
def _hold(ctx):
    ctx_holder[:] = [ctx]
    yield


def test_checkpoint_recipe_reduced(gpu):
    n = 1 << 19   # 4 MiB per replica, 64 blocks of 64 KiB
    reps = synth.checkpoint_set(n, nstuck=40, nflip=20)
    base = reps[0]
    # forced: a stuck word (r1) and a flip (r2) in the same block -> no majority
    b = 17 * 8192
    reps[1][b + 5] = 0.0
    reps[2].view(np.uint64)[b + 900] ^= np.uint64(1 << 51)
    print("case: checkpoint recipe, 2^19 fp64, k=5", flush=True)
    ref = _block_case(gpu, reps, oracle.exact(), gpu.exact(), 65536)
    assert ref.fallback_blocks >= 1 and np.array_equal(ref.consensus.view(np.uint64), base.view(np.uint64))


@pytest.mark.parametrize("k", [2, 3, 4, 5, 6, 7])
def test_block_vote_k_dtype_matrix(gpu, k):
    rng = np.random.default_rng(k)
    for dtype, tol_o, tol_f, bb in ((np.float64, oracle.ulp(2), gpu.ulp(2), 4096),
                                     (np.float32, oracle.rel(1e-3), gpu.rel(1e-3), 16384),
                                     (np.int32, oracle.exact(), gpu.exact(), 8192)):
        n = (3 * bb + 520) // np.dtype(dtype).itemsize   # ragged last block
        base = synth.values("f64" if dtype == np.float64 else ("f32" if dtype == np.float32 else "i32"),
                            synth.INTFULL if dtype == np.int32 else synth.NORMAL, 3, 0, n)
        reps = [base.copy() for _ in range(k)]
        per = bb // np.dtype(dtype).itemsize
        for r in range(1, k):
            for blk in rng.choice(4, size=2, replace=False):
                i = min(n - 1, int(blk) * per + int(rng.integers(0, per)))
                reps[r].view(np.uint32 if dtype != np.float64 else np.uint64)[i] ^= 1 << int(rng.integers(0, 20))
        print(f"case: block vote k={k} {np.dtype(dtype).name} block={bb}", flush=True)
        _block_case(gpu, reps, tol_o, tol_f, bb)
        _block_case(gpu, reps, tol_o, tol_f, bb, want_fps=False, want_mask=False)


@pytest.mark.parametrize("k", [3, 5])
def test_block_vote_replica0_outlier(gpu, k):
    """Replica 0 is the odd one out in some blocks (whole ones and the ragged
    last one): the consensus of those blocks is re-copied from the source
    replica; one more block has no fingerprint majority at all."""
    for dtype, bb in ((np.float32, 32768), (np.int64, 65536), (np.float64, 4096)):
        isz = np.dtype(dtype).itemsize
        per = bb // isz
        n = 5 * per + 136 // isz                       # five whole blocks + a partial one
        kind = {np.float32: "f32", np.int64: "i64", np.float64: "f64"}[dtype]
        base = synth.values(kind, synth.INTFULL if dtype == np.int64 else synth.NORMAL, 11, k, n)
        reps = [base.copy() for _ in range(k)]
        u = reps[0].view(np.uint32 if isz == 4 else np.uint64)
        for i in (1 * per + 7, 3 * per + per - 1, 5 * per + 2):  # blocks 1, 3 and the partial one
            u[i] ^= 1
        for r in range(1, k):                          # block 4: every replica different
            reps[r].view(np.uint32 if isz == 4 else np.uint64)[4 * per + 3 * r] ^= 4
        tol_o, tol_f = (oracle.exact(), gpu.exact()) if dtype == np.int64 else (oracle.ulp(0), gpu.ulp(0))
        print(f"case: block vote replica-0 outlier k={k} {np.dtype(dtype).name} block={bb}", flush=True)
        ref = _block_case(gpu, reps, tol_o, tol_f, bb)
        assert ref.replica_blocks[0] >= 3 and ref.fallback_blocks >= 1


def test_xcd_block_order_many_runs(gpu, ctx):
    """More whole blocks than two runs of the XCD block order (8 x 64 blocks
    per run) plus a partial run and a ragged last block: every block is
    hashed once, in the fingerprints and in the block vote (replica 0 outvoted
    in blocks of different runs, one block without a fingerprint majority)."""
    import torch
    rng = np.random.default_rng(2024)
    bb = 4096
    nwhole = 2 * 512 + 37
    raw = rng.integers(0, 256, nwhole * bb + 1000, dtype=np.uint8)
    print(f"case: fingerprint of {nwhole} whole blocks + a partial one", flush=True)
    fp = gpu.fingerprint(ctx, torch.from_numpy(raw).cuda(), bb)
    torch.cuda.synchronize()
    assert np.array_equal(fp.cpu().numpy().view(np.uint64), oracle.fingerprint(raw, bb))
    per = bb // 8
    n = nwhole * per + 100
    base = synth.values("f64", synth.NORMAL, 17, 0, n)
    reps = [base.copy() for _ in range(5)]
    for blk in (3, 511, 512, 700, 1030, nwhole):        # replica 0 outvoted (the last: the partial block)
        reps[0].view(np.uint64)[min(n - 1, blk * per + 5)] ^= 2
    for r in range(1, 5):                               # block 600: no fingerprint majority
        reps[r].view(np.uint64)[600 * per + r] ^= 1
    for r, blk in ((2, 100), (3, 513), (4, 1060)):
        reps[r].view(np.uint64)[blk * per + 11] ^= 8
    print(f"case: block vote k=5 fp64 over {nwhole} whole blocks + a partial one", flush=True)
    ref = _block_case(gpu, reps, oracle.ulp(0), gpu.ulp(0), bb)
    assert ref.replica_blocks[0] == 6 and ref.fallback_blocks == 1


def test_block_vote_empty_and_tiny(gpu):
    for n in (0, 1, 5):
        reps = [np.arange(n, dtype=np.float64) for _ in range(3)]
        if n:
            reps[1][0] = 9.0
        print(f"case: block vote n={n}", flush=True)
        _block_case(gpu, reps, oracle.exact(), gpu.exact(), 4096)


def test_checkpoint_full_size(gpu):
    """k=5 fp64 16384x16384 checkpoint: every fault-carrying block plus a random
    sample of blocks checked against the oracle, and the block-level counts
    against the fault plan."""
    import torch
    import synth.device as sd
    n = 16384 * 16384
    bb = 65536
    per = bb // 8
    print("case: checkpoint full size", flush=True)
    reps = sd.checkpoint_set(n)
    fb = 4321
    reps[1][fb * per + 3] = 0.0                       # forced no-majority block
    iv = reps[2].view(torch.int64)
    iv[fb * per + 777] ^= (1 << 33)
    out = gpu.vote_blocks(ctx_holder[0], reps, gpu.exact(), bb)
    torch.cuda.synchronize()
    s = gpu.read_block_stats(out["bstats"])
    nblocks = n // per
    diff = [(reps[r].view(torch.int64) != reps[0].view(torch.int64)).view(nblocks, per).any(dim=1).cpu().numpy()
            for r in range(5)]
    assert s["blocks"] == nblocks
    assert s["replica_blocks"][0] == 0 and s["replica_blocks"][4] == 0
    assert s["replica_blocks"][1] == diff[1].sum() and s["replica_blocks"][2] == diff[2].sum()
    assert s["replica_blocks"][3] == diff[3].sum() == nblocks
    nofall = diff[1] & diff[2]
    assert s["fallback_blocks"] == nofall.sum() >= 1
    assert s["unresolved_elems"] == 0 and s["verdict"] == gpu.ELEMENT_MAJORITY
    assert s["disagree_blocks"] == nblocks
    cons = out["consensus"]
    assert torch.equal(cons.view(torch.int64), reps[0].view(torch.int64))
    blockmap = out["blockmap"].cpu().numpy()
    fps = out["fps"].cpu().numpy().view(np.uint64).reshape(5, nblocks)
    mask = out["mask"]
    rng = np.random.default_rng(5)
    sample = sorted(set(np.nonzero(diff[1] | diff[2])[0].tolist()) |
                    set(rng.choice(nblocks, 40, replace=False).tolist()) | {0, nblocks - 1, fb})
    for blk in sample:
        sl = slice(blk * per, (blk + 1) * per)
        rb = [r[sl].cpu().numpy() for r in reps]
        ref = oracle.vote_blocks(rb, oracle.exact(), bb)
        assert np.array_equal(fps[:, blk], ref.fps[:, 0]), blk
        assert blockmap[blk] == ref.blockmap[0], blk
        assert np.array_equal(cons[sl].cpu().numpy().view(np.uint64), ref.consensus.view(np.uint64)), blk
        assert np.array_equal(mask[sl].cpu().numpy(), ref.mask), blk


@pytest.mark.parametrize("dtype,bb", [("f64", 65536), ("f32", 4096), ("i32", 16384), ("i64", 8192)])
def test_block_vote_planted_nonzero_argmin_winner(gpu, dtype, bb):
    """Replica blocks with their minimum at replica 1 and every replica
    differing somewhere: ELEMENT_MAJORITY, and UNRESOLVED with a fallback block
    holding an element without majority -- winner a non-zero argmin, identical
    to the oracle (a ragged tail block included)."""
    for per in ([3, 1, 2], [3, 1, 2, 1, 4], [3, 1, 2, 1, 4, 5, 6]):
        for unresolved in (False, True):
            _, reps, ub = synth.planted_blocks(dtype, 40, bb, per, unresolved, tail_elems=37)
            tol_o, tol_f = (oracle.exact(), gpu.exact()) if dtype[0] == "i" else (oracle.ulp(2), gpu.ulp(2))
            print(f"case: planted block winner {dtype} block={bb} k={len(per)} unresolved={unresolved}", flush=True)
            ref = _block_case(gpu, reps, tol_o, tol_f, bb)
            assert ref.winner != 0
            assert ref.verdict == (oracle.UNRESOLVED if unresolved else oracle.ELEMENT_MAJORITY)
