"""GPU parity of ftv_vote_batch_noalloc, the batched vote without a context or
any allocation: on two calls in a row (the second with fewer and smaller
tasks, so counts the first call left in the static workspace would show), its
consensus, mask and stats are bit-identical to ftv_vote_batch's on the same
tasks and to the oracle.  Sizes beyond its limit are rejected before any work
is enqueued."""

import numpy as np
import pytest

from test_gpu_batch import check_oracle, make_batch, outputs, same

pytestmark = pytest.mark.gpu


def _clear(tasks, stats):
    stats.fill_(0x5A)
    for t in tasks:
        t["cons"].zero_()
        t["mask"].fill_(0xEE)


def test_noalloc_batch_matches_batched_vote_twice(gpu):
    import torch
    ctx = gpu.Context(0)
    try:
        rng = np.random.default_rng(4097)
        for ntasks, max_elems in ((160, 300000), (23, 20000)):
            print(f"case: no-alloc batch of {ntasks} tasks, up to {max_elems} elements", flush=True)
            tasks, descs, stats = make_batch(gpu, rng, ntasks, max_elems)
            gpu.vote_batch(ctx, descs)
            ref = outputs(gpu, tasks, stats)
            check_oracle(tasks, ref)
            _clear(tasks, stats)
            gpu.vote_batch_noalloc(descs)
            got = outputs(gpu, tasks, stats)
            assert same(got, ref), ntasks
            assert sum(1 for (_, _, s) in got if s["verdict"] != gpu.UNANIMOUS) > 0
        # a planted task on a side stream: ordered by that stream alone
        side = torch.cuda.Stream()
        tasks, descs, stats = make_batch(gpu, rng, 7, 5000)
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            gpu.vote_batch_noalloc(descs, stream=side)
        side.synchronize()
        check_oracle(tasks, outputs(gpu, tasks, stats))
    finally:
        ctx.close()


def test_noalloc_rejects_oversize_and_empty(gpu):
    lib = gpu.load()
    arr = (gpu.VoteDesc * 1)()
    rc = lib.ftv_vote_batch_noalloc(arr, gpu.NOALLOC_MAX_TASKS + 1, None)
    assert rc == gpu.E_INVALID
    assert b"at most 4096 tasks" in lib.ftv_last_error()
    assert lib.ftv_vote_batch_noalloc(arr, 0, None) == gpu.OK
    # an invalid descriptor is reported with its index, nothing enqueued
    assert lib.ftv_vote_batch_noalloc(arr, 1, None) == gpu.E_K
    assert lib.ftv_last_error().startswith(b"task 0")
