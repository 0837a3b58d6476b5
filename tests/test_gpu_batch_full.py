"""GPU: the uneven-batch workload at its full size (4096 tasks of 1 KiB to
64 MiB per replica, fp32/fp64/i32, k in {2,3,5}, 1% faulty tasks), voted in one
persistent launch under two different schedules: both must give identical
bytes for every consensus, mask and stats record, and every task given faults,
the three largest, the smallest and some random tasks are checked whole,
element by element, against the oracle."""
import os
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_full_uneven_batch(gpu):
    import torch
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import bench
    ctx = gpu.Context(0)
    print("case: full uneven batch, 4096 tasks", flush=True)
    tasks, _, out_sizes = bench.make_uneven_tasks(gpu, 4096, 14052912 + 3)
    cons_a, mask_a, st_a, descs_a = bench.output_set(gpu, tasks, out_sizes)
    cons_b, mask_b, st_b, descs_b = bench.output_set(gpu, tasks, out_sizes)
    ctx.set_batch_config(gpu.BatchCfg(131072, 512, 2, 1, 1, 0))
    gpu.vote_batch(ctx, descs_a)
    ctx.set_batch_config(gpu.BatchCfg(2048, 256, 4, 2, 0, 0))
    gpu.vote_batch(ctx, descs_b)
    torch.cuda.synchronize()
    assert torch.equal(cons_a, cons_b) and torch.equal(mask_a, mask_b) and torch.equal(st_a, st_b)
    # whole tasks against the oracle: every task given faults, the three
    # largest (64 MiB per replica and near it), the 16 smallest and 16 random
    sample = bench.batch_sample(tasks, n_small=16, n_large=3, n_faulty=len(tasks), n_random=16, seed=3)
    nfaulty = sum(1 for t in tasks if t["faulty"])
    print(f"case: oracle check of {len(sample)} tasks ({nfaulty} faulty, largest "
          f"{max(t['n'] for t in tasks)} elements)", flush=True)
    for i in sample:
        assert bench.check_batch_task(gpu, tasks, descs_a, cons_a, mask_a, st_a, i), i
    assert nfaulty >= 40 and all(i in sample for i, t in enumerate(tasks) if t["faulty"])
    assert max(tasks[i]["n"] for i in sample) == max(t["n"] for t in tasks)
    del cons_a, mask_a, cons_b, mask_b, tasks
    ctx.close()
    torch.cuda.empty_cache()
