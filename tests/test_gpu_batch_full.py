"""GPU: the uneven-batch workload at its full size (4096 tasks of 1 KiB to
64 MiB per replica, fp32/fp64/i32, k in {2,3,5}, 1% faulty tasks), voted in one
persistent launch under two different schedules: both must give identical
bytes for every consensus, mask and stats record, and a sample of tasks is
checked element by element against the oracle."""
import os
import sys

import numpy as np
import pytest

import oracle

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
    st_host = st_a.cpu()
    order = np.argsort([t["n"] for t in tasks])
    rng = np.random.default_rng(3)
    faulty = [i for i in range(len(tasks)) if gpu.read_stats(st_host, i)["verdict"] != gpu.UNANIMOUS]
    sample = sorted(set(order[:16].tolist()) | set(rng.choice(len(tasks), 16, replace=False).tolist()) |
                    set(faulty[:8]))
    checked = 0
    for i in sample:
        t = tasks[int(i)]
        if t["n"] > (1 << 22):
            continue
        host = [r.cpu().numpy() for r in t["reps"]]
        otol = oracle.exact() if t["dt"] == "i32" else oracle.ulp(t["tol"].max_ulp)
        ref = oracle.vote(host, otol)
        d = descs_a[int(i)]
        es = host[0].itemsize
        co = d.consensus - cons_a.data_ptr()
        mo = d.mask - mask_a.data_ptr()
        got_c = cons_a[co:co + t["n"] * es].cpu().numpy()
        got_m = mask_a[mo:mo + t["n"]].cpu().numpy()
        assert np.array_equal(got_c, ref.consensus.view(np.uint8)), i
        assert np.array_equal(got_m, ref.mask), i
        s = gpu.read_stats(st_host, int(i))
        k = t["k"]
        assert np.array_equal(s["pair"][:k, :k], ref.pair), i
        assert np.array_equal(s["disagree"][:k], ref.disagree), i
        assert (s["no_majority"], s["verdict"], s["winner"]) == (ref.no_majority, ref.verdict, ref.winner), i
        checked += 1
    assert checked >= 24 and len(faulty) >= 1
    del cons_a, mask_a, cons_b, mask_b, tasks
    ctx.close()
    torch.cuda.empty_cache()
