"""Outputs that share memory with a replica or with each other are rejected
before anything is launched (the general vote of an element may read its
replicas again after outputs of the same launch are stored, and the block
restore copies whole blocks while every replica's blocks are still read);
replicas may overlap each other."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu):
    c = gpu.Context(0)
    yield c
    c.close()


def test_overlaps_rejected(gpu, ctx):
    import torch
    n = 4096
    buf = torch.zeros(3 * n + 8, dtype=torch.float32, device="cuda")
    a, b, c = buf[:n], buf[n:2 * n], buf[2 * n:3 * n]
    spare = torch.zeros(n + 4, dtype=torch.float32, device="cuda")
    cases = {
        "consensus is replica 0": dict(consensus=a),
        "consensus is replica 1": dict(consensus=b),
        "consensus shifted into replica 0": dict(consensus=buf[1:n + 1]),
        "consensus runs into replica 2": dict(consensus=buf[2 * n - 4:3 * n - 4]),
        "mask inside replica 1": dict(consensus=spare[:n], mask=b.view(torch.uint8)[:n]),
        "stats inside replica 2": dict(consensus=spare[:n], stats=c.view(torch.uint8)[:1024]),
        "mask inside the consensus": dict(consensus=spare[:n], mask=spare.view(torch.uint8)[:n]),
    }
    for where, kw in cases.items():
        print("case:", where, flush=True)
        with pytest.raises(gpu.FtvError) as e:
            gpu.vote(ctx, [a, b, c], gpu.ulp(1), **kw)
        assert e.value.code == gpu.E_INVALID, where
    print("case: batched task writing a replica", flush=True)
    stats = gpu.stats_tensor(torch.device("cuda:0"), 2)
    good = gpu.make_desc([a, b, c], gpu.ulp(1), spare[:n], None, stats)
    bad = gpu.make_desc([a, b, c], gpu.ulp(1), c, None, None)
    bad.stats = stats.data_ptr() + ctypes.sizeof(gpu.Stats)
    with pytest.raises(gpu.FtvError) as e:
        gpu.vote_batch(ctx, [good, bad])
    assert e.value.code == gpu.E_INVALID
    print("case: block vote restoring over replica 0", flush=True)
    with pytest.raises(gpu.FtvError) as e:
        gpu.vote_blocks(ctx, [a, b, c], gpu.ulp(1), 4096, consensus=a)
    assert e.value.code == gpu.E_INVALID
    with pytest.raises(gpu.FtvError) as e:
        gpu.vote_blocks(ctx, [a, b, c], gpu.ulp(1), 4096, consensus=spare[:n],
                        blockmap=b.view(torch.uint8)[:8])
    assert e.value.code == gpu.E_INVALID
    # nothing was written by the rejected calls
    assert not buf.any().item() and not spare.any().item()
    print("case: replicas overlapping each other", flush=True)
    buf[:] = torch.arange(buf.numel(), dtype=torch.float32, device="cuda")
    cons, mask, st = gpu.vote(ctx, [a, a, buf[1:n + 1]], gpu.ulp(0), consensus=spare[:n])
    torch.cuda.synchronize()
    s = gpu.read_stats(st)
    assert s["verdict"] == gpu.TASK_MAJORITY and s["disagree"][2] == n
    assert np.array_equal(cons[:n].cpu().numpy(), a.cpu().numpy())
