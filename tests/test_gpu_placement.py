"""Placement of the voter across host and device (ftv_vote_placed) and the
redundant voter, through the C ABI.

Every unit -- one host thread, all host cores, the MI355X voter -- must return
the oracle's result bit for bit wherever the replicas and outputs lie; the
database must try each unit once per key, then run the unit of lowest
fault-aware runtime; in redundant mode a planted voter fault must be outvoted
by the two other units and counted against its unit, and a unit whose runs
all failed must be re-tried at its check interval and regain a finite F.
"""
import math

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


def _host(t):
    return t.cpu().numpy() if t.is_cuda else t.numpy()


def _check(ftv, out, ref, k, where):
    cons, mask, st, _ = out
    u = np.uint32 if ref.consensus.dtype.itemsize == 4 else np.uint64
    assert np.array_equal(_host(cons).view(u), ref.consensus.view(u)), where
    assert np.array_equal(_host(mask), ref.mask), where
    s = ftv.read_stats(st)
    assert np.array_equal(s["pair"][:k, :k], ref.pair), where
    assert np.array_equal(s["disagree"][:k], ref.disagree), where
    assert s["no_majority"] == ref.no_majority and s["n"] == ref.mask.size, where
    assert (s["verdict"], s["winner"]) == (ref.verdict, ref.winner), where


def _tensors(reps, where_dev):
    import torch
    return [torch.from_numpy(r).to("cuda:0") if d else torch.from_numpy(r.copy()) for r, d in zip(reps, where_dev)]


@pytest.mark.parametrize("place", ["device", "host", "mixed"])
@pytest.mark.parametrize("out_mem", ["device", "host"])
def test_every_unit_matches_the_oracle(gpu, ctx, place, out_mem):
    """The first three calls of a key run the three units in turn; each result
    equals the oracle's, for fp32 / fp64 / int32 tasks with ragged sizes."""
    import torch
    for dtype, per, nomaj in (("f32", [40, 10, 30], 0), ("f64", [40, 10, 30, 10, 50], 3), ("i32", [5, 9, 2], 0)):
        _, reps = synth.planted_set(dtype, 70001, per, nomaj)
        k = len(reps)
        wd = {"device": [True] * k, "host": [False] * k, "mixed": [r % 2 == 0 for r in range(k)]}[place]
        ts = _tensors(reps, wd)
        tol_o, tol_f = (oracle.exact(), gpu.exact()) if dtype == "i32" else (oracle.ulp(4), gpu.ulp(4))
        ref = oracle.vote(reps, tol_o)
        db = gpu.VoterDB(check_interval=0, host_threads=4)
        om = gpu.MEM_DEVICE if out_mem == "device" else gpu.MEM_HOST
        seen = []
        for call in range(4):
            print(f"case: placed {dtype} k={k} replicas={place} outputs={out_mem} call {call}", flush=True)
            out = gpu.vote_placed(ctx, db, ts, tol_f, out_memory=om)
            torch.cuda.synchronize()
            _check(gpu, out, ref, k, f"{dtype} {place} {out_mem} call {call}")
            seen.append(out[3]["result_unit"])
        assert seen[:3] == [gpu.VOTER_HOST1, gpu.VOTER_HOSTMT, gpu.VOTER_GPU]
        nbytes = 70001 * reps[0].itemsize * k
        mask_bits = sum(1 << r for r in range(k) if not wd[r])
        prof = [db.profile(u, nbytes, mask_bits, om) for u in range(3)]
        assert all(p.total >= 1 and p.valid == p.total and p.runtime > 0 for p in prof)
        assert prof[seen[3]].valid == 2 and sum(p.total for p in prof) == 4
        db.close()


def test_avoid_keeps_the_vote_off_a_unit(gpu, ctx):
    import torch
    _, reps = synth.planted_set("f32", 20000, [3, 1, 2], 0)
    ts = _tensors(reps, [True] * 3)
    ref = oracle.vote(reps, oracle.ulp(4))
    db = gpu.VoterDB(check_interval=0, host_threads=2)
    for call in range(5):
        out = gpu.vote_placed(ctx, db, ts, gpu.ulp(4), avoid=1 << gpu.VOTER_GPU)
        torch.cuda.synchronize()
        _check(gpu, out, ref, 3, f"avoid call {call}")
        assert out[3]["result_unit"] != gpu.VOTER_GPU
    db.close()


def test_redundant_voters_agree_and_outvote_a_planted_fault(gpu, ctx):
    """Redundant mode: two voters on different devices agree; with a fault
    planted in one unit's result, a third voter settles the vote, the returned
    result is the oracle's, and the faulty unit's run counts as not valid."""
    import torch
    _, reps = synth.planted_set("f32", 50021, [40, 10, 30], 2)
    ts = _tensors(reps, [True, False, True])
    ref = oracle.vote(reps, oracle.ulp(4))
    for out_mem in (gpu.MEM_DEVICE, gpu.MEM_HOST):
        db = gpu.VoterDB(check_interval=0, host_threads=4)
        # learn all three units first
        for _ in range(3):
            gpu.vote_placed(ctx, db, ts, gpu.ulp(4), out_memory=out_mem)
        out = gpu.vote_placed(ctx, db, ts, gpu.ulp(4), out_memory=out_mem, redundant=True)
        torch.cuda.synchronize()
        rep = out[3]
        print(f"case: redundant agree out={out_mem} units={rep['units']}", flush=True)
        assert rep["agreed"] and len(rep["units"]) == 2
        assert (rep["units"][0] == gpu.VOTER_GPU) != (rep["units"][1] == gpu.VOTER_GPU)
        _check(gpu, out, ref, 3, "redundant agree")
        for victim in range(3):
            db.inject(victim, 1)
            out = gpu.vote_placed(ctx, db, ts, gpu.ulp(4), out_memory=out_mem, redundant=True)
            torch.cuda.synchronize()
            rep = out[3]
            print(f"case: redundant planted fault in unit {victim}: {rep}", flush=True)
            _check(gpu, out, ref, 3, f"planted fault in unit {victim}")
            if victim in rep["units"][:2]:
                assert not rep["agreed"] and len(rep["units"]) == 3
                assert rep["result_unit"] != victim
                p = db.profile(victim, reps[0].nbytes * 3, 0b010, out_mem)
                assert p.valid < p.total
            db.inject(victim, 0)
        db.close()


def test_failed_unit_is_probed_at_its_check_interval_and_recovers(gpu, ctx):
    """A unit whose every run for a key failed has F = +infinity and is passed
    over; after check_interval - 1 decisions it votes again as an extra run
    checked against the result, and a good run gives it a finite F again."""
    import torch
    _, reps = synth.planted_set("f64", 30011, [4, 1, 3], 0)
    ts = _tensors(reps, [True] * 3)
    ref = oracle.vote(reps, oracle.ulp(2))
    db = gpu.VoterDB(check_interval=3, host_threads=2)
    nbytes = reps[0].nbytes * 3
    # first contact of each unit; the GPU unit's result is corrupted in redundant mode
    db.inject(gpu.VOTER_GPU, 1)
    out = gpu.vote_placed(ctx, db, ts, gpu.ulp(2), redundant=True)
    torch.cuda.synchronize()
    _check(gpu, out, ref, 3, "first redundant call")
    assert out[3]["units"] == [gpu.VOTER_HOST1, gpu.VOTER_GPU, gpu.VOTER_HOSTMT]
    g = db.profile(gpu.VOTER_GPU, nbytes, 0, gpu.MEM_DEVICE)
    assert (g.valid, g.total) == (0, 1)   # F = +infinity
    probed_at = None
    for call in range(1, 6):
        out = gpu.vote_placed(ctx, db, ts, gpu.ulp(2))
        torch.cuda.synchronize()
        _check(gpu, out, ref, 3, f"call {call}")
        rep = out[3]
        print(f"case: check interval call {call}: {rep}", flush=True)
        assert rep["result_unit"] != gpu.VOTER_GPU
        if rep["probed"]:
            probed_at = call
            assert rep["units"][-1] == gpu.VOTER_GPU
            break
    assert probed_at == 3
    g = db.profile(gpu.VOTER_GPU, nbytes, 0, gpu.MEM_DEVICE)
    assert (g.valid, g.total) == (1, 2) and math.isfinite(gpu.fault_aware_runtime(g))
    db.close()


def test_host_voter_equals_gpu_voter_on_the_large_recipe(gpu, ctx):
    """The k=3 fp32 single-task recipe at 2^24 elements: the host voter on
    every core and the MI355X voter give identical bytes."""
    import torch
    import synth.device as sd
    n = 1 << 24
    print("case: host voter vs GPU voter, 2^24 fp32", flush=True)
    reps_d = sd.large_task_set(n, "f32")
    cons, mask, st = gpu.vote(ctx, reps_d, gpu.ulp(4))
    torch.cuda.synchronize()
    reps_h = [r.cpu().numpy() for r in reps_d]
    hc, hm, hs = gpu.vote_host(reps_h, gpu.ulp(4), threads=0)
    assert np.array_equal(hc.view(np.uint32), cons.cpu().numpy().view(np.uint32))
    assert np.array_equal(hm, mask.cpu().numpy())
    s = gpu.read_stats(st)
    for key in ("pair", "disagree"):
        assert np.array_equal(hs[key], s[key])
    assert (hs["no_majority"], hs["verdict"], hs["winner"], hs["n"]) == \
        (s["no_majority"], s["verdict"], s["winner"], s["n"])


def test_placed_errors(gpu, ctx):
    import torch
    _, reps = synth.planted_set("f32", 1000, [3, 1, 2], 0)
    ts = _tensors(reps, [True] * 3)
    db = gpu.VoterDB()
    with pytest.raises(gpu.FtvError) as e:
        gpu.vote_placed(ctx, db, ts, gpu.ulp(4), out_memory=5)
    assert e.value.code == gpu.E_INVALID
    with pytest.raises(gpu.FtvError) as e:
        gpu.vote_placed(ctx, db, ts, gpu.ulp(4), avoid=1 << 5)
    assert e.value.code == gpu.E_INVALID
    with pytest.raises(ValueError):
        gpu.vote_placed(ctx, db, ts, gpu.ulp(4), out_memory=gpu.MEM_HOST,
                        consensus=torch.empty(1000, dtype=torch.float32, device="cuda:0"))
    db.close()
