"""The host voter (ftv_vote_host, one thread or OpenMP) against the CPU oracle,
bit for bit: consensus bits, mask bytes, the k x k counts, the disagreement and
no-majority counts, the verdict and the winner.  It runs on the host's cores,
so these tests need no GPU; its agreement with the MI355X voter is checked in
the GPU tests of the placement.
"""
import numpy as np
import pytest

import oracle
import synth

U = {np.dtype(np.float32): np.uint32, np.dtype(np.float64): np.uint64,
     np.dtype(np.int32): np.uint32, np.dtype(np.int64): np.uint64}


@pytest.fixture(scope="module")
def ftv():
    import paper_1405_2912_amd as m
    m.load()
    return m


def _tols(ftv, dtype):
    if np.dtype(dtype).kind == "i":
        return [(oracle.exact(), ftv.exact())]
    return [(oracle.exact(), ftv.exact()), (oracle.ulp(0), ftv.ulp(0)), (oracle.ulp(4), ftv.ulp(4)),
            (oracle.ulp(2 ** 40), ftv.ulp(2 ** 40)), (oracle.rel(1e-3), ftv.rel(1e-3)),
            (oracle.rel(1e-3, 1e-30), ftv.rel(1e-3, 1e-30))]


def _replicas(rng, dtype, k, n):
    """Replicas that differ by bit flips (integers) or by ULP noise, perturbed
    values and special values (floats: zeros of both signs, infinities, NaN,
    denormals), so every branch of the tolerance test and the vote is taken."""
    dtype = np.dtype(dtype)
    if dtype.kind == "i":
        info = np.iinfo(dtype)
        base = rng.integers(info.min, info.max, n, dtype=dtype, endpoint=True)
        reps = []
        for _ in range(k):
            x = base.copy()
            idx = rng.choice(n, n // 10, replace=False) if n else np.zeros(0, int)
            x.view(U[dtype])[idx] ^= (np.ones(idx.size, U[dtype]) <<
                                      rng.integers(0, 8 * dtype.itemsize, idx.size).astype(U[dtype]))
            reps.append(x)
        return reps
    base = rng.standard_normal(n).astype(dtype)
    sp = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 1e-45 if dtype == np.float32 else 5e-324,
                   -1e-40 if dtype == np.float32 else -1e-310], dtype=dtype)
    if n:
        idx = rng.choice(n, min(n, max(1, n // 50)), replace=False)
        base[idx] = sp[rng.integers(0, sp.size, idx.size)]
    reps = []
    for r in range(k):
        x = base.copy()
        synth.ulp_noise(x, 1234, r, round(0.3 * (1 << 24)), 6)
        if n:
            idx = rng.choice(n, max(1, n // 20), replace=False)
            x[idx] = rng.standard_normal(idx.size).astype(dtype) * (1 + 1e-3 * rng.standard_normal(idx.size))
            idx2 = rng.choice(n, max(1, n // 200), replace=False)
            x[idx2] = sp[rng.integers(0, sp.size, idx2.size)]
        reps.append(x)
    return reps


def _check(got, ref, k, where=""):
    cons, mask, s = got
    if cons is not None:
        u = U[ref.consensus.dtype]
        bad = np.nonzero(cons.view(u) != ref.consensus.view(u))[0]
        assert bad.size == 0, f"{where}: consensus differs at {bad[:8]}"
    if mask is not None:
        bad = np.nonzero(mask != ref.mask)[0]
        assert bad.size == 0, f"{where}: mask differs at {bad[:8]}"
    assert np.array_equal(s["pair"][:k, :k], ref.pair), where
    assert not s["pair"][k:, :].any() and not s["pair"][:, k:].any(), where
    assert np.array_equal(s["disagree"][:k], ref.disagree), where
    assert not s["disagree"][k:].any(), where
    assert s["no_majority"] == ref.no_majority, where
    assert s["n"] == ref.mask.size, where
    assert (s["verdict"], s["winner"]) == (ref.verdict, ref.winner), where


@pytest.mark.parametrize("dtype", [np.float32, np.float64, np.int32, np.int64])
def test_host_voter_dtype_tol_k_matrix(ftv, dtype):
    rng = np.random.default_rng(300 + np.dtype(dtype).itemsize)
    n = 4099
    for k in range(2, 8):
        reps = _replicas(rng, dtype, k, n)
        for tol_o, tol_f in _tols(ftv, dtype):
            ref = oracle.vote(reps, tol_o)
            for threads in (1, 3):
                where = f"{np.dtype(dtype).name} k={k} tol={tol_o} threads={threads}"
                _check(ftv.vote_host(reps, tol_f, threads=threads), ref, k, where)


@pytest.mark.parametrize("n", [0, 1, 2, 63, 64, 65, 127, 1000])
def test_host_voter_edge_sizes_more_threads_than_elements(ftv, n):
    rng = np.random.default_rng(n + 7)
    for dtype, k in ((np.float32, 3), (np.float64, 5), (np.int32, 2), (np.int64, 7)):
        reps = _replicas(rng, dtype, k, n)
        tol_o, tol_f = _tols(ftv, dtype)[-1 if np.dtype(dtype).kind == "f" else 0]
        ref = oracle.vote(reps, tol_o)
        for threads in (1, 8, 0):
            _check(ftv.vote_host(reps, tol_f, threads=threads), ref, k, f"n={n} {dtype} threads={threads}")


def test_host_voter_optional_outputs(ftv):
    reps = synth.small_task_set(n=1 << 14)
    ref = oracle.vote(reps, oracle.ulp(4))
    for wc, wm in ((False, True), (True, False), (False, False)):
        cons, mask, s = ftv.vote_host(reps, ftv.ulp(4), threads=2, want_consensus=wc, want_mask=wm)
        assert (cons is None) != wc and (mask is None) != wm
        _check((cons, mask, s), ref, 3, f"outputs {wc} {wm}")


@pytest.mark.parametrize("dtype", ["f32", "f64", "i32", "i64"])
def test_host_voter_planted_nonzero_argmin_winner(ftv, dtype):
    """Every replica faulty somewhere, disagreement minimal at replica 1: the
    ELEMENT_MAJORITY and UNRESOLVED winners are a non-zero argmin."""
    for per in ([40, 10, 30], [40, 10, 30, 10, 50], [40, 10, 30, 10, 50, 60, 70]):
        for nomaj in (0, 3):
            _, reps = synth.planted_set(dtype, 20011, per, nomaj)
            pairs = _tols(ftv, np.dtype(synth._np[dtype]))
            tol_o, tol_f = pairs[0] if dtype[0] == "i" else pairs[2]
            ref = oracle.vote(reps, tol_o)
            assert ref.winner != 0
            for threads in (1, 4):
                _check(ftv.vote_host(reps, tol_f, threads=threads), ref, len(per), f"{dtype} {per} {nomaj}")


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_host_voter_tolerance_edges(ftv, dtype):
    """Elements on the tolerance edges (ULP steps around m across zero,
    denormals, max, inf and the NaN keys; relative distances at the delta;
    ties; a random strict majority per element), one thread and several."""
    from edge_sets import boundary_set
    rng = np.random.default_rng(91 + np.dtype(dtype).itemsize)
    tiny = float(np.finfo(dtype).smallest_normal) * 4
    for k in (2, 3, 4, 5, 7):
        for m, delta, anchored in ((1, 1e-3, False), (1000, 1e-6, False), (4, 1e-3, True)):
            reps = boundary_set(rng, dtype, k, 20011, m, delta, anchored)
            for tol_o, tol_f in ((oracle.ulp(m), ftv.ulp(m)), (oracle.exact(), ftv.exact()),
                                 (oracle.rel(delta), ftv.rel(delta)), (oracle.rel(delta, tiny), ftv.rel(delta, tiny))):
                ref = oracle.vote(reps, tol_o)
                for threads in (1, 3):
                    _check(ftv.vote_host(reps, tol_f, threads=threads), ref, k,
                           f"{np.dtype(dtype).name} k={k} m={m} anchored={anchored} tol={tol_o} threads={threads}")


def test_host_voter_large_many_threads(ftv):
    """The single-large-task recipe at 2^22 elements on every core: counts are
    per thread and summed, so the result equals the sequential oracle's."""
    reps = synth.large_task_set(1 << 22, "f32")
    ref = oracle.vote(reps, oracle.ulp(4))
    assert ref.verdict == oracle.TASK_MAJORITY
    _check(ftv.vote_host(reps, ftv.ulp(4), threads=0), ref, 3, "2^22 all cores")


def test_host_voter_errors(ftv):
    reps = synth.small_task_set(n=64)
    with pytest.raises(ftv.FtvError) as e:   # integers are compared bit-wise only
        ftv.vote_host([r.view(np.int32) for r in reps], ftv.ulp(4))
    assert e.value.code == ftv.E_DTYPE
    with pytest.raises(ftv.FtvError) as e:
        ftv.vote_host(reps, ftv.Tol(7, 0, 0, 0.0, 0.0))
    assert e.value.code == ftv.E_INVALID
    with pytest.raises(ftv.FtvError) as e:
        ftv.vote_host(reps, ftv.rel(-1.0))
    assert e.value.code == ftv.E_INVALID
    with pytest.raises(ftv.FtvError) as e:
        ftv.vote_host(reps[:1], ftv.ulp(4))
    assert e.value.code == ftv.E_K


def test_host_voter_overlaps_rejected(ftv):
    """Outputs share no byte with a replica or with each other (the same rule
    as the device voter's); replicas may overlap each other."""
    n = 1000
    buf = np.zeros(3 * n + 8, dtype=np.float32)
    a, b, c = buf[:n], buf[n:2 * n], buf[2 * n:3 * n]
    spare = np.zeros(n + 4, dtype=np.float32)
    cases = {
        "consensus is replica 0": dict(consensus=a),
        "consensus is replica 1": dict(consensus=b),
        "consensus shifted into replica 0": dict(consensus=buf[1:n + 1]),
        "consensus runs into replica 2": dict(consensus=buf[2 * n - 4:3 * n - 4]),
        "mask inside replica 1": dict(consensus=spare[:n], mask=b.view(np.uint8)[:n]),
        "mask inside the consensus": dict(consensus=spare[:n], mask=spare.view(np.uint8)[:n]),
    }
    for where, kw in cases.items():
        with pytest.raises(ftv.FtvError) as e:
            ftv.vote_host([a, b, c], ftv.ulp(1), **kw)
        assert e.value.code == ftv.E_INVALID, where
    assert not buf.any() and not spare.any()      # nothing was written
    buf[:] = np.arange(buf.size, dtype=np.float32)
    cons, _, s = ftv.vote_host([a, a, buf[1:n + 1]], ftv.ulp(0), consensus=spare[:n])
    assert s["verdict"] == ftv.TASK_MAJORITY and s["disagree"][2] == n
    assert np.array_equal(cons[:n], a)
