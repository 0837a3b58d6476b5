"""Redundant execution with light-weight fault tolerance: the model in
oracle/redundancy.py pinned to what the paper fixes (Sec. IV-B, IV-C, IV-D)."""
import math

import numpy as np

import oracle
from oracle.redundancy import ERROR, OK, SLOW, Unit, fault_aware, run_redundant


def _vals(seed, n=257):
    return np.random.default_rng(seed).standard_normal(n).astype(np.float32)


def test_fault_aware_runtime_is_the_papers():
    """Sec. IV-B: F = R / (1 - p), p = 1 - v/t; no history: F = R; v = 0: inf."""
    assert fault_aware(Unit(2.0)) == 2.0
    assert fault_aware(Unit(1.0, 1, 4)) == 4.0            # p = 0.75 -> 4R
    assert fault_aware(Unit(1.0, 0, 3)) == math.inf
    # a unit twice as fast breaks even at p = 50%
    assert fault_aware(Unit(1.0, 1, 2)) == fault_aware(Unit(2.0))


def test_dmr_on_the_two_best_units():
    """Sec. IV-D: the task is duplicated onto the two lowest fault-aware runtimes."""
    good = _vals(1)
    units = [Unit(3.0), Unit(1.0), Unit(2.0, 1, 2)]          # F = 3, 1, 4
    rep = run_redundant([0, 1, 2], units, 2, 3, 0.0, oracle.exact(),
                        lambda a, i: (OK, good, 1.0))
    assert [t.chosen for t in rep.attempts] == [[1, 0]]
    assert rep.verdict == oracle.UNANIMOUS
    assert [(u.valid, u.total) for u in units] == [(1, 1), (1, 1), (1, 2)]
    assert np.array_equal(rep.consensus, good)


def test_direct_fault_restarts_on_the_next_best():
    """Sec. IV-C: a run that reports an API error is abandoned and the task goes
    on with the best-ranked remaining pairing of kernel and unit."""
    good = _vals(2)
    units = [Unit(1.0), Unit(2.0), Unit(3.0)]
    beh = {0: (ERROR, None, 0.0), 1: (OK, good, 2.0), 2: (OK, good, 3.0)}
    rep = run_redundant([0, 1, 2], units, 2, 3, 0.0, oracle.exact(), lambda a, i: beh[i])
    assert [t.chosen for t in rep.attempts] == [[0, 1], [1, 2]]
    assert rep.attempts[0].failed == [0] and rep.attempts[0].verdict is None
    assert rep.errors == 1 and rep.verdict == oracle.UNANIMOUS
    assert (units[0].valid, units[0].total) == (0, 1)
    assert fault_aware(units[0]) == math.inf


def test_timeout_from_the_profile():
    """Sec. IV-C: timeout = profiled runtime x user factor; a unit without a
    profile has no timeout."""
    good = _vals(3)
    units = [Unit(1.0, 4, 4), Unit(2.0), Unit(3.0, 1, 1)]
    beh = {0: (SLOW, good, 9.0), 1: (SLOW, good, 9.0), 2: (OK, good, 3.0)}
    rep = run_redundant([0, 1, 2], units, 2, 3, 2.0, oracle.exact(), lambda a, i: beh[i])
    # unit 0 (profiled) times out; unit 1 (no profile) is slow but kept
    assert [t.chosen for t in rep.attempts] == [[0, 1], [1, 2]]
    assert rep.timeouts == 1 and rep.verdict == oracle.UNANIMOUS
    assert (units[0].valid, units[0].total) == (4, 5)
    # factor 0: no timeout at all
    units = [Unit(1.0, 4, 4), Unit(2.0)]
    rep = run_redundant([0, 1], units, 2, 1, 0.0, oracle.exact(), lambda a, i: (SLOW, good, 9.0))
    assert rep.timeouts == 0 and rep.verdict == oracle.UNANIMOUS


def test_tmr_outvotes_a_corrupted_run_and_profiles_learn_it():
    good = _vals(4)
    bad = good.copy()
    bad[17] = 5.0
    units = [Unit(1.0), Unit(1.5), Unit(2.0)]
    beh = {0: (OK, bad, 1.0), 1: (OK, good, 1.5), 2: (OK, good, 2.0)}
    rep = run_redundant([0, 1, 2], units, 3, 3, 0.0, oracle.exact(), lambda a, i: beh[i])
    assert rep.verdict == oracle.TASK_MAJORITY and rep.winner_unit == 1
    assert [(u.valid, u.total) for u in units] == [(0, 1), (1, 1), (1, 1)]
    assert np.array_equal(rep.consensus, good)
    # the next task ranks the faulty unit last
    rep = run_redundant([0, 1, 2], units, 2, 3, 0.0, oracle.exact(), lambda a, i: beh[i])
    assert rep.attempts[0].chosen == [1, 2]


def test_dmr_detects_but_cannot_decide():
    """Two disagreeing runs: no majority; every attempt re-runs the pair (no
    profile changes on an unresolved vote) until the attempts run out."""
    good = _vals(5)
    bad = good.copy()
    bad[3] = -1.0
    units = [Unit(1.0), Unit(1.0)]
    beh = {0: (OK, good, 1.0), 1: (OK, bad, 1.0)}
    rep = run_redundant([0, 1], units, 2, 3, 0.0, oracle.exact(), lambda a, i: beh[i])
    assert len(rep.attempts) == 3 and rep.verdict == oracle.UNRESOLVED
    assert [(u.valid, u.total) for u in units] == [(0, 0), (0, 0)]


def test_fewer_than_two_left_ends_the_call():
    units = [Unit(1.0), Unit(1.0), Unit(1.0)]
    rep = run_redundant([0, 1, 2], units, 2, 5, 0.0, oracle.exact(), lambda a, i: (ERROR, None, 0.0))
    # the first attempt loses both runs; one implementation is left: no second attempt
    assert len(rep.attempts) == 1 and rep.errors == 2 and rep.verdict == oracle.UNRESOLVED


def test_check_interval_retries_a_failed_unit_and_it_recovers():
    """Sec. IV-B: a unit with fault probability 1 (F infinite) is used only at
    check intervals.  With an interval of 3 it is passed over twice, then runs
    as an extra replica; it has recovered, so its run is valid and F is finite
    again.  Without check intervals it is never run again."""
    good = _vals(6)
    beh = {0: (OK, good, 1.0), 1: (OK, good, 1.0), 2: (OK, good, 0.5)}
    units = [Unit(1.0), Unit(1.0), Unit(0.5, 0, 2)]
    chosen = []
    for _ in range(4):
        rep = run_redundant([0, 1, 2], units, 2, 1, 0.0, oracle.exact(), lambda a, i: beh[i], check_interval=3)
        chosen.append(rep.attempts[0].chosen)
        assert rep.verdict == oracle.UNANIMOUS
    assert chosen[:3] == [[0, 1], [0, 1], [0, 1, 2]]
    assert (units[2].valid, units[2].total) == (1, 3) and fault_aware(units[2]) == 1.5
    assert chosen[3] == [0, 1]          # F = 1.5 now ranks it third, and finite: no more re-try
    units = [Unit(1.0), Unit(1.0), Unit(0.5, 0, 2)]
    for _ in range(5):
        rep = run_redundant([0, 1, 2], units, 2, 1, 0.0, oracle.exact(), lambda a, i: beh[i])
        assert rep.attempts[0].chosen == [0, 1]
    assert fault_aware(units[2]) == math.inf


def test_check_interval_still_faulty_unit_is_outvoted_and_retried_again():
    good = _vals(7)
    bad = good.copy()
    bad[100] = 9.0
    beh = {0: (OK, good, 1.0), 1: (OK, good, 1.0), 2: (OK, bad, 0.5)}
    units = [Unit(1.0), Unit(1.0), Unit(0.5, 0, 1)]
    chosen = []
    for _ in range(4):
        rep = run_redundant([0, 1, 2], units, 2, 1, 0.0, oracle.exact(), lambda a, i: beh[i], check_interval=2)
        chosen.append(rep.attempts[0].chosen)
        assert np.array_equal(rep.consensus, good)
    assert chosen == [[0, 1], [0, 1, 2], [0, 1], [0, 1, 2]]
    assert (units[2].valid, units[2].total) == (0, 3) and fault_aware(units[2]) == math.inf
    # a probe that fails directly counts as a run that was not valid as well
    beh[2] = (ERROR, None, 0.0)
    units = [Unit(1.0), Unit(1.0), Unit(0.5, 0, 1)]
    rep = run_redundant([0, 1, 2], units, 2, 1, 0.0, oracle.exact(), lambda a, i: beh[i], check_interval=1)
    assert rep.attempts[0].chosen == [0, 1, 2] and rep.errors == 1 and rep.verdict == oracle.UNANIMOUS
    assert (units[2].valid, units[2].total) == (0, 2)
