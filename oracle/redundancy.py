"""Model of redundant execution with light-weight fault tolerance -- TEST INFRASTRUCTURE.

Plain Python, written from the paper's description (Kicherer & Karl,
Sec. IV-B fault-aware runtime, Sec. IV-C light-weight fault tolerance,
Sec. IV-D dual-modular redundancy and the voter), against which the
library's `ftv_run_redundant` is checked attempt by attempt.  It shares no
code with the library; the vote itself is the C oracle's.

What the paper fixes:
  * each processing unit / kernel has a profile: runtime R, valid runs v,
    runs t; the fault-aware runtime is F = R * t / v (R with no history,
    infinite when v = 0 < t);
  * a task is duplicated onto the combinations with the lowest fault-aware
    runtime and the voter decides which result is taken as correct;
  * a run that reports a direct fault (an API error) is abandoned, its data
    invalid, and the task goes on with the best-ranked remaining pairing
    of kernel and unit;
  * a run that does not finish within its profiled runtime times a
    user-defined factor is abandoned the same way.

Readings where the paper is silent (the library's):
  * an attempt runs the k best implementations not yet failed in this call
    (ranked by F of their unit, ties by lower index); fewer than two left
    ends the call unresolved;
  * a failed run (error or timeout) counts as a run that was not valid
    (t + 1) and excludes that implementation for the rest of the call;
  * the surviving runs (at least two) are voted; every voted run is
    counted (t + 1) and is valid (v + 1) when it agrees with the consensus
    everywhere; the runtime profile of a valid run becomes the running mean
    of its valid runs' times; an UNRESOLVED vote counts nothing and the next
    attempt re-ranks;
  * a timeout applies only to a unit with a profile (R > 0 and v > 0); its
    limit is R * factor;
  * check intervals (Sec. IV-B: a unit with p = 1 is tried again only at
    fixed intervals): with an interval N > 0, each attempt passes over the
    units with F = inf outside its k best runs and counts one more skip for
    each; the first such unit (in rank order) whose count would reach N runs
    instead as an extra replica of the attempt, voted and counted like the
    others; a unit that runs has its count reset.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import oracle

OK, ERROR, SLOW = 0, 1, 2


@dataclass
class Unit:
    runtime: float
    valid: int = 0
    total: int = 0
    skipped: int = 0


def fault_aware(u: Unit) -> float:
    if u.total == 0:
        return u.runtime
    if u.valid == 0:
        return math.inf
    return u.runtime * (u.total / u.valid)


@dataclass
class Attempt:
    chosen: list            # implementation indices, in rank order
    failed: list            # of those, the ones that erred or timed out
    verdict: int | None     # None: fewer than two survivors, no vote


@dataclass
class Report:
    attempts: list = field(default_factory=list)
    verdict: int = oracle.UNRESOLVED
    winner_unit: int = 0
    timeouts: int = 0
    errors: int = 0
    consensus: object = None


def run_redundant(impl_units, units, k, max_attempts, timeout_factor, tol, behave, check_interval=0):
    """impl_units[i]: unit of implementation i; units: list of Unit (updated in
    place); behave(attempt, impl) -> (kind, result array, seconds): OK with
    its result and run time, ERROR, or SLOW (would exceed any timeout; its
    result is used only when no timeout applies)."""
    rep = Report()
    failed_impls = set()
    for a in range(max_attempts):
        f = [fault_aware(units[impl_units[i]]) for i in range(len(impl_units))]
        order = sorted(range(len(impl_units)), key=lambda i: (f[i], i))
        alive = [i for i in order if i not in failed_impls]
        chosen = alive[:k]
        if check_interval:
            seen = set()
            for i in chosen:
                seen.add(impl_units[i])
                units[impl_units[i]].skipped = 0
            extra = None
            for i in alive[k:]:
                u = units[impl_units[i]]
                if impl_units[i] in seen or not math.isinf(fault_aware(u)):
                    continue
                seen.add(impl_units[i])
                if extra is None and u.skipped + 1 >= check_interval:
                    extra = i
                    u.skipped = 0
                else:
                    u.skipped += 1
            if extra is not None and 2 <= len(chosen) < 7:
                chosen.append(extra)
        if len(chosen) < 2:
            break
        survivors, failed_now = [], []
        for i in chosen:
            u = units[impl_units[i]]
            kind, res, secs = behave(a, i)
            has_profile = u.runtime > 0 and u.valid > 0
            timed_out = kind == SLOW and timeout_factor > 0 and has_profile
            if kind == ERROR or timed_out:
                failed_now.append(i)
                failed_impls.add(i)
                u.total += 1
                if kind == ERROR:
                    rep.errors += 1
                else:
                    rep.timeouts += 1
                continue
            survivors.append((i, res, secs))
        if len(survivors) < 2:
            rep.attempts.append(Attempt(chosen, failed_now, None))
            continue
        v = oracle.vote([r for _, r, _ in survivors], tol)
        rep.attempts.append(Attempt(chosen, failed_now, v.verdict))
        rep.verdict = v.verdict
        if v.verdict == oracle.UNRESOLVED:
            continue
        for j, (i, _, secs) in enumerate(survivors):
            u = units[impl_units[i]]
            u.total += 1
            if v.disagree[j] == 0:
                u.valid += 1
                u.runtime = secs if u.runtime <= 0 else u.runtime + (secs - u.runtime) / u.valid
        rep.winner_unit = impl_units[survivors[v.winner][0]]
        rep.consensus = v.consensus
        return rep
    return rep
