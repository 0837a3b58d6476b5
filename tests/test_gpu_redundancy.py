"""GPU: ftv_run_redundant against the model in oracle/redundancy.py, call by
call.  Implementations are callbacks that enqueue a device copy of a prepared
result (correct or corrupted) on the stream they are given, report a direct
fault, or first run a bounded busy-wait kernel so that their unit's deadline
passes (the kernel always finishes on its own)."""
import ctypes

import numpy as np
import pytest

import oracle
from oracle.redundancy import ERROR, OK, SLOW, Unit, run_redundant

pytestmark = pytest.mark.gpu

N = 4099
SLEEP_CYCLES = 5_000_000     # a bounded busy-wait; far beyond the deadlines below


def _hip():
    return ctypes.CDLL("libamdhip64.so")


class Impls:
    """Scripted implementations: behaviour[i] in {OK, ERROR, SLOW} and the
    result (good or bad) each one produces."""

    def __init__(self, gpu, results):
        import torch
        self.gpu = gpu
        self.dev = [torch.from_numpy(r).cuda() for r in results]
        self.behaviour = [OK] * len(results)
        self.result = list(range(len(results)))
        self.hip = _hip()
        torch.cuda.synchronize()

    def fn(self, i):
        def run(out_ptr, stream_ptr):
            import torch
            b = self.behaviour[i]
            if b == ERROR:
                return 1
            if b == SLOW:
                with torch.cuda.stream(torch.cuda.ExternalStream(stream_ptr)):
                    torch.cuda._sleep(SLEEP_CYCLES)
            src = self.dev[self.result[i]]
            rc = self.hip.hipMemcpyAsync(ctypes.c_void_p(out_ptr), ctypes.c_void_p(src.data_ptr()),
                                         ctypes.c_size_t(src.numel() * src.element_size()), 3,
                                         ctypes.c_void_p(stream_ptr))
            return int(rc)
        return run


def _call(gpu, ctx, impls, units_lib, units_model, impl_units, k, attempts, factor, results, check_interval=0):
    import torch
    out = torch.empty(N, dtype=torch.float32, device="cuda")
    rep = gpu.run_redundant(ctx, [(impls.fn(i), impl_units[i]) for i in range(len(impl_units))],
                            units_lib, out, gpu.exact(), k=k, max_attempts=attempts, timeout_factor=factor,
                            check_interval=check_interval)
    torch.cuda.synchronize()

    def behave(a, i):
        b = impls.behaviour[i]
        return (b, results[impls.result[i]] if b != ERROR else None, 0.0)
    want = run_redundant(impl_units, units_model, k, attempts, factor, oracle.exact(), behave, check_interval)
    assert rep["attempts"] == len(want.attempts)
    assert rep["verdict"] == want.verdict
    assert (rep["errors"], rep["timeouts"]) == (want.errors, want.timeouts)
    assert [(u.valid, u.total, u.skipped) for u in units_lib] == \
        [(u.valid, u.total, u.skipped) for u in units_model]
    if want.verdict != oracle.UNRESOLVED:
        assert rep["winner_unit"] == want.winner_unit
        assert np.array_equal(out.cpu().numpy().view(np.uint32), want.consensus.view(np.uint32))
    # the measured runtimes of valid runs feed the next ranking: copy them over
    for ul, um in zip(units_lib, units_model):
        um.runtime = ul.runtime
    return rep


def _setup(gpu, runtimes, profiles=None):
    units_lib = (gpu.Unit * len(runtimes))()
    units_model = []
    for i, r in enumerate(runtimes):
        v, t = profiles[i] if profiles else (0, 0)
        units_lib[i] = gpu.Unit(r, v, t)
        units_model.append(Unit(r, v, t))
    return units_lib, units_model


@pytest.fixture(scope="module")
def ctx(gpu):
    c = gpu.Context(0)
    yield c
    c.close()


def _results():
    rng = np.random.default_rng(11)
    good = rng.standard_normal(N).astype(np.float32)
    bad = good.copy()
    bad[[5, 900, 4098]] += 1.0
    other = good.copy()
    other[77] = -3.0
    return [good, bad, other]


def test_dmr_error_and_tmr(gpu, ctx):
    results = _results()
    impls = Impls(gpu, results)
    impl_units = [0, 1, 2, 3]
    units_lib, units_model = _setup(gpu, [1e-3, 2e-3, 3e-3, 4e-3])
    impls.result = [0, 0, 0, 0]
    print("case: DMR, every run good", flush=True)
    rep = _call(gpu, ctx, impls, units_lib, units_model, impl_units, 2, 3, 0.0, results)
    assert rep["verdict"] == gpu.UNANIMOUS
    print("case: DMR, the best implementation reports a fault", flush=True)
    impls.behaviour = [ERROR, OK, OK, OK]
    rep = _call(gpu, ctx, impls, units_lib, units_model, impl_units, 2, 3, 0.0, results)
    assert rep["errors"] == 1 and rep["attempts"] == 2
    print("case: TMR outvotes a corrupted run", flush=True)
    impls.behaviour = [OK, OK, OK, OK]
    impls.result = [0, 1, 0, 0]
    rep = _call(gpu, ctx, impls, units_lib, units_model, impl_units, 3, 3, 0.0, results)
    assert rep["verdict"] == gpu.TASK_MAJORITY
    print("case: DMR of two different wrong results: unresolved", flush=True)
    impls.result = [1, 2, 1, 2]
    _call(gpu, ctx, impls, units_lib, units_model, [0, 1], 2, 2, 0.0, results)


def test_timeout_on_a_profiled_unit(gpu, ctx):
    results = _results()
    impls = Impls(gpu, results)
    impl_units = [0, 1, 2]
    # unit 0 is profiled and fast (deadline 0.5 ms), unit 1 has no profile
    units_lib, units_model = _setup(gpu, [1e-4, 5e-3, 1e-2], [(3, 3), (0, 0), (1, 1)])
    impls.result = [0, 0, 0]
    impls.behaviour = [SLOW, SLOW, OK]
    print("case: timeout of a profiled unit, an unprofiled slow unit kept", flush=True)
    rep = _call(gpu, ctx, impls, units_lib, units_model, impl_units, 2, 3, 5.0, results)
    assert rep["timeouts"] == 1 and rep["verdict"] == gpu.UNANIMOUS
    # a later call reuses the abandoned replica buffer only after its kernel drained
    impls.behaviour = [OK, OK, OK]
    _call(gpu, ctx, impls, units_lib, units_model, impl_units, 3, 2, 0.0, results)


def test_random_calls_match_the_model(gpu, ctx):
    results = _results()
    impls = Impls(gpu, results)
    rng = np.random.default_rng(12)
    impl_units = [0, 1, 2, 3, 1]          # two implementations on unit 1
    units_lib, units_model = _setup(gpu, [1e-3, 1.5e-3, 2e-3, 2.5e-3])
    for call in range(24):
        impls.behaviour = [int(x) for x in rng.choice([OK, OK, OK, ERROR], size=5)]
        impls.result = [int(x) for x in rng.choice([0, 0, 0, 1, 2], size=5)]
        k = int(rng.choice([2, 3]))
        print(f"case: random call {call}: behaviour={impls.behaviour} results={impls.result} k={k}", flush=True)
        _call(gpu, ctx, impls, units_lib, units_model, impl_units, k, 3, 0.0, results)


def test_check_interval_retries_a_failed_unit(gpu, ctx):
    """A unit whose every run failed (F infinite) is passed over and re-tried
    as an extra replica every third attempt; while its results are wrong it is
    outvoted, and once it returns good results it regains a finite F --
    profiles, skip counts, verdicts and consensus call by call equal to the
    model's."""
    results = _results()
    impls = Impls(gpu, results)
    impl_units = [0, 1, 2]
    units_lib, units_model = _setup(gpu, [1e-3, 2e-3, 5e-4], [(0, 0), (0, 0), (0, 2)])
    impls.behaviour = [OK, OK, OK]
    for call in range(7):
        impls.result = [0, 0, 1 if call < 3 else 0]      # unit 2 recovers after its first re-try
        print(f"case: check interval 3, call {call}, unit 2 result {impls.result[2]}", flush=True)
        _call(gpu, ctx, impls, units_lib, units_model, impl_units, 2, 1, 0.0, results, check_interval=3)
    assert units_lib[2].valid >= 1 and gpu.fault_aware_runtime(units_lib[2]) < float("inf")
