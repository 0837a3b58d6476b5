"""GPU tests of the continuous-batching server: every result is the same alone
and in the mix (bit for bit) and equal to the oracle; requests that arrive
while others run share launches; admission respects the HBM budget."""
import ctypes
import time

import numpy as np
import pytest

import oracle
import synth
from test_gpu_vote import U, _replicas

pytestmark = pytest.mark.gpu


def _hip():
    lib = ctypes.CDLL("libamdhip64.so")
    lib.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    lib.hipMemcpy.restype = ctypes.c_int
    return lib


def _d2h(ptr, nbytes, dtype):
    out = np.empty(nbytes // np.dtype(dtype).itemsize, dtype=dtype)
    if nbytes:
        assert _hip().hipMemcpy(out.ctypes.data, ptr, nbytes, 2) == 0   # DeviceToHost
    return out


def _requests(gpu, rng, count, max_elems):
    import torch
    reqs = []
    for i in range(count):
        dtype = [np.float32, np.float32, np.float64, np.int32][i % 4]
        k = [3, 3, 5, 2][i % 4]
        n = int(np.exp(rng.uniform(np.log(1024), np.log(max_elems))))
        if i == 7:
            n = 0
        reps = _replicas(rng, dtype, k, n)
        tol_o, tol_f = ((oracle.ulp(4), gpu.ulp(4)) if dtype == np.float32 else
                        (oracle.ulp(2), gpu.ulp(2)) if dtype == np.float64 else
                        (oracle.exact(), gpu.exact()))
        t = [torch.from_numpy(r).cuda() for r in reps]
        outs = [(torch.empty(max(n, 1), dtype=t[0].dtype, device="cuda"),
                 torch.empty(max(n, 1), dtype=torch.uint8, device="cuda")) for _ in range(2)]
        reqs.append(dict(reps=reps, t=t, tol_o=tol_o, tol_f=tol_f, outs=outs, n=n, k=k))
    return reqs


def test_alone_equals_mix_equals_oracle(gpu):
    import torch
    rng = np.random.default_rng(31)
    reqs = _requests(gpu, rng, 48, 400000)
    torch.cuda.synchronize()
    srv = gpu.Server(hbm_budget_bytes=8 << 30, chunk_bytes=256 << 10, max_slots=64)
    # the mix: Poisson arrivals at ~10000/s, submitted as they "arrive"
    print("case: serving mix of 48 requests", flush=True)
    t0 = gpu.now_ns()
    arrivals = t0 + np.cumsum(rng.exponential(100e3, len(reqs))).astype(np.int64)
    tickets = []
    for r, ta in zip(reqs, arrivals):
        while gpu.now_ns() < ta:
            pass
        c, m = r["outs"][0]
        tickets.append(srv.submit_vote(r["t"], r["tol_f"], c, m, t_arrival_ns=int(ta), n=r["n"]))
    mix = [srv.poll(tk, -1) for tk in tickets]
    st = srv.stats()
    # requests that arrived while others were on the GPU shared launches with them
    assert st["completed"] == len(reqs) and st["shared_iterations"] >= 1
    assert st["max_requests_per_iteration"] >= 2
    # overlap: some request was admitted before another one finished
    spans = sorted((res.t_admit_ns, res.t_done_ns) for res in mix)
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    for tk in tickets:
        srv.release(tk)
    # alone: one request at a time
    print("case: serving the same requests alone", flush=True)
    alone = []
    for r in reqs:
        c, m = r["outs"][1]
        tk = srv.submit_vote(r["t"], r["tol_f"], c, m, n=r["n"])
        alone.append(srv.poll(tk, -1))
        srv.release(tk)
    srv.close()
    for i, (r, a, b) in enumerate(zip(reqs, mix, alone)):
        n = r["n"]
        assert a.status == 0 and b.status == 0
        ca, ma = r["outs"][0][0][:n].cpu().numpy(), r["outs"][0][1][:n].cpu().numpy()
        cb, mb = r["outs"][1][0][:n].cpu().numpy(), r["outs"][1][1][:n].cpu().numpy()
        u = U[ca.dtype]
        assert np.array_equal(ca.view(u), cb.view(u)) and np.array_equal(ma, mb), i
        sa, sb = gpu.result_stats(a), gpu.result_stats(b)
        assert all(np.array_equal(sa[key], sb[key]) for key in sa), i
        ref = oracle.vote(r["reps"], r["tol_o"])
        assert np.array_equal(ca.view(u), ref.consensus.view(u)) and np.array_equal(ma, ref.mask), i
        k = r["k"]
        assert np.array_equal(sa["pair"][:k, :k], ref.pair) and sa["no_majority"] == ref.no_majority
        assert (sa["verdict"], sa["winner"]) == (ref.verdict, ref.winner), i


def test_server_owned_outputs_and_fingerprints(gpu):
    import torch
    rng = np.random.default_rng(5)
    ctx = gpu.Context(0)
    srv = gpu.Server(hbm_budget_bytes=1 << 30, arena_bytes=256 << 20, chunk_bytes=1 << 20, max_slots=8)
    reps = synth.small_task_set(n=(1 << 20) + 3)
    t = [torch.from_numpy(r).cuda() for r in reps]
    tk = srv.submit_vote(t, gpu.ulp(4))
    raw = rng.integers(0, 256, 3 * 65536 + 100, dtype=np.uint8)
    buf = torch.from_numpy(raw).cuda()
    tf = srv.submit_fingerprint(buf, 65536)
    res = srv.poll(tk, -1)
    fres = srv.poll(tf, -1)
    n = reps[0].size
    cons = _d2h(res.consensus, 4 * n, np.uint32)
    mask = _d2h(res.mask, n, np.uint8)
    ref = oracle.vote(reps, oracle.ulp(4))
    assert np.array_equal(cons, ref.consensus.view(np.uint32)) and np.array_equal(mask, ref.mask)
    fps = _d2h(fres.fps, 8 * fres.nfps, np.uint64)
    assert np.array_equal(fps, oracle.fingerprint(raw, 65536))
    srv.release(tk)
    srv.release(tf)
    with pytest.raises(gpu.FtvError):
        srv.release(tk)      # unknown ticket now
    srv.close()
    ctx.close()


def test_budget_queue_and_errors(gpu):
    import torch
    x = torch.zeros(1 << 20, dtype=torch.float32, device="cuda")
    one = 3 * 4 * (1 << 20) + 5 * (1 << 20)        # footprint of one k=3 fp32 request
    srv = gpu.Server(hbm_budget_bytes=one, arena_bytes=64 << 20, chunk_bytes=1 << 20, max_slots=4,
                     max_queue=1)
    with pytest.raises(gpu.FtvError) as e:
        srv.submit_vote([torch.zeros(2 << 20, device="cuda")] * 3, gpu.ulp(1))
    assert e.value.code == gpu.E_NOMEM
    t1 = srv.submit_vote([x, x, x], gpu.ulp(1))
    assert srv.poll(t1, -1).stats.verdict == gpu.UNANIMOUS
    # t1's server-owned outputs hold the whole budget until released
    t2 = srv.submit_vote([x, x, x], gpu.ulp(1))
    time.sleep(0.05)
    assert srv.poll(t2, 0) is None
    with pytest.raises(gpu.FtvError) as e:
        srv.submit_vote([x, x, x], gpu.ulp(1))
    assert e.value.code == gpu.E_BUSY
    st = srv.stats()
    assert st["queued"] == 1 and st["peak_bytes_in_flight"] <= one
    srv.release(t1)
    assert srv.poll(t2, 5_000_000) is not None
    srv.release(t2)
    assert srv.stats()["bytes_in_flight"] == 0
    xi = x.int()
    with pytest.raises(gpu.FtvError) as e:
        srv.submit_vote([xi, xi, xi], gpu.ulp(1))
    assert e.value.code == gpu.E_DTYPE
    srv.close()


def test_concurrent_submitters(gpu):
    """Submit, poll and release are thread-safe: four host threads serve their
    own requests at once (some with server-owned outputs), and every result
    equals the oracle's."""
    import threading
    import torch
    rng = np.random.default_rng(77)
    reqs = _requests(gpu, rng, 32, 200000)
    torch.cuda.synchronize()
    refs = [oracle.vote(r["reps"], r["tol_o"]) for r in reqs]
    srv = gpu.Server(hbm_budget_bytes=8 << 30, arena_bytes=512 << 20, chunk_bytes=512 << 10, max_slots=16)
    results = [None] * len(reqs)
    errors = []

    def worker(w):
        try:
            for i in range(w, len(reqs), 4):
                r = reqs[i]
                own = i % 3 == 0   # server-owned outputs for every third request
                c, m = (None, None) if own else r["outs"][0]
                tk = srv.submit_vote(r["t"], r["tol_f"], c, m, n=r["n"])
                res = srv.poll(tk, -1)
                n = r["n"]
                u = U[r["reps"][0].dtype]
                if own:
                    cons = _d2h(res.consensus, n * r["reps"][0].itemsize, u) if n else np.zeros(0, u)
                    mask = _d2h(res.mask, n, np.uint8) if n else np.zeros(0, np.uint8)
                else:
                    cons = c[:n].cpu().numpy().view(u)
                    mask = m[:n].cpu().numpy()
                results[i] = (res.status, cons, mask, gpu.result_stats(res))
                srv.release(tk)
        except Exception as e:  # reported by the main thread
            errors.append(repr(e))

    print("case: four threads submitting 32 requests", flush=True)
    threads = [threading.Thread(target=worker, args=(w,)) for w in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=60)
    srv.close()
    assert not errors, errors
    for i, (r, ref) in enumerate(zip(reqs, refs)):
        status, cons, mask, s = results[i]
        u = U[r["reps"][0].dtype]
        k = r["k"]
        assert status == 0, i
        assert np.array_equal(cons, ref.consensus.view(u)) and np.array_equal(mask, ref.mask), i
        assert np.array_equal(s["pair"][:k, :k], ref.pair) and s["no_majority"] == ref.no_majority, i
        assert (s["verdict"], s["winner"]) == (ref.verdict, ref.winner), i
