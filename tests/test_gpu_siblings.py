"""GPU: the library's sibling/version manager with device siblings against
the model in oracle/siblings.py, operation by operation, with the bytes of
every handed-out sibling compared; fingerprint checks of the newest siblings
against the model's vote over oracle fingerprints."""
import ctypes

import numpy as np
import pytest

import oracle
from oracle.siblings import DEVICE, HOST, READ, WRITE, BusyError, Manager, NoDataError

pytestmark = pytest.mark.gpu


def _data(seed, n):
    return np.random.default_rng(seed).integers(0, 256, n, dtype=np.uint8)


def _read(ftv, ptr, memory, n):
    import torch
    if memory == ftv.MEM_HOST:
        return np.frombuffer(ctypes.string_at(ptr, n), dtype=np.uint8).copy()
    out = np.empty(n, dtype=np.uint8)
    torch.cuda.synchronize()
    hip = ctypes.CDLL("libamdhip64.so")
    assert hip.hipMemcpy(ctypes.c_void_p(out.ctypes.data), ctypes.c_void_p(ptr), ctypes.c_size_t(n), 2) == 0
    return out


def _write(ftv, ptr, memory, data):
    import torch
    if memory == ftv.MEM_HOST:
        ctypes.memmove(ptr, data.ctypes.data, data.size)
        return
    torch.cuda.synchronize()
    hip = ctypes.CDLL("libamdhip64.so")
    assert hip.hipMemcpy(ctypes.c_void_p(ptr), ctypes.c_void_p(data.ctypes.data), ctypes.c_size_t(data.size), 1) == 0


def _table(mm, area):
    return [(s["memory"], s["version"], s["valid"], s["readers"], s["writing"]) for s in mm.siblings(area)]


@pytest.mark.parametrize("ft", [False, True])
def test_device_manager_matches_model(gpu, ft):
    import torch
    n = 3 * 65536 + 40
    mm = gpu.MemoryManager(device=0, fault_tolerant=ft)
    model = Manager(fault_tolerant=ft)
    areas = []
    for i in range(2):
        d = _data(60 + i, n)
        areas.append((mm.register(d.copy()), model.register(d)))
    rng = np.random.default_rng(70 + ft)
    held = []
    print(f"case: device manager vs model, fault_tolerant={ft}", flush=True)
    for step in range(250):
        ai = int(rng.integers(0, 2))
        la, ma = areas[ai]
        if held and rng.random() < 0.35:
            (la2, ma2), s, acc, mem = held.pop(int(rng.integers(0, len(held))))
            ok = bool(rng.random() < 0.8)
            new = _data(1000 + step, n) if (acc & WRITE) and ok else None
            if new is not None:
                _write(gpu, mm.siblings(la2)[s]["ptr"], mem, new)
            mm.release(la2, s, ok)
            model.release(ma2, s, ok, new)
        else:
            mem = int(rng.integers(0, 2))
            acc = int(rng.integers(1, 4))
            try:
                want = model.request(ma, mem, acc)
            except (BusyError, NoDataError):
                with pytest.raises(RuntimeError):
                    mm.request(la, mem, acc)
                continue
            ptr, got = mm.request(la, mem, acc)
            assert got == want, step
            torch.cuda.synchronize()
            assert np.array_equal(_read(gpu, ptr, mem, n), model.areas[ma].sibs[want].data), step
            held.append(((la, ma), got, acc, mem))
        for la_, ma_ in areas:
            assert _table(mm, la_) == model.table(ma_), step
    mm.close()


def test_fig1_on_the_device(gpu):
    import torch
    n = 65536
    mm = gpu.MemoryManager(device=0, fault_tolerant=True)
    d = _data(80, n)
    a = mm.register(d.copy())
    p, s = mm.request(a, gpu.MEM_DEVICE, gpu.ACC_WRITE)
    torch.cuda.synchronize()
    assert s == 1 and np.array_equal(_read(gpu, p, gpu.MEM_DEVICE, n), d)
    mm.release(a, s, ok=False)                       # a fault: the device copy is invalid
    p2, s2 = mm.request(a, gpu.MEM_DEVICE, gpu.ACC_WRITE)
    assert s2 == 1                                   # restarted from the host copy
    new = _data(81, n)
    _write(gpu, p2, gpu.MEM_DEVICE, new)
    mm.release(a, s2, ok=True)
    assert [(t[1], t[2]) for t in _table(mm, a)] == [(1, True), (2, True)]
    p3, s3 = mm.request(a, gpu.MEM_HOST, gpu.ACC_READ)
    assert s3 == 0 and np.array_equal(_read(gpu, p3, gpu.MEM_HOST, n), new)
    mm.release(a, s3, ok=True)
    mm.close()


def test_check_against_model(gpu):
    import torch
    n = 5 * 65536 + 1000
    mm = gpu.MemoryManager(device=0, fault_tolerant=True)
    model = Manager(fault_tolerant=True)
    d = _data(90, n)
    a, ma = mm.register(d.copy()), model.register(d)
    new = _data(91, n)
    for mem, acc, data in ((DEVICE, WRITE, new), (DEVICE, READ, None), (HOST, READ, None)):
        p, s = mm.request(a, mem, acc)
        sm = model.request(ma, mem, acc)
        assert s == sm
        if data is not None:
            _write(gpu, p, mem, data)
        mm.release(a, s, True)
        model.release(ma, sm, True, data)
    assert _table(mm, a) == model.table(ma) and [t[1] for t in model.table(ma)] == [2, 2, 2]
    print("case: check with three newest siblings, one corrupted", flush=True)
    sibs = mm.siblings(a)
    bad = np.array(new)
    bad[2 * 65536 + 17] ^= 0x40
    _write(gpu, sibs[2]["ptr"], gpu.MEM_DEVICE, bad)
    model.areas[ma].sibs[2].data = bad.copy()
    r = mm.check(a, 65536)
    assert (r["checked"], r["invalidated"], r["unresolved"]) == model.check(ma, 65536, oracle.fingerprint)
    assert r["blocks"] == 6 and r["invalidated"] == 1
    assert _table(mm, a) == model.table(ma)
    print("case: check with two disagreeing siblings", flush=True)
    host = np.array(new)
    host[9] ^= 1
    _write(gpu, sibs[0]["ptr"], gpu.MEM_HOST, host)
    model.areas[ma].sibs[0].data = host.copy()
    r = mm.check(a, 4096)
    assert (r["checked"], r["invalidated"], r["unresolved"]) == model.check(ma, 4096, oracle.fingerprint) == (2, 0, 1)
    mm.close()
