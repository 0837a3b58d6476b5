"""Sibling/version memory management (Sec. IV-A, IV-C): the model in
oracle/siblings.py pinned to the paper's narrative (Fig. 1), its invariants,
and the library's host-only manager checked against it operation by
operation (no GPU needed: every sibling lives in host memory)."""
import ctypes

import numpy as np
import pytest

import oracle
from oracle.siblings import DEVICE, HOST, READ, READWRITE, WRITE, BusyError, Manager, NoDataError


def _data(seed, n=4096):
    return np.random.default_rng(seed).integers(0, 256, n, dtype=np.uint8)


# ---- pins: the paper's worked example -------------------------------------
def test_fig1_fault_on_the_device_and_restart():
    """Sec. IV-A, Fig. 1: "input" and "output" registered in host memory; a
    kernel on a GPU gets new siblings; a fault invalidates the GPU's
    "output"; the up-to-date host "output" allows the restart; the successful
    run raises the GPU sibling's version by one; a later read elsewhere copies
    from it, the highest version."""
    m = Manager(fault_tolerant=True)
    inp, out = m.register(_data(1)), m.register(_data(2))
    si = m.request(inp, DEVICE, READ)
    so = m.request(out, DEVICE, WRITE)
    # new siblings in device memory, copies of version 1; host areas untouched
    assert (si, so) == (1, 1)
    assert m.table(inp) == [(HOST, 1, True, 0, False), (DEVICE, 1, True, 1, False)]
    assert m.table(out) == [(HOST, 1, True, 0, False), (DEVICE, 1, True, 0, True)]
    # fault during execution: "output" on the device is invalidated
    m.release(inp, si, ok=True)
    m.release(out, so, ok=False)
    assert m.table(out) == [(HOST, 1, True, 0, False), (DEVICE, 1, False, 0, False)]
    # restart: the host copy is still up to date; the device gets a fresh copy
    so2 = m.request(out, DEVICE, WRITE)
    assert so2 == 1 and m.table(out)[1] == (DEVICE, 1, True, 0, True)
    new = _data(3)
    m.release(out, so2, ok=True, new_data=new)
    assert m.table(out) == [(HOST, 1, True, 0, False), (DEVICE, 2, True, 0, False)]
    # read access from another processing unit: transferred from the device
    # sibling, the highest version (fault-tolerant: the device copy stays)
    sh = m.request(out, HOST, READ)
    assert sh == 0 and m.table(out)[0] == (HOST, 2, True, 1, False)
    assert np.array_equal(m.areas[out].sibs[0].data, new)


def test_normal_mode_reuses_the_sibling_in_place():
    """Sec. IV-A: a request returns the address of an up-to-date sibling that
    is already in the memory; a write raises the version by one; a request
    elsewhere copies from the newest-version sibling."""
    m = Manager(fault_tolerant=False)
    a = m.register(_data(4))
    s = m.request(a, HOST, READWRITE)
    assert s == 0                      # no copy: the registered area itself
    m.release(a, s, ok=True, new_data=_data(5))
    assert m.table(a) == [(HOST, 2, True, 0, False)]
    d = m.request(a, DEVICE, READ)
    assert d == 1 and m.table(a)[1] == (DEVICE, 2, True, 1, False)
    m.release(a, d, ok=True)
    d2 = m.request(a, DEVICE, WRITE)   # in place, normal mode
    assert d2 == 1
    m.release(a, d2, ok=True, new_data=_data(6))
    assert [t[1] for t in m.table(a)] == [2, 3]
    h = m.request(a, HOST, READ)       # stale host area refreshed from the device
    assert h == 0 and m.table(a)[0] == (HOST, 3, True, 1, False)
    assert np.array_equal(m.areas[a].sibs[0].data, _data(6))


def test_fault_tolerant_mode_keeps_a_backup():
    """Sec. IV-A: with only one highest-version sibling a new one is created
    even in the same memory; with two, the request gets the one in its memory."""
    m = Manager(fault_tolerant=True)
    a = m.register(_data(7))
    s = m.request(a, HOST, WRITE)      # only one newest copy: a new host sibling
    assert s == 1 and m.table(a)[0] == (HOST, 1, True, 0, False)
    m.release(a, s, ok=False)          # fault: the backup (the registered area) is intact
    assert m.table(a) == [(HOST, 1, True, 0, False), (HOST, 1, False, 0, False)]
    r = m.request(a, DEVICE, READ)     # one valid newest copy -> a new device sibling
    assert r == 2
    m.release(a, r, ok=True)
    r2 = m.request(a, DEVICE, READ)    # two newest (host 0, device 2): used in place
    assert r2 == 2


def test_busy_and_lost_data_are_errors():
    m = Manager(fault_tolerant=False)
    a = m.register(_data(8))
    s = m.request(a, HOST, WRITE)
    with pytest.raises(BusyError):
        m.request(a, DEVICE, READ)
    m.release(a, s, ok=False)
    with pytest.raises(NoDataError):
        m.request(a, DEVICE, READ)


def test_check_invalidates_the_minority():
    m = Manager(fault_tolerant=True)
    a = m.register(_data(9, 65536 * 3 + 100))
    w = m.request(a, DEVICE, WRITE)
    m.release(a, w, ok=True, new_data=_data(10, 65536 * 3 + 100))
    r = m.request(a, DEVICE, READ)     # second device copy (fault-tolerant)
    m.release(a, r, ok=True)
    h = m.request(a, HOST, READ)       # host refreshed: three newest siblings
    m.release(a, h, ok=True)
    assert [t[1] for t in m.table(a)] == [2, 2, 2]
    m.areas[a].sibs[r].data[70000] ^= 1          # a fault in one copy, block 1
    assert m.check(a, 65536, oracle.fingerprint) == (3, 1, 0)
    assert [t[2] for t in m.table(a)] == [True, True, False]
    # two copies that disagree: no strict majority, nothing invalidated
    m.areas[a].sibs[0].data[5] ^= 1
    assert m.check(a, 65536, oracle.fingerprint) == (2, 0, 1)


# ---- invariants under random operation sequences ---------------------------
def _random_ops(seed, steps=300):
    rng = np.random.default_rng(seed)
    ops = []
    for _ in range(steps):
        ops.append((int(rng.integers(0, 2)), int(rng.integers(0, 2)), int(rng.integers(1, 4)),
                    bool(rng.random() < 0.8), int(rng.integers(0, 1 << 30))))
    return ops


@pytest.mark.parametrize("ft", [False, True])
def test_model_invariants(ft):
    m = Manager(fault_tolerant=ft)
    areas = [m.register(_data(20 + i, 512)) for i in range(2)]
    held = []
    for area_i, mem, acc, ok, seed in _random_ops(11 + ft):
        a = areas[area_i]
        if held and seed % 3 == 0:
            a2, s, acc2 = held.pop(seed % len(held))
            before = Manager.newest(m.areas[a2])
            m.release(a2, s, ok, _data(seed, 512) if acc2 & WRITE else None)
            if (acc2 & WRITE) and ok:   # a successful write is the new newest, one above
                assert m.areas[a2].sibs[s].version == before + 1 == Manager.newest(m.areas[a2])
        else:
            try:
                s = m.request(a, mem, acc)
            except (BusyError, NoDataError):
                continue
            sib = m.areas[a].sibs[s]
            assert sib.memory == mem and sib.valid
            if ft:   # a valid copy of the newest data survives this request
                others = [i for i in m.candidates(m.areas[a]) if i != s]
                assert others
            held.append((a, s, acc))
        for ar in areas:
            c = m.candidates(m.areas[ar])
            if len(c) > 1:
                first = m.areas[ar].sibs[c[0]].data
                assert all(np.array_equal(m.areas[ar].sibs[i].data, first) for i in c)


# ---- the library's host-only manager against the model ---------------------
def _lib_table(mm, area):
    return [(s["memory"], s["version"], s["valid"], s["readers"], s["writing"])
            for s in mm.siblings(area)]


def _lib_bytes(ptr, n):
    return np.frombuffer(ctypes.string_at(ptr, n), dtype=np.uint8)


@pytest.mark.parametrize("ft", [False, True])
def test_host_only_manager_matches_model(ft):
    import paper_1405_2912_amd as ftv
    mm = ftv.MemoryManager(device=-1, fault_tolerant=ft)
    model = Manager(fault_tolerant=ft)
    areas = []
    for i in range(2):
        d = _data(30 + i, 777)
        areas.append((mm.register(d.copy()), model.register(d)))
    held = []
    for area_i, _mem, acc, ok, seed in _random_ops(40 + ft, 400):
        la, ma = areas[area_i]
        if held and seed % 3 == 0:
            (la2, ma2), s, acc2 = held.pop(seed % len(held))
            new = _data(seed, 777) if (acc2 & WRITE) and ok else None
            if new is not None:
                ptr = mm.siblings(la2)[s]["ptr"]
                ctypes.memmove(ptr, new.ctypes.data, new.size)
            mm.release(la2, s, ok)
            model.release(ma2, s, ok, new)
        else:
            try:
                want = model.request(ma, HOST, acc)
            except BusyError:
                with pytest.raises(RuntimeError, match="being written"):
                    mm.request(la, ftv.MEM_HOST, acc)
                continue
            except NoDataError:
                with pytest.raises(RuntimeError, match="no valid sibling"):
                    mm.request(la, ftv.MEM_HOST, acc)
                continue
            ptr, got = mm.request(la, ftv.MEM_HOST, acc)
            assert got == want
            assert np.array_equal(_lib_bytes(ptr, 777), model.areas[ma].sibs[want].data)
            held.append(((la, ma), got, acc))
        for la_, ma_ in areas:
            assert _lib_table(mm, la_) == model.table(ma_)
    mm.close()


def test_host_only_manager_rejects_device_use():
    import paper_1405_2912_amd as ftv
    mm = ftv.MemoryManager(device=-1, fault_tolerant=True)
    a = mm.register(_data(50))
    with pytest.raises(RuntimeError, match="host-only"):
        mm.request(a, ftv.MEM_DEVICE, ftv.ACC_READ)
    with pytest.raises(RuntimeError, match="host-only"):
        mm.check(a)
    with pytest.raises(RuntimeError):
        mm.release(a, 0, True)          # not in use
    mm.close()
