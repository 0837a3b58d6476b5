"""Model of the runtime's sibling/version memory management -- TEST INFRASTRUCTURE.

A plain Python state machine, written from the paper's description of its
memory management unit (Kicherer & Karl, Sec. IV-A) and of how fault-tolerant
execution uses it (Sec. IV-A, second half, Fig. 1; Sec. IV-C), against which
the library's manager (`ftv_mm_*`) is checked operation by operation.  It
shares no code with the library.

What the paper fixes:
  * a registered area has copies ("siblings") in one or more memories, each
    tagged with a version that every write raises by one;
  * a request for an area in some memory looks for the newest version; if
    that memory holds a sibling at it, that sibling's address comes back,
    otherwise a sibling is made there and filled from a newest-version one;
  * fault-tolerant mode: if the desired memory holds a highest-version sibling
    and another highest-version sibling exists anywhere, the request gets the
    one in its own memory; if the newest version has a single sibling, the
    request gets a fresh one, so that the old one survives as the backup;
  * a fault detected during the kernel marks the sibling it used invalid; the
    next request copies from another valid sibling.

Readings where the paper is silent (the same readings the library takes):
  * a request that needs a new sibling reuses, in the desired memory, the
    lowest-indexed sibling that is stale or invalid and not in use, before
    allocating another; the registered host area is sibling 0;
  * among several candidates the lowest index is used; a copy source in the
    desired memory is preferred, else the lowest-indexed candidate;
  * a sibling handed out for writing is neither a candidate nor a copy source
    until it is released; a write is not given a sibling that has readers;
  * a sibling released after a detected fault is invalid whatever the access;
  * `check` fingerprints every valid highest-version sibling per block and
    invalidates those that differ from a strict majority of them in some block.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

HOST, DEVICE = 0, 1
READ, WRITE, READWRITE = 1, 2, 3


@dataclass
class Sibling:
    memory: int
    version: int
    valid: bool
    data: np.ndarray
    readers: int = 0
    writing: bool = False
    caller: bool = False     # the registered area itself


@dataclass
class Area:
    nbytes: int
    sibs: list = field(default_factory=list)


class BusyError(Exception):
    pass


class NoDataError(Exception):
    pass


class Manager:
    def __init__(self, fault_tolerant: bool):
        self.ft = bool(fault_tolerant)
        self.areas: list[Area] = []

    # -- registration: the caller's host area is sibling 0, version 1 -------
    def register(self, data: np.ndarray) -> int:
        raw = np.frombuffer(np.ascontiguousarray(data).tobytes(), dtype=np.uint8).copy()
        a = Area(raw.size, [Sibling(HOST, 1, True, raw, caller=True)])
        self.areas.append(a)
        return len(self.areas) - 1

    @staticmethod
    def newest(a: Area) -> int:
        vs = [s.version for s in a.sibs if s.valid]
        return max(vs) if vs else 0

    def candidates(self, a: Area) -> list[int]:
        v = self.newest(a)
        return [i for i, s in enumerate(a.sibs) if s.valid and not s.writing and s.version == v]

    def request(self, area: int, memory: int, access: int) -> int:
        a = self.areas[area]
        cands = self.candidates(a)
        if not cands:
            if any(s.valid and s.writing for s in a.sibs):
                raise BusyError("the newest sibling is being written")
            raise NoDataError("no valid sibling")
        writes = bool(access & WRITE)
        usable = [i for i in cands if a.sibs[i].memory == memory and not (writes and a.sibs[i].readers)]
        if usable and (not self.ft or len(cands) >= 2):
            pick = usable[0]
        else:
            pick = self._new_sibling(a, memory, cands)
        s = a.sibs[pick]
        if writes:
            s.writing = True
        else:
            s.readers += 1
        return pick

    def _new_sibling(self, a: Area, memory: int, cands: list[int]) -> int:
        v = self.newest(a)
        same = [i for i in cands if a.sibs[i].memory == memory]
        src = same[0] if same else cands[0]
        slot = None
        for i, s in enumerate(a.sibs):
            if s.memory == memory and not (s.valid and s.version == v) and not s.readers and not s.writing:
                slot = i
                break
        if slot is None:
            a.sibs.append(Sibling(memory, v, True, a.sibs[src].data.copy()))
            return len(a.sibs) - 1
        s = a.sibs[slot]
        s.data = a.sibs[src].data.copy()
        s.version = v
        s.valid = True
        return slot

    # -- release: a write that succeeded makes the sibling the newest --------
    def release(self, area: int, sib: int, ok: bool, new_data: np.ndarray | None = None):
        a = self.areas[area]
        s = a.sibs[sib]
        if s.writing:
            s.writing = False
            if ok:
                s.version = self.newest(a) + 1
                if new_data is not None:
                    s.data = np.frombuffer(np.ascontiguousarray(new_data).tobytes(), dtype=np.uint8).copy()
            else:
                s.valid = False
        else:
            if s.readers <= 0:
                raise ValueError("sibling not acquired")
            s.readers -= 1
            if not ok:
                s.valid = False

    # -- check: fingerprint vote among the newest siblings --------------------
    def check(self, area: int, block_bytes: int, fingerprint) -> tuple[int, int, int]:
        """Returns (siblings checked, siblings invalidated, blocks without a
        strict majority).  `fingerprint(bytes, block_bytes)` gives one u64 per
        block."""
        a = self.areas[area]
        cands = self.candidates(a)
        m = len(cands)
        if m < 2:
            return m, 0, 0
        fps = np.stack([fingerprint(a.sibs[i].data, block_bytes) for i in cands])   # (m, nblocks)
        bad = np.zeros(m, dtype=bool)
        unresolved = 0
        for b in range(fps.shape[1]):
            col = fps[:, b]
            support = np.array([(col == col[j]).sum() for j in range(m)])
            best = int(np.argmax(support))
            if 2 * support[best] > m:
                bad |= col != col[best]
            elif (col != col[0]).any():
                unresolved += 1
        for j, i in enumerate(cands):
            if bad[j]:
                a.sibs[i].valid = False
        return m, int(bad.sum()), unresolved

    def table(self, area: int) -> list[tuple[int, int, bool, int, bool]]:
        """(memory, version, valid, readers, writing) per sibling."""
        return [(s.memory, s.version, s.valid, s.readers, s.writing) for s in self.areas[area].sibs]
