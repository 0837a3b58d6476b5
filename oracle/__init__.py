"""CPU oracle for the heterogeneity-aware majority voter -- TEST INFRASTRUCTURE.

Plain, slow, sequential C (``ftv_oracle.c``) behind a ctypes wrapper.  Only the
test suite, the smoke check and the CPU-baseline leg of the benchmark may import
this package; the GPU library never does, and the two share no code.

The definitions follow the paper's statement of the voter (Kicherer & Karl,
Sec. IV-D): integer values are compared bit-wise, floating-point values are
equal when they differ by no more than a programmer-set maximum, and the voter
decides which of the duplicated task runs' results is to be taken as correct.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ftv_oracle.c")
_LIB = os.path.join(_HERE, "libftv_oracle.so")

# value types and tolerance kinds (numbering private to the oracle)
F32, F64, I32, I64 = 0, 1, 2, 3
EXACT, ULP, REL = 0, 1, 2
UNANIMOUS, TASK_MAJORITY, ELEMENT_MAJORITY, UNRESOLVED = 0, 1, 2, 3
NOMAJ_BIT = 0x80

_NP2DT = {np.dtype(np.float32): F32, np.dtype(np.float64): F64,
          np.dtype(np.int32): I32, np.dtype(np.int64): I64}
_DT2UINT = {F32: np.uint32, F64: np.uint64, I32: np.uint32, I64: np.uint64}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: no FMA contraction, no fast-math."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-Wall", "-Wextra", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        u64, i32, dbl, vp = ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        L.fto_eq.argtypes = [i32, i32, u64, dbl, dbl, u64, u64]
        L.fto_eq.restype = i32
        L.fto_ulp_distance.argtypes = [i32, u64, u64]
        L.fto_ulp_distance.restype = u64
        L.fto_order_key.argtypes = [i32, u64]
        L.fto_order_key.restype = u64
        L.fto_vote.argtypes = [i32, i32, u64, vp, i32, u64, dbl, dbl, vp, vp, vp, vp]
        L.fto_vote.restype = i32
        L.fto_vote_threads.argtypes = [i32, i32, u64, vp, i32, u64, dbl, dbl, vp, vp, vp, vp, i32, vp]
        L.fto_vote_threads.restype = i32
        L.fto_fnv1a_words.argtypes = [vp, u64]
        L.fto_fnv1a_words.restype = u64
        L.fto_fingerprint.argtypes = [vp, u64, u64, vp]
        L.fto_fingerprint.restype = i32
        L.fto_vote_blocks.argtypes = [i32, i32, u64, vp, i32, u64, dbl, dbl, u64,
                                      vp, vp, vp, vp, vp, vp]
        L.fto_vote_blocks.restype = i32
        L.fto_fault_aware_runtime.argtypes = [dbl, u64, u64]
        L.fto_fault_aware_runtime.restype = dbl
        _lib = L
    return _lib


@dataclass(frozen=True)
class Tol:
    """Tolerance: EXACT (bit-wise), ULP (ordered-key distance <= max_ulp) or
    REL (|a-b| <= delta*max(|a|,|b|) or <= abs_floor, in binary64)."""
    kind: int = EXACT
    max_ulp: int = 0
    delta: float = 0.0
    abs_floor: float = 0.0


def exact() -> Tol:
    return Tol(EXACT)


def ulp(n: int) -> Tol:
    return Tol(ULP, max_ulp=int(n))


def rel(delta: float = 1e-3, abs_floor: float = 0.0) -> Tol:
    return Tol(REL, delta=float(delta), abs_floor=float(abs_floor))


def dtype_code(dt) -> int:
    return _NP2DT[np.dtype(dt)]


def _bits(a: np.ndarray) -> np.ndarray:
    return a.view(_DT2UINT[dtype_code(a.dtype)])


def eq(dtype, tol: Tol, a_bits: int, b_bits: int) -> bool:
    return bool(lib().fto_eq(dtype_code(dtype), tol.kind, tol.max_ulp, tol.delta, tol.abs_floor,
                             int(a_bits), int(b_bits)))


def ulp_distance(dtype, a_bits: int, b_bits: int) -> int:
    return int(lib().fto_ulp_distance(dtype_code(dtype), int(a_bits), int(b_bits)))


def order_key(dtype, bits: int) -> int:
    return int(lib().fto_order_key(dtype_code(dtype), int(bits)))


@dataclass
class VoteResult:
    consensus: np.ndarray
    mask: np.ndarray
    pair: np.ndarray          # (k, k) uint64, symmetric, zero diagonal
    disagree: np.ndarray      # (k,) uint64
    no_majority: int
    verdict: int
    winner: int


def _ptr_array(arrs):
    ptrs = (ctypes.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
    return ptrs


def vote(replicas, tol: Tol) -> VoteResult:
    """Element-wise majority vote over k replica arrays of one dtype."""
    reps = [np.ascontiguousarray(r) for r in replicas]
    k = len(reps)
    dt = reps[0].dtype
    n = reps[0].size
    for r in reps:
        if r.dtype != dt or r.size != n:
            raise ValueError("replicas must share dtype and size")
    cons = np.empty(n, dtype=dt)
    mask = np.empty(n, dtype=np.uint8)
    counts = np.zeros(57, dtype=np.uint64)
    vw = np.zeros(2, dtype=np.int32)
    ptrs = _ptr_array(reps)
    rc = lib().fto_vote(dtype_code(dt), k, n, ctypes.cast(ptrs, ctypes.c_void_p), tol.kind,
                        tol.max_ulp, tol.delta, tol.abs_floor, cons.ctypes.data,
                        mask.ctypes.data, counts.ctypes.data, vw.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle vote rejected arguments (code {rc})")
    pair = counts[:49].reshape(7, 7)[:k, :k].copy()
    return VoteResult(cons, mask, pair, counts[49:49 + k].copy(), int(counts[56]),
                      int(vw[0]), int(vw[1]))


def vote_threads(replicas, tol: Tol, nthreads: int = 0):
    """The same vote with the element loop split over host threads (OpenMP);
    returns (VoteResult, threads used).  nthreads = 0: OpenMP's default."""
    reps = [np.ascontiguousarray(r) for r in replicas]
    k = len(reps)
    dt = reps[0].dtype
    n = reps[0].size
    for r in reps:
        if r.dtype != dt or r.size != n:
            raise ValueError("replicas must share dtype and size")
    cons = np.empty(n, dtype=dt)
    mask = np.empty(n, dtype=np.uint8)
    counts = np.zeros(57, dtype=np.uint64)
    vw = np.zeros(2, dtype=np.int32)
    used = ctypes.c_int(0)
    ptrs = _ptr_array(reps)
    rc = lib().fto_vote_threads(dtype_code(dt), k, n, ctypes.cast(ptrs, ctypes.c_void_p), tol.kind,
                                tol.max_ulp, tol.delta, tol.abs_floor, cons.ctypes.data,
                                mask.ctypes.data, counts.ctypes.data, vw.ctypes.data, int(nthreads),
                                ctypes.byref(used))
    if rc != 0:
        raise ValueError(f"oracle vote rejected arguments (code {rc})")
    pair = counts[:49].reshape(7, 7)[:k, :k].copy()
    return VoteResult(cons, mask, pair, counts[49:49 + k].copy(), int(counts[56]),
                      int(vw[0]), int(vw[1])), int(used.value)


def fnv1a_words(words) -> int:
    w = np.ascontiguousarray(np.asarray(words, dtype=np.uint64))
    return int(lib().fto_fnv1a_words(w.ctypes.data, w.size))


def fingerprint(buf, block_bytes: int = 65536) -> np.ndarray:
    """One 64-bit fingerprint per block of block_bytes (zero-padded tail)."""
    b = np.ascontiguousarray(np.frombuffer(memoryview(buf).cast("B"), dtype=np.uint8)
                             if not isinstance(buf, np.ndarray) else buf.reshape(-1).view(np.uint8))
    nblocks = (b.size + block_bytes - 1) // block_bytes
    out = np.zeros(nblocks, dtype=np.uint64)
    rc = lib().fto_fingerprint(b.ctypes.data, b.size, block_bytes, out.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle fingerprint rejected arguments (code {rc})")
    return out


@dataclass
class BlockVoteResult:
    fps: np.ndarray           # (k, nblocks)
    blockmap: np.ndarray      # (nblocks,) uint8
    consensus: np.ndarray
    mask: np.ndarray
    blocks: int
    disagree_blocks: int
    fallback_blocks: int
    unresolved_elems: int
    replica_blocks: np.ndarray
    verdict: int
    winner: int


def vote_blocks(replicas, tol: Tol, block_bytes: int = 65536) -> BlockVoteResult:
    reps = [np.ascontiguousarray(r) for r in replicas]
    k = len(reps)
    dt = reps[0].dtype
    n = reps[0].size
    nbytes = reps[0].nbytes
    nblocks = (nbytes + block_bytes - 1) // block_bytes
    fps = np.zeros((k, nblocks), dtype=np.uint64)
    bmap = np.zeros(nblocks, dtype=np.uint8)
    cons = np.empty(n, dtype=dt)
    mask = np.empty(n, dtype=np.uint8)
    bst = np.zeros(11, dtype=np.uint64)
    vw = np.zeros(2, dtype=np.int32)
    ptrs = _ptr_array(reps)
    rc = lib().fto_vote_blocks(dtype_code(dt), k, nbytes, ctypes.cast(ptrs, ctypes.c_void_p),
                               tol.kind, tol.max_ulp, tol.delta, tol.abs_floor, block_bytes,
                               fps.ctypes.data, bmap.ctypes.data, cons.ctypes.data,
                               mask.ctypes.data, bst.ctypes.data, vw.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle block vote rejected arguments (code {rc})")
    return BlockVoteResult(fps, bmap, cons, mask, int(bst[0]), int(bst[1]), int(bst[2]),
                           int(bst[3]), bst[4:4 + k].copy(), int(vw[0]), int(vw[1]))


def fault_aware_runtime(runtime: float, valid: int, total: int) -> float:
    """F = R / (1 - p) with p = 1 - valid/total (Sec. IV-B)."""
    return float(lib().fto_fault_aware_runtime(float(runtime), int(valid), int(total)))
