"""ctypes binding of libftv.so -- argument marshalling only.

Every step of the vote, the fingerprints, the block vote, the batched launch
and the server runs in the gfx950 library; PyTorch only provides device memory
(tensors) and streams.  If the library is missing, load() raises: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, Structure, c_char_p, c_double, c_int, c_int32, c_int64, c_uint8,
                    c_uint32, c_uint64, c_void_p)

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libftv.so")

# ---- constants mirrored from include/ftv.h ---------------------------------
OK, E_INVALID, E_DTYPE, E_K, E_ALIGN, E_HIP, E_NOMEM, E_BUSY, E_NOTREADY, E_CLOSED, E_MISMATCH = \
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10
F32, F64, I32, I64 = 0, 1, 2, 3
TOL_EXACT, TOL_ULP, TOL_REL = 0, 1, 2
UNANIMOUS, TASK_MAJORITY, ELEMENT_MAJORITY, UNRESOLVED = 0, 1, 2, 3
MAX_K = 7
MASK_NOMAJ = 0x80
NOALLOC_MAX_TASKS = 4096
REQ_VOTE, REQ_FINGERPRINT = 0, 1
VOTER_HOST1, VOTER_HOSTMT, VOTER_GPU = 0, 1, 2
NUM_VOTERS = 3
PLACE_REDUNDANT = 1


class FtvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ftv error {code}: {msg}")
        self.code = code


class Tol(Structure):
    _fields_ = [("kind", c_int32), ("reserved", c_uint32), ("max_ulp", c_uint64),
                ("delta", c_double), ("abs_floor", c_double)]


class Stats(Structure):
    _fields_ = [("pair", c_uint64 * 49), ("disagree", c_uint64 * 7), ("no_majority", c_uint64),
                ("n", c_uint64), ("verdict", c_int32), ("winner", c_int32)]


class VoteDesc(Structure):
    _fields_ = [("replicas", c_void_p * 7), ("k", c_uint32), ("dtype", c_int32), ("n", c_uint64),
                ("tol", Tol), ("consensus", c_void_p), ("mask", c_void_p), ("stats", c_void_p)]


class BatchCfg(Structure):
    _fields_ = [("tile_vecs", c_uint32), ("block", c_uint32), ("grid_mult", c_uint32),
                ("order", c_uint32), ("nt_stores", c_uint32), ("reserved", c_uint32)]


class BlockStats(Structure):
    _fields_ = [("blocks", c_uint64), ("disagree_blocks", c_uint64), ("fallback_blocks", c_uint64),
                ("unresolved_elems", c_uint64), ("replica_blocks", c_uint64 * 7),
                ("verdict", c_int32), ("winner", c_int32)]


class ServerCfg(Structure):
    _fields_ = [("hbm_budget_bytes", c_uint64), ("arena_bytes", c_uint64), ("chunk_bytes", c_uint64),
                ("max_slots", c_uint32), ("max_queue", c_uint32), ("device", c_int32),
                ("reserved", c_uint32)]


class Request(Structure):
    _fields_ = [("kind", c_int32), ("reserved", c_uint32), ("vote", VoteDesc),
                ("fp_buf", c_void_p), ("fp_bytes", c_uint64), ("block_bytes", c_uint64),
                ("t_arrival_ns", c_int64), ("user_tag", c_uint64), ("ready", c_void_p)]


class Result(Structure):
    _fields_ = [("status", c_int32), ("kind", c_int32), ("stats", Stats), ("consensus", c_void_p),
                ("mask", c_void_p), ("fps", c_void_p), ("nfps", c_uint64),
                ("t_arrival_ns", c_int64), ("t_submit_ns", c_int64), ("t_admit_ns", c_int64),
                ("t_done_ns", c_int64), ("user_tag", c_uint64)]


class ServerStats(Structure):
    _fields_ = [("submitted", c_uint64), ("completed", c_uint64), ("queued", c_uint64),
                ("in_flight", c_uint64), ("rejected", c_uint64), ("bytes_in_flight", c_uint64),
                ("peak_bytes_in_flight", c_uint64), ("iterations", c_uint64),
                ("peak_queue_depth", c_uint64), ("shared_iterations", c_uint64),
                ("max_requests_per_iteration", c_uint64), ("mean_queue_depth", c_double),
                ("p50_us", c_double), ("p99_us", c_double), ("mean_us", c_double),
                ("max_us", c_double), ("replica_gbps", c_double)]


class Unit(Structure):
    _fields_ = [("runtime", c_double), ("valid", c_uint64), ("total", c_uint64), ("skipped", c_uint64)]


class SiblingInfo(Structure):
    _fields_ = [("ptr", c_void_p), ("memory", c_int32), ("valid", c_int32), ("version", c_uint64),
                ("readers", c_uint32), ("writing", c_int32), ("caller", c_int32),
                ("reserved", c_uint32)]


TaskFn = ctypes.CFUNCTYPE(c_int, c_void_p, c_void_p, c_void_p)


class Impl(Structure):
    _fields_ = [("run", TaskFn), ("user", c_void_p), ("unit", c_uint32), ("reserved", c_uint32)]


class RedundancyCfg(Structure):
    _fields_ = [("k", c_uint32), ("max_attempts", c_uint32), ("timeout_factor", c_double),
                ("dtype", c_int32), ("check_interval", c_uint32), ("tol", Tol)]


class RedundancyReport(Structure):
    _fields_ = [("attempts", c_uint32), ("verdict", c_int32), ("timeouts", c_uint32),
                ("errors", c_uint32), ("winner_unit", c_uint32), ("reserved", c_uint32),
                ("seconds", c_double)]


class PlaceReport(Structure):
    _fields_ = [("unit", c_int32 * 3), ("runs", c_uint32), ("result_unit", c_int32), ("agreed", c_int32),
                ("probed", c_uint32), ("reserved", c_uint32), ("seconds", c_double * 3)]


class MMCheckResult(Structure):
    _fields_ = [("checked", c_uint32), ("invalidated", c_uint32), ("unresolved", c_uint64),
                ("blocks", c_uint64)]


EXPORTS = ["ftv_version", "ftv_last_error", "ftv_now_ns", "ftv_ctx_create", "ftv_ctx_destroy",
           "ftv_vote", "ftv_vote_batch", "ftv_batch_get_config", "ftv_batch_set_config",
           "ftv_tune_batch", "ftv_fingerprint", "ftv_vote_blocks", "ftv_server_create",
           "ftv_submit", "ftv_poll", "ftv_release", "ftv_server_get_stats",
           "ftv_server_destroy", "ftv_fault_aware_runtime", "ftv_rank_units", "ftv_record_vote",
           "ftv_mm_create", "ftv_mm_destroy", "ftv_mm_register", "ftv_mm_request", "ftv_mm_release",
           "ftv_mm_siblings", "ftv_mm_check", "ftv_run_redundant", "ftv_vote_mem",
           "ftv_ctx_set_timing", "ftv_ctx_kernel_times", "ftv_vote_batch_noalloc", "ftv_vote_host",
           "ftv_voter_db_create", "ftv_voter_db_destroy", "ftv_voter_db_profile", "ftv_voter_db_inject",
           "ftv_vote_placed"]

_lib = None


def load():
    """Load libftv.so (built in-tree by build()); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1405_2912_amd.build` (there is no CPU fallback)")
    # PyTorch supplies the device memory and streams; it is imported before the
    # library makes its first HIP call (importing it afterwards left torch
    # seeing no GPU on MI355X).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp = c_void_p
    L.ftv_version.restype = c_char_p
    L.ftv_last_error.restype = c_char_p
    L.ftv_now_ns.restype = c_int64
    L.ftv_ctx_create.argtypes = [c_int, POINTER(vp)]
    L.ftv_ctx_destroy.argtypes = [vp]
    L.ftv_vote.argtypes = [vp, POINTER(VoteDesc), vp]
    L.ftv_ctx_set_timing.argtypes = [vp, c_int]
    L.ftv_ctx_kernel_times.argtypes = [vp, POINTER(ctypes.c_float), c_uint32, POINTER(c_uint32)]
    L.ftv_vote_batch.argtypes = [vp, POINTER(VoteDesc), c_uint64, vp]
    L.ftv_vote_batch_noalloc.argtypes = [POINTER(VoteDesc), c_uint64, vp]
    L.ftv_vote_mem.argtypes = [vp, POINTER(VoteDesc), POINTER(ctypes.c_int32), c_uint64, vp]
    L.ftv_batch_get_config.argtypes = [vp, POINTER(BatchCfg)]
    L.ftv_batch_set_config.argtypes = [vp, POINTER(BatchCfg)]
    L.ftv_tune_batch.argtypes = [vp, POINTER(VoteDesc), c_uint64, vp, c_uint32, POINTER(BatchCfg)]
    L.ftv_fingerprint.argtypes = [vp, vp, c_uint64, c_uint64, vp, vp]
    L.ftv_vote_blocks.argtypes = [vp, POINTER(c_void_p), c_uint32, c_int32, c_uint64, c_uint64,
                                  POINTER(Tol), vp, vp, vp, vp, vp, vp]
    if hasattr(L, "ftv_server_create"):
        L.ftv_server_create.argtypes = [POINTER(ServerCfg), POINTER(vp)]
        L.ftv_submit.argtypes = [vp, POINTER(Request), POINTER(c_uint64)]
        L.ftv_poll.argtypes = [vp, c_uint64, POINTER(Result), c_int64]
        L.ftv_release.argtypes = [vp, c_uint64]
        L.ftv_server_get_stats.argtypes = [vp, POINTER(ServerStats)]
        L.ftv_server_destroy.argtypes = [vp]
    L.ftv_fault_aware_runtime.argtypes = [POINTER(Unit)]
    L.ftv_rank_units.argtypes = [POINTER(Unit), c_uint32, c_int, POINTER(c_uint32)]
    L.ftv_record_vote.argtypes = [POINTER(Unit), c_uint32, POINTER(c_uint32), c_uint32, POINTER(Stats)]
    L.ftv_mm_create.argtypes = [c_int, c_int, POINTER(vp)]
    L.ftv_mm_destroy.argtypes = [vp]
    L.ftv_mm_register.argtypes = [vp, vp, c_uint64, POINTER(c_uint32)]
    L.ftv_mm_request.argtypes = [vp, c_uint32, c_int, c_int, vp, POINTER(vp), POINTER(c_uint32)]
    L.ftv_mm_release.argtypes = [vp, c_uint32, c_uint32, c_int]
    L.ftv_mm_siblings.argtypes = [vp, c_uint32, POINTER(SiblingInfo), c_uint32, POINTER(c_uint32)]
    L.ftv_mm_check.argtypes = [vp, c_uint32, c_uint64, vp, POINTER(MMCheckResult)]
    L.ftv_run_redundant.argtypes = [vp, POINTER(Impl), c_uint32, POINTER(Unit), c_uint32,
                                    POINTER(RedundancyCfg), c_uint64, vp, POINTER(RedundancyReport)]
    L.ftv_vote_host.argtypes = [POINTER(VoteDesc), c_uint32]
    L.ftv_voter_db_create.argtypes = [c_uint32, c_uint32, POINTER(vp)]
    L.ftv_voter_db_destroy.argtypes = [vp]
    L.ftv_voter_db_profile.argtypes = [vp, c_uint32, c_uint64, c_uint32, c_int32, POINTER(Unit)]
    L.ftv_voter_db_inject.argtypes = [vp, c_uint32, c_uint32]
    L.ftv_vote_placed.argtypes = [vp, vp, POINTER(VoteDesc), POINTER(c_int32), c_int32, c_uint32, c_uint32, vp,
                                  POINTER(PlaceReport)]
    for name in EXPORTS:
        fn = getattr(L, name, None)
        if fn is not None and name not in ("ftv_version", "ftv_last_error", "ftv_now_ns",
                                           "ftv_fault_aware_runtime"):
            fn.restype = c_int
    L.ftv_fault_aware_runtime.restype = c_double
    _lib = L
    return L


def _check(rc: int):
    if rc != OK:
        raise FtvError(rc, load().ftv_last_error().decode())


def now_ns() -> int:
    return int(load().ftv_now_ns())


# ---- tolerances ------------------------------------------------------------
def exact() -> Tol:
    return Tol(TOL_EXACT, 0, 0, 0.0, 0.0)


def ulp(n: int) -> Tol:
    return Tol(TOL_ULP, 0, int(n), 0.0, 0.0)


def rel(delta: float = 1e-3, abs_floor: float = 0.0) -> Tol:
    return Tol(TOL_REL, 0, 0, float(delta), float(abs_floor))


# ---- torch plumbing ----------------------------------------------------------
def _torch():
    import torch
    return torch


def dtype_code(t) -> int:
    torch = _torch()
    m = {torch.float32: F32, torch.float64: F64, torch.int32: I32, torch.int64: I64}
    if t.dtype not in m:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return m[t.dtype]


def _stream_handle(stream) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def stats_tensor(device, count: int = 1):
    """Device buffer for `count` ftv_stats records (8-byte aligned)."""
    torch = _torch()
    return torch.zeros(count * ctypes.sizeof(Stats) // 8, dtype=torch.int64, device=device)


def read_stats(buf, index: int = 0) -> dict:
    raw = buf.detach().cpu().numpy().view(np.uint8)
    sz = ctypes.sizeof(Stats)
    s = Stats.from_buffer_copy(raw[index * sz:(index + 1) * sz].tobytes())
    pair = np.array(s.pair, dtype=np.uint64).reshape(7, 7)
    return {"pair": pair, "disagree": np.array(s.disagree, dtype=np.uint64),
            "no_majority": int(s.no_majority), "n": int(s.n), "verdict": int(s.verdict),
            "winner": int(s.winner)}


class Context:
    """An ftv context on one device (its workspace, batch tables and graph)."""

    def __init__(self, device: int = 0):
        L = load()
        h = c_void_p()
        _check(L.ftv_ctx_create(int(device), ctypes.byref(h)))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            load().ftv_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- kernel timing -----------------------------------------------------------
    def set_timing(self, on: bool):
        _check(load().ftv_ctx_set_timing(self.handle, int(bool(on))))

    def kernel_times(self):
        """Kernel times (ms) of the launches recorded since timing was turned
        on or last read, in launch order; clears the record."""
        n = c_uint32()
        buf = (ctypes.c_float * 1024)()
        _check(load().ftv_ctx_kernel_times(self.handle, buf, 1024, ctypes.byref(n)))
        return [float(x) for x in buf[:min(n.value, 1024)]]

    # -- batch schedule ---------------------------------------------------------
    def get_batch_config(self) -> BatchCfg:
        c = BatchCfg()
        _check(load().ftv_batch_get_config(self.handle, ctypes.byref(c)))
        return c

    def set_batch_config(self, cfg: BatchCfg):
        _check(load().ftv_batch_set_config(self.handle, ctypes.byref(cfg)))


# ---- argument checks ---------------------------------------------------------
# The C ABI sees only pointers, so this is the one place where a tensor's
# device, type and size can be checked: a short replica, a small output or a
# host tensor passed as device memory would otherwise become an out-of-bounds
# or host-pointer access inside a kernel.  Every public call checks its
# tensors before it allocates anything or calls the library.
def _bad(msg: str):
    raise ValueError(msg)


def _check_tensor(t, name: str, *, device=None, dtype=None, min_numel: int = 0, host_ok: bool = False,
                  min_bytes: int = 0):
    if not t.is_contiguous():
        _bad(f"{name} must be a contiguous tensor")
    if not t.is_cuda and not host_ok:
        _bad(f"{name} must be a CUDA (device) tensor")
    if device is not None and t.is_cuda and t.device != device:
        _bad(f"{name} is on {t.device}, expected {device}")
    if dtype is not None and t.dtype != dtype:
        _bad(f"{name} has dtype {t.dtype}, expected {dtype}")
    if t.numel() < min_numel:
        _bad(f"{name} has {t.numel()} elements, needs at least {min_numel}")
    if t.numel() * t.element_size() < min_bytes:
        _bad(f"{name} has {t.numel() * t.element_size()} bytes, needs at least {min_bytes}")


def _check_replicas(replicas, n=None, host_ok: bool = False):
    """Replicas share one dtype, are device tensors (or host ones where the call
    takes them) on one device, and hold at least n elements each.  Returns
    (n, device of the device replicas or None)."""
    if len(replicas) == 0:
        _bad("no replicas")
    if len(replicas) > MAX_K:
        _bad(f"at most {MAX_K} replicas")
    x0 = replicas[0]
    n = int(x0.numel() if n is None else n)
    if n < 0:
        _bad("n must be >= 0")
    dev = next((r.device for r in replicas if r.is_cuda), None)
    for r, t in enumerate(replicas):
        _check_tensor(t, f"replica {r}", device=dev, dtype=x0.dtype, min_numel=n, host_ok=host_ok)
    return n, dev


def _check_outputs(n: int, dtype, device, consensus=None, mask=None, stats=None):
    import torch
    if consensus is not None:
        _check_tensor(consensus, "consensus", device=device, dtype=dtype, min_numel=n)
    if mask is not None:
        _check_tensor(mask, "mask", device=device, dtype=torch.uint8, min_numel=n)
    if stats is not None:
        _check_tensor(stats, "stats", device=device, min_bytes=ctypes.sizeof(Stats))


def make_desc(replicas, tol: Tol, consensus=None, mask=None, stats=None, n=None, host_ok: bool = False) -> VoteDesc:
    """A checked vote descriptor (see the argument checks above)."""
    n, dev = _check_replicas(replicas, n, host_ok)
    if dev is None and (consensus is not None or mask is not None or stats is not None):
        dev = next(t.device for t in (consensus, mask, stats) if t is not None)
    _check_outputs(n, replicas[0].dtype, dev, consensus, mask, stats)
    d = VoteDesc()
    for r, t in enumerate(replicas):
        d.replicas[r] = t.data_ptr()
    d.k = len(replicas)
    d.dtype = dtype_code(replicas[0])
    d.n = n
    d.tol = tol
    d.consensus = consensus.data_ptr() if consensus is not None else None
    d.mask = mask.data_ptr() if mask is not None else None
    d.stats = stats.data_ptr() if stats is not None else None
    return d


def vote(ctx: Context, replicas, tol: Tol, consensus=None, mask=None, stats=None, stream=None,
         want_consensus: bool = True, want_mask: bool = True):
    """ftv_vote on k device tensors of one dtype; returns (consensus, mask, stats buffer)."""
    n, dev = _check_replicas(replicas)
    _check_outputs(n, replicas[0].dtype, dev, consensus, mask, stats)
    torch = _torch()
    x0 = replicas[0]
    if consensus is None and want_consensus:
        consensus = torch.empty_like(x0)
    if mask is None and want_mask:
        mask = torch.empty(x0.numel(), dtype=torch.uint8, device=x0.device)
    if stats is None:
        stats = stats_tensor(x0.device)
    d = make_desc(replicas, tol, consensus, mask, stats)
    _check(load().ftv_vote(ctx.handle, ctypes.byref(d), c_void_p(_stream_handle(stream))))
    return consensus, mask, stats


def vote_mem(ctx: Context, replicas, tol: Tol, consensus=None, mask=None, stats=None, chunk_bytes: int = 64 << 20,
             stream=None, want_consensus: bool = True, want_mask: bool = True):
    """ftv_vote_mem: replicas are torch tensors in host memory (CPU tensors,
    pinned or not) or on the GPU; outputs are device tensors."""
    n, dev = _check_replicas(replicas, host_ok=True)
    torch = _torch()
    if dev is None:
        dev = torch.device("cuda", torch.cuda.current_device())
    _check_outputs(n, replicas[0].dtype, dev, consensus, mask, stats)
    x0 = replicas[0]
    if consensus is None and want_consensus:
        consensus = torch.empty(x0.numel(), dtype=x0.dtype, device=dev)
    if mask is None and want_mask:
        mask = torch.empty(x0.numel(), dtype=torch.uint8, device=dev)
    if stats is None:
        stats = stats_tensor(dev)
    d = make_desc(replicas, tol, consensus, mask, stats, host_ok=True)
    mem = (ctypes.c_int32 * len(replicas))(*[MEM_DEVICE if r.is_cuda else MEM_HOST for r in replicas])
    _check(load().ftv_vote_mem(ctx.handle, ctypes.byref(d), mem, c_uint64(int(chunk_bytes)),
                               c_void_p(_stream_handle(stream))))
    return consensus, mask, stats


def vote_batch(ctx: Context, descs, stream=None):
    arr = (VoteDesc * len(descs))(*descs)
    _check(load().ftv_vote_batch(ctx.handle, arr, len(descs), c_void_p(_stream_handle(stream))))


def vote_batch_noalloc(descs, stream=None):
    """ftv_vote_batch_noalloc: the batched vote without a context or any
    allocation (at most NOALLOC_MAX_TASKS descriptors), on the current device."""
    arr = (VoteDesc * max(len(descs), 1))(*descs)
    _check(load().ftv_vote_batch_noalloc(arr, len(descs), c_void_p(_stream_handle(stream))))


def tune_batch(ctx: Context, descs, iters: int = 3, stream=None) -> BatchCfg:
    arr = (VoteDesc * len(descs))(*descs)
    best = BatchCfg()
    _check(load().ftv_tune_batch(ctx.handle, arr, len(descs), c_void_p(_stream_handle(stream)),
                                 int(iters), ctypes.byref(best)))
    return best


def fingerprint(ctx: Context, buf, block_bytes: int = 65536, out=None, stream=None):
    _check_tensor(buf, "buffer")
    nbytes = buf.numel() * buf.element_size()
    nblocks = (nbytes + block_bytes - 1) // block_bytes if block_bytes > 0 else 0
    if out is not None:
        _check_tensor(out, "fingerprint output", device=buf.device, min_bytes=8 * nblocks)
    torch = _torch()
    if out is None:
        out = torch.empty(nblocks, dtype=torch.int64, device=buf.device)
    _check(load().ftv_fingerprint(ctx.handle, c_void_p(buf.data_ptr()), nbytes, block_bytes,
                                  c_void_p(out.data_ptr()), c_void_p(_stream_handle(stream))))
    return out


def block_stats_tensor(device):
    torch = _torch()
    return torch.zeros(ctypes.sizeof(BlockStats) // 8, dtype=torch.int64, device=device)


def read_block_stats(buf) -> dict:
    raw = buf.detach().cpu().numpy().view(np.uint8).tobytes()
    s = BlockStats.from_buffer_copy(raw[:ctypes.sizeof(BlockStats)])
    return {"blocks": int(s.blocks), "disagree_blocks": int(s.disagree_blocks),
            "fallback_blocks": int(s.fallback_blocks), "unresolved_elems": int(s.unresolved_elems),
            "replica_blocks": np.array(s.replica_blocks, dtype=np.uint64),
            "verdict": int(s.verdict), "winner": int(s.winner)}


def vote_blocks(ctx: Context, replicas, fallback_tol: Tol, block_bytes: int = 65536,
                want_fps: bool = True, want_mask: bool = True, consensus=None, mask=None,
                blockmap=None, fps=None, bstats=None, stream=None):
    """ftv_vote_blocks; returns dict of device tensors (fps, blockmap, consensus, mask, bstats)."""
    n, dev = _check_replicas(replicas)
    x0 = replicas[0]
    k = len(replicas)
    nbytes = n * x0.element_size()
    nblocks = (nbytes + block_bytes - 1) // block_bytes if block_bytes > 0 else 0
    _check_outputs(n, x0.dtype, dev, consensus, mask)
    if fps is not None:
        _check_tensor(fps, "fps", device=dev, min_bytes=8 * k * nblocks)
    if blockmap is not None:
        _check_tensor(blockmap, "blockmap", device=dev, min_bytes=nblocks)
    if bstats is not None:
        _check_tensor(bstats, "bstats", device=dev, min_bytes=ctypes.sizeof(BlockStats))
    torch = _torch()
    if fps is None and want_fps:
        fps = torch.empty(k * nblocks, dtype=torch.int64, device=dev)
    if blockmap is None:
        blockmap = torch.empty(max(nblocks, 1), dtype=torch.uint8, device=dev)
    if consensus is None:
        consensus = torch.empty_like(x0)
    if mask is None and want_mask:
        mask = torch.empty(x0.numel(), dtype=torch.uint8, device=dev)
    if bstats is None:
        bstats = block_stats_tensor(dev)
    ptrs = (c_void_p * k)(*[t.data_ptr() for t in replicas])
    tol = fallback_tol
    _check(load().ftv_vote_blocks(
        ctx.handle, ptrs, k, dtype_code(x0), nbytes, block_bytes, ctypes.byref(tol),
        c_void_p(fps.data_ptr()) if fps is not None else None, c_void_p(blockmap.data_ptr()),
        c_void_p(consensus.data_ptr()), c_void_p(mask.data_ptr()) if mask is not None else None,
        c_void_p(bstats.data_ptr()), c_void_p(_stream_handle(stream))))
    return {"fps": fps, "blockmap": blockmap[:nblocks], "consensus": consensus, "mask": mask,
            "bstats": bstats}


# ---- serving ---------------------------------------------------------------
class Server:
    """Continuous-batching voter service (ftv_server_*)."""

    def __init__(self, hbm_budget_bytes: int, arena_bytes: int = 0, chunk_bytes: int = 32 << 20,
                 max_slots: int = 1024, max_queue: int = 1 << 20, device: int = 0):
        L = load()
        cfg = ServerCfg(int(hbm_budget_bytes), int(arena_bytes), int(chunk_bytes), int(max_slots),
                        int(max_queue), int(device), 0)
        h = c_void_p()
        _check(L.ftv_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self._events = {}   # ticket -> the ready event, kept until release

    def submit(self, req: Request, ready_event=None) -> int:
        t = c_uint64()
        _check(load().ftv_submit(self.handle, ctypes.byref(req), ctypes.byref(t)))
        if ready_event is not None:
            self._events[int(t.value)] = ready_event
        return int(t.value)

    def _ready(self, req: Request, stream):
        """Record an event after the work queued so far on `stream` (torch's
        current stream by default), which produces the request's inputs."""
        torch = _torch()
        ev = torch.cuda.Event()
        ev.record(stream if stream is not None else torch.cuda.current_stream())
        req.ready = ev.cuda_event
        return ev

    @staticmethod
    def vote_request(replicas, tol: Tol, consensus=None, mask=None, n=None, user_tag: int = 0) -> Request:
        """A checked vote request (inputs complete, no ready event), to be
        passed to submit() later -- e.g. prepared before the request is due."""
        req = Request()
        req.kind = REQ_VOTE
        req.vote = make_desc(replicas, tol, consensus, mask, None, n=n)
        req.user_tag = int(user_tag)
        return req

    def submit_vote(self, replicas, tol: Tol, consensus=None, mask=None, t_arrival_ns: int = 0,
                    user_tag: int = 0, n=None, stream=None, inputs_ready: bool = False) -> int:
        """inputs_ready: the replicas are complete already (no event is passed)."""
        req = self.vote_request(replicas, tol, consensus, mask, n=n, user_tag=user_tag)
        req.t_arrival_ns = int(t_arrival_ns)
        ev = None if inputs_ready else self._ready(req, stream)
        return self.submit(req, ev)

    def submit_fingerprint(self, buf, block_bytes: int = 65536, t_arrival_ns: int = 0,
                           user_tag: int = 0, stream=None, inputs_ready: bool = False) -> int:
        _check_tensor(buf, "buffer")
        req = Request()
        req.kind = REQ_FINGERPRINT
        req.fp_buf = buf.data_ptr()
        req.fp_bytes = buf.numel() * buf.element_size()
        req.block_bytes = int(block_bytes)
        req.t_arrival_ns = int(t_arrival_ns)
        req.user_tag = int(user_tag)
        ev = None if inputs_ready else self._ready(req, stream)
        return self.submit(req, ev)

    def poll(self, ticket: int, wait_us: int = -1):
        """Result structure when done, None while in flight."""
        res = Result()
        rc = load().ftv_poll(self.handle, int(ticket), ctypes.byref(res), int(wait_us))
        if rc == E_NOTREADY:
            return None
        _check(rc)
        return res

    def release(self, ticket: int):
        _check(load().ftv_release(self.handle, int(ticket)))
        self._events.pop(int(ticket), None)

    def stats(self) -> dict:
        st = ServerStats()
        _check(load().ftv_server_get_stats(self.handle, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in ServerStats._fields_}

    def close(self):
        if self.handle:
            load().ftv_server_destroy(self.handle)
            self.handle = None
            self._events.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def result_stats(res: Result) -> dict:
    s = res.stats
    return {"pair": np.array(s.pair, dtype=np.uint64).reshape(7, 7),
            "disagree": np.array(s.disagree, dtype=np.uint64), "no_majority": int(s.no_majority),
            "n": int(s.n), "verdict": int(s.verdict), "winner": int(s.winner)}


# ---- fault-aware runtime estimation ------------------------------------------
def fault_aware_runtime(unit: Unit) -> float:
    return float(load().ftv_fault_aware_runtime(ctypes.byref(unit)))


def rank_units(units, probe: bool = False):
    arr = (Unit * len(units))(*units)
    order = (c_uint32 * len(units))()
    _check(load().ftv_rank_units(arr, len(units), int(probe), order))
    return list(order)


def record_vote(units, unit_of_replica, stats: Stats):
    """units: a ctypes array of Unit (updated in place); stats: a host Stats."""
    k = len(unit_of_replica)
    u = (c_uint32 * k)(*unit_of_replica)
    _check(load().ftv_record_vote(units, len(units), u, k, ctypes.byref(stats)))


# ---- memory areas with siblings and versions ----------------------------------
MEM_HOST, MEM_DEVICE = 0, 1
ACC_READ, ACC_WRITE, ACC_READWRITE = 1, 2, 3


class MemoryManager:
    """Siblings and versions of registered host areas (the C calls ftv_mm_*).
    device = -1 makes a host-only manager (no HIP call)."""

    def __init__(self, device: int = 0, fault_tolerant: bool = True):
        h = c_void_p()
        _check(load().ftv_mm_create(int(device), int(bool(fault_tolerant)), ctypes.byref(h)))
        self.handle = h
        self.device = int(device)
        self._held = []   # registered host buffers stay alive with the manager

    def _stream(self, stream) -> int:
        # a host-only manager makes no HIP call: it needs no stream (and no GPU)
        if stream is None and self.device < 0:
            return 0
        return _stream_handle(stream)

    def register(self, host_array) -> int:
        """Register a C-contiguous numpy array (the caller's area, sibling 0)."""
        if not host_array.flags["C_CONTIGUOUS"]:
            raise ValueError("the area must be C-contiguous")
        self._held.append(host_array)
        a = c_uint32()
        _check(load().ftv_mm_register(self.handle, c_void_p(host_array.ctypes.data), host_array.nbytes,
                                      ctypes.byref(a)))
        return int(a.value)

    def request(self, area: int, memory: int, access: int, stream=None):
        """-> (address, sibling index)."""
        p, sib = c_void_p(), c_uint32()
        _check(load().ftv_mm_request(self.handle, area, memory, access,
                                     c_void_p(self._stream(stream)), ctypes.byref(p),
                                     ctypes.byref(sib)))
        return int(p.value or 0), int(sib.value)

    def release(self, area: int, sibling: int, ok: bool = True):
        _check(load().ftv_mm_release(self.handle, area, sibling, int(bool(ok))))

    def siblings(self, area: int):
        n = c_uint32()
        _check(load().ftv_mm_siblings(self.handle, area, None, 0, ctypes.byref(n)))
        arr = (SiblingInfo * max(1, n.value))()
        _check(load().ftv_mm_siblings(self.handle, area, arr, n.value, ctypes.byref(n)))
        return [{"ptr": int(s.ptr or 0), "memory": int(s.memory), "valid": bool(s.valid),
                 "version": int(s.version), "readers": int(s.readers), "writing": bool(s.writing),
                 "caller": bool(s.caller)} for s in arr[:n.value]]

    def check(self, area: int, block_bytes: int = 65536, stream=None) -> dict:
        r = MMCheckResult()
        _check(load().ftv_mm_check(self.handle, area, block_bytes, c_void_p(self._stream(stream)),
                                   ctypes.byref(r)))
        return {"checked": int(r.checked), "invalidated": int(r.invalidated),
                "unresolved": int(r.unresolved), "blocks": int(r.blocks)}

    def close(self):
        if self.handle:
            load().ftv_mm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- the voter on the host's cores and its placement -------------------------
def _stats_dict(s: Stats) -> dict:
    return {"pair": np.array(s.pair, dtype=np.uint64).reshape(7, 7),
            "disagree": np.array(s.disagree, dtype=np.uint64), "no_majority": int(s.no_majority),
            "n": int(s.n), "verdict": int(s.verdict), "winner": int(s.winner)}


def vote_host(replicas, tol: Tol, threads: int = 1, want_consensus: bool = True, want_mask: bool = True,
              consensus=None, mask=None):
    """ftv_vote_host on k C-contiguous numpy arrays of one dtype (host memory);
    returns (consensus, mask, stats dict).  threads: 1 = one thread, 0 = every core.
    consensus / mask: caller arrays to write; otherwise new arrays when wanted."""
    if not 1 <= len(replicas) <= MAX_K:
        _bad(f"1 to {MAX_K} replicas")
    x0 = replicas[0]
    codes = {np.dtype(np.float32): F32, np.dtype(np.float64): F64, np.dtype(np.int32): I32,
             np.dtype(np.int64): I64}
    if x0.dtype not in codes:
        _bad(f"unsupported dtype {x0.dtype}")
    n = x0.size
    for r, a in enumerate(replicas):
        if not isinstance(a, np.ndarray) or not a.flags["C_CONTIGUOUS"]:
            _bad(f"replica {r} must be a C-contiguous numpy array")
        if a.dtype != x0.dtype or a.size < n:
            _bad(f"replica {r} must have dtype {x0.dtype} and at least {n} elements")
    for name, a, dt in (("consensus", consensus, x0.dtype), ("mask", mask, np.dtype(np.uint8))):
        if a is not None and (not isinstance(a, np.ndarray) or not a.flags["C_CONTIGUOUS"] or a.dtype != dt
                              or a.size < n or not a.flags["WRITEABLE"]):
            _bad(f"{name} must be a writeable C-contiguous numpy array of {dt} with at least {n} elements")
    cons = consensus if consensus is not None else (np.empty(n, dtype=x0.dtype) if want_consensus else None)
    mask = mask if mask is not None else (np.empty(n, dtype=np.uint8) if want_mask else None)
    st = Stats()
    d = VoteDesc()
    for r, a in enumerate(replicas):
        d.replicas[r] = a.ctypes.data
    d.k, d.dtype, d.n, d.tol = len(replicas), codes[x0.dtype], n, tol
    d.consensus = cons.ctypes.data if cons is not None else None
    d.mask = mask.ctypes.data if mask is not None else None
    d.stats = ctypes.addressof(st)
    _check(load().ftv_vote_host(ctypes.byref(d), int(threads)))
    return cons, mask, _stats_dict(st)


class VoterDB:
    """Performance database of the voter units (the C calls ftv_voter_db_*)."""

    def __init__(self, check_interval: int = 8, host_threads: int = 0):
        h = c_void_p()
        _check(load().ftv_voter_db_create(int(check_interval), int(host_threads), ctypes.byref(h)))
        self.handle = h

    def profile(self, unit: int, nbytes: int, host_mask: int, out_memory: int) -> Unit:
        u = Unit()
        _check(load().ftv_voter_db_profile(self.handle, int(unit), int(nbytes), int(host_mask),
                                           int(out_memory), ctypes.byref(u)))
        return u

    def inject(self, unit: int, count: int):
        _check(load().ftv_voter_db_inject(self.handle, int(unit), int(count)))

    def close(self):
        if self.handle:
            load().ftv_voter_db_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def vote_placed(ctx: Context, db: VoterDB, replicas, tol: Tol, out_memory: int = MEM_DEVICE, consensus=None,
                mask=None, stats=None, avoid: int = 0, redundant: bool = False, stream=None,
                want_consensus: bool = True, want_mask: bool = True):
    """ftv_vote_placed: replicas are torch tensors in host memory (CPU) or on the
    GPU; outputs lie in out_memory.  Returns (consensus, mask, stats, report)."""
    torch = _torch()
    for name, t in (("consensus", consensus), ("mask", mask), ("stats", stats)):
        if t is not None and t.is_cuda != (out_memory == MEM_DEVICE):
            _bad(f"{name} must lie in out_memory")
    n, dev = _check_replicas(replicas, host_ok=True)
    if dev is None:
        dev = torch.device("cuda", torch.cuda.current_device())
    odev = dev if out_memory == MEM_DEVICE else torch.device("cpu")
    x0 = replicas[0]
    if consensus is not None:
        _check_tensor(consensus, "consensus", device=dev if odev.type == "cuda" else None, dtype=x0.dtype,
                      min_numel=n, host_ok=True)
    if mask is not None:
        _check_tensor(mask, "mask", device=dev if odev.type == "cuda" else None, dtype=torch.uint8, min_numel=n,
                      host_ok=True)
    if stats is not None:
        _check_tensor(stats, "stats", device=dev if odev.type == "cuda" else None,
                      min_bytes=ctypes.sizeof(Stats), host_ok=True)
    if consensus is None and want_consensus:
        consensus = torch.empty(n, dtype=x0.dtype, device=odev)
    if mask is None and want_mask:
        mask = torch.empty(n, dtype=torch.uint8, device=odev)
    if stats is None:
        stats = torch.zeros(ctypes.sizeof(Stats) // 8, dtype=torch.int64, device=odev)
    d = make_desc(replicas, tol, n=n, host_ok=True)
    d.consensus = consensus.data_ptr() if consensus is not None else None
    d.mask = mask.data_ptr() if mask is not None else None
    d.stats = stats.data_ptr()
    mem = (c_int32 * len(replicas))(*[MEM_DEVICE if r.is_cuda else MEM_HOST for r in replicas])
    rep = PlaceReport()
    _check(load().ftv_vote_placed(ctx.handle, db.handle, ctypes.byref(d), mem, int(out_memory), int(avoid),
                                  PLACE_REDUNDANT if redundant else 0, c_void_p(_stream_handle(stream)),
                                  ctypes.byref(rep)))
    report = {"units": [int(u) for u in rep.unit[:rep.runs]], "result_unit": int(rep.result_unit),
              "agreed": bool(rep.agreed), "probed": bool(rep.probed),
              "seconds": [float(x) for x in rep.seconds[:rep.runs]]}
    return consensus, mask, stats, report


# ---- redundant execution with timeouts and retries ----------------------------
def run_redundant(ctx: Context, impls, units, out, tol: Tol, k: int = 2, max_attempts: int = 3,
                  timeout_factor: float = 0.0, check_interval: int = 0) -> dict:
    """impls: list of (fn, unit) where fn(out_ptr: int, stream_ptr: int) -> int
    enqueues the task into the device buffer at out_ptr on the HIP stream
    stream_ptr and returns 0 (non-zero: a direct fault).  units: a ctypes array
    of Unit (updated in place).  out: the device tensor for the consensus."""
    keep = []

    def wrap(fn):
        def cb(_user, out_ptr, stream_ptr):
            try:
                return int(fn(int(out_ptr or 0), int(stream_ptr or 0)))
            except Exception:
                return -1
        c = TaskFn(cb)
        keep.append(c)
        return c
    arr = (Impl * len(impls))(*[Impl(wrap(fn), None, int(u), 0) for fn, u in impls])
    cfg = RedundancyCfg(int(k), int(max_attempts), float(timeout_factor), dtype_code(out), int(check_interval), tol)
    rep = RedundancyReport()
    _check(load().ftv_run_redundant(ctx.handle, arr, len(impls), units, len(units),
                                    ctypes.byref(cfg), out.numel(), c_void_p(out.data_ptr()),
                                    ctypes.byref(rep)))
    return {"attempts": int(rep.attempts), "verdict": int(rep.verdict), "timeouts": int(rep.timeouts),
            "errors": int(rep.errors), "winner_unit": int(rep.winner_unit), "seconds": float(rep.seconds)}
