"""Device twin of the seeded replica generator (``ftv_synth.hip``).

Builds the large replica sets directly in HBM with the same definitions as
the numpy generator in ``synth/__init__.py`` (checked element for element by
the tests).  Sparse fault plans (positions, bits, the zeroed block) are drawn
on the host with the numpy generator and applied with torch indexing.
"""
from __future__ import annotations

import ctypes
import os
import shutil
import subprocess

import numpy as np

from . import (INTFULL, NORMAL, SEED_BASE, UNIFORM, distinct_positions, flip_plan,  # noqa: F401
               rand_u64)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ftv_synth.hip")
_LIB = os.path.join(_HERE, "libftv_synth.so")
_DT = {"f32": 0, "f64": 1, "i32": 2, "i64": 3}


def build() -> str:
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    tmp = _LIB + ".tmp"
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
                           "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise RuntimeError(f"{_LIB} missing: run synth.device.build()")
        L = ctypes.CDLL(_LIB)
        u64, vp, ci = ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int
        L.ftvs_fill.argtypes = [vp, u64, ci, ci, u64, u64, u64, vp]
        L.ftvs_fill.restype = ci
        L.ftvs_ulp_noise.argtypes = [vp, u64, ci, u64, u64, ctypes.c_uint32, ctypes.c_uint32, vp]
        L.ftvs_ulp_noise.restype = ci
        _lib = L
    return _lib


def _stream():
    import torch
    return ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream))


def fill(t, dtype: str, dist: int, seed: int, stream: int, offset: int = 0):
    rc = lib().ftvs_fill(ctypes.c_void_p(t.data_ptr()), t.numel(), _DT[dtype], dist,
                         seed & (2 ** 64 - 1), stream & (2 ** 64 - 1), offset, _stream())
    if rc:
        raise RuntimeError(f"ftvs_fill failed ({rc})")
    return t


def ulp_noise(t, dtype: str, seed: int, stream: int, thresh24: int, maxd: int):
    rc = lib().ftvs_ulp_noise(ctypes.c_void_p(t.data_ptr()), t.numel(), _DT[dtype],
                              seed & (2 ** 64 - 1), stream & (2 ** 64 - 1), thresh24, maxd,
                              _stream())
    if rc:
        raise RuntimeError(f"ftvs_ulp_noise failed ({rc})")
    return t


def _torch_dtype(dtype: str):
    import torch
    return {"f32": torch.float32, "f64": torch.float64, "i32": torch.int32, "i64": torch.int64}[dtype]


def _int_view(t):
    import torch
    return t.view(torch.int32 if t.element_size() == 4 else torch.int64)


def flip_bits(t, pos: np.ndarray, bits: np.ndarray):
    import torch
    iv = _int_view(t)
    p = torch.as_tensor(pos.astype(np.int64), device=t.device)
    one = torch.ones(len(pos), dtype=iv.dtype, device=t.device)
    masks = torch.bitwise_left_shift(one, torch.as_tensor(bits.astype(np.int64), device=t.device).to(iv.dtype))
    iv[p] = torch.bitwise_xor(iv[p], masks)


def large_task_set(n: int, dtype: str = "f32", seed: int = SEED_BASE + 2, device="cuda",
            flip_rate: float = 1e-7):
    """Device version of synth.large_task_set (same values, same faults)."""
    import torch
    td = _torch_dtype(dtype)
    base = torch.empty(n, dtype=td, device=device)
    fill(base, dtype, NORMAL, seed, 0)
    r1 = base.clone()
    ulp_noise(r1, dtype, seed, 1, round(0.30 * (1 << 24)), 1)
    r2 = base.clone()
    es = base.element_size()
    zb = 4096 // es
    nzb = max(1, n // zb)
    b = int(rand_u64(seed, 3, 0) % np.uint64(nzb))
    r2[b * zb:min(n, (b + 1) * zb)] = 0
    nflip = max(1, int(round(flip_rate * n)))
    pos, bits = flip_plan(n, nflip, 8 * es, seed, 2)
    flip_bits(r2, pos, bits)
    return [base, r1, r2]


def checkpoint_set(n: int, seed: int = SEED_BASE + 5, device="cuda", nstuck: int = 256, nflip=None,
            flip_rate: float = 1e-7):
    """Device version of synth.checkpoint_set."""
    import torch
    base = torch.empty(n, dtype=torch.float64, device=device)
    fill(base, "f64", NORMAL, seed, 0)
    r1 = base.clone()
    sp = distinct_positions(n, min(nstuck, n), seed, 1).astype(np.int64)
    r1[torch.as_tensor(sp, device=device)] = 0.0
    r2 = base.clone()
    nf = nflip if nflip is not None else max(1, int(round(flip_rate * n)))
    pos, bits = flip_plan(n, nf, 64, seed, 2)
    flip_bits(r2, pos, bits)
    r3 = torch.roll(base, 1)
    return [base, r1, r2, r3, base.clone()]
