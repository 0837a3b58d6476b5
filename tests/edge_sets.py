"""Replica sets whose elements sit on the edges of the tolerance decisions
(Sec. IV-D: integers bit-wise, floating point within a tolerance), shared by
the GPU and the host-voter parity tests.

The replicas of an element lie 0, 1, m-1, m, m+1 or 2m+1 ordered-key steps
from a base value (m = the ULP tolerance), so that each pair is just inside
or just outside the tolerance, with base values at +-0, the denormal range,
the smallest normal, +-max, +-inf and NaNs, where the steps cross zero, leave
the finite range or enter the NaN keys; or at relative distances of a
fraction (just below 1, 1, just above 1) of the relative delta; or split into
two equal-sized groups (ties, no strict majority).  The sets hold no voting
arithmetic: only the construction of the inputs.
"""
import numpy as np

U = {np.dtype(np.float32): np.uint32, np.dtype(np.float64): np.uint64}


def step_keys(x: np.ndarray, d: np.ndarray) -> np.ndarray:
    """x moved by d steps of the IEEE totalOrder key (saturating at both
    ends of the key range), computed on the bits."""
    u = U[x.dtype]
    nb = 8 * x.itemsize
    sign = u(1) << u(nb - 1)
    top = np.iinfo(u).max
    bits = x.view(u)
    key = np.where(bits & sign, ~bits, bits | sign).astype(u)
    dd = np.abs(d).astype(u)
    up = np.where(key <= top - dd, key + dd, top)
    down = np.where(key >= dd, key - dd, u(0))
    key2 = np.where(d >= 0, up, down).astype(u)
    out = np.where(key2 & sign, key2 & ~sign, ~key2).astype(u)
    return out.view(x.dtype)


def specials(dtype):
    f = np.finfo(dtype)
    u = U[np.dtype(dtype)]
    nan_payload = np.array([(u(0x7fc00123) if dtype == np.float32 else u(0x7ff8000000000123))], dtype=u).view(dtype)[0]
    return np.array([0.0, -0.0, f.smallest_subnormal, -f.smallest_subnormal, f.smallest_normal - f.smallest_subnormal,
                     f.smallest_normal, -f.smallest_normal, 1.0, -1.0, f.max, -f.max, np.inf, -np.inf, np.nan,
                     -np.nan, nan_payload], dtype=dtype)


def boundary_set(rng, dtype, k, n, m, delta, anchored=False):
    """k replicas of n elements on the edges of a ULP tolerance m and of a
    relative tolerance delta (see the module docstring).  Anchored: for each
    element a random k//2 + 1 of the replicas hold the base value itself and
    there are no tie splits, so every element has a strict majority and only
    the other replicas sit on the edges."""
    dtype = np.dtype(dtype)
    sp = specials(dtype)
    # 0, 1: ULP edges, 2: relative edges, 3: tie split (in every other set)
    kind = rng.integers(0, 4 if rng.random() < 0.5 and not anchored else 3, n)
    base = (rng.standard_normal(n) * 10.0 ** rng.integers(-20, 21, n)).astype(dtype)
    at_special = rng.random(n) < 0.35
    base[at_special] = sp[rng.integers(0, sp.size, int(at_special.sum()))]
    offs = np.array([0, 1, -1, m - 1, -(m - 1), m, -m, m + 1, -(m + 1), 2 * m + 1, -(2 * m + 1)], dtype=np.int64)
    reps = []
    # relative edges: base * (1 + s * delta * f), f just below 1, 1, just above 1, in fp64 then rounded
    fr = np.array([0.0, 0.5, 1.0 - 2.0 ** -30, 1.0, 1.0 + 2.0 ** -30, 2.0])
    b64 = base.astype(np.float64)
    other = step_keys(base, np.full(n, m + 1 + int(rng.integers(0, 3)), dtype=np.int64))
    split = rng.random(n) < 0.5
    rank = np.argsort(np.argsort(rng.random((k, n)), axis=0), axis=0)   # per element, a random order of replicas
    for r in range(k):
        d = offs[rng.integers(0, offs.size, n)]
        x = step_keys(base, d)
        s = np.where(rng.random(n) < 0.5, -1.0, 1.0)
        with np.errstate(over="ignore", invalid="ignore"):
            rel = (b64 * (1.0 + s * delta * fr[rng.integers(0, fr.size, n)])).astype(dtype)
        x = np.where(kind == 2, rel, x)
        # tie split: the first half of the replicas hold base, the rest `other`
        # (or the halves swapped), so no value has a strict majority for even k
        first = r < k // 2
        x = np.where(kind == 3, np.where(first ^ split, base, other), x)
        if anchored:
            x = np.where(rank[r] <= k // 2, base, x)
        reps.append(np.ascontiguousarray(x.astype(dtype)))
    return reps
