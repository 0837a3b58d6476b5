"""Seeded synthetic replica sets and fault injectors.

This module is shared by the tests, the benchmark and the smoke check.  It
holds no part of the voter's arithmetic: it only produces inputs -- base values,
rounding-diversity noise and injected faults -- for the replicas of duplicated
task runs.

All randomness comes from one counter-based generator (the SplitMix64 output
function of Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) applied to (seed, stream, index), so that a value can
be recomputed anywhere: on the host here with numpy, or on the device by the
HIP twin in ``ftv_synth.hip`` (same definition, checked against this one).

Value recipes (every conversion exact or a single IEEE round-to-nearest-even):
  * ``uniform``: U[-1, 1) with 24 (fp32) or 53 (fp64) random bits;
  * ``normal``: Irwin-Hall sum of 12 U[0,1) minus 6 (mean 0, variance 1, the
    classic stand-in for N(0,1)), plus 24 extra low random bits;
  * ``intfull``: uniform over the whole int32 / int64 range.
Fault models: +-d ULP (magnitude step) noise on a hashed subset of elements;
single-bit flips at distinct positions; zeroed (stuck-at-0) elements or words;
a replica rotated by one element.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 14052912

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_STREAM_SALT = np.uint64(0x632BE59BD9B4E019)

UNIFORM, NORMAL, INTFULL = 0, 1, 2

_np = {"f32": np.float32, "f64": np.float64, "i32": np.int32, "i64": np.int64}
_u = {"f32": np.uint32, "f64": np.uint64, "i32": np.uint32, "i64": np.uint64}


def _mix(z):
    """SplitMix64 finaliser (wrapping uint64 arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        s = _mix(np.uint64(stream & 0xFFFFFFFFFFFFFFFF) + _STREAM_SALT)
        return np.uint64(_mix(np.uint64(seed & 0xFFFFFFFFFFFFFFFF) ^ s))


def rand_u64(seed: int, stream: int, idx) -> np.ndarray:
    """Output idx of stream `stream` under `seed`: mix(key + (idx+1)*GAMMA)."""
    idx = np.asarray(idx, dtype=np.uint64)
    key = stream_key(seed, stream)
    with np.errstate(over="ignore"):
        return _mix(key + (idx + np.uint64(1)) * GAMMA)


def values(dtype: str, dist: int, seed: int, stream: int, n: int, offset: int = 0) -> np.ndarray:
    """n values of the given recipe, elements offset..offset+n-1 of the stream."""
    i = np.arange(offset, offset + n, dtype=np.uint64)
    if dist == INTFULL:
        r = rand_u64(seed, stream, i)
        if dtype == "i32":
            return (r >> np.uint64(32)).astype(np.uint32).view(np.int32)
        return r.view(np.int64)
    if dist == UNIFORM:
        r = rand_u64(seed, stream, i)
        if dtype == "f32":
            m = (r >> np.uint64(40)).astype(np.float64)
            return (m * 2.0 ** -23 - 1.0).astype(np.float32)
        m = (r >> np.uint64(11)).astype(np.float64)
        return m * 2.0 ** -52 - 1.0
    if dist == NORMAL:
        # 13 draws per element: indices 13*i .. 13*i+12 of the stream
        base = i * np.uint64(13)
        acc = np.zeros(n, dtype=np.uint64)
        for j in range(12):
            acc += rand_u64(seed, stream, base + np.uint64(j)) >> np.uint64(40)
        extra = rand_u64(seed, stream, base + np.uint64(12)) >> np.uint64(40)
        integer = (acc << np.uint64(24)) + extra          # < 2^52, exact
        x = integer.astype(np.float64) * 2.0 ** -48 - 6.0  # exact in binary64
        return x.astype(np.float32) if dtype == "f32" else x
    raise ValueError(dist)


def ulp_noise(a: np.ndarray, seed: int, stream: int, thresh24: int, maxd: int) -> np.ndarray:
    """In place: element i is perturbed iff (r_i >> 40) < thresh24, by a magnitude
    step of d = 1 + ((r_i >> 1) % maxd) ULP, away from zero if bit 0 of r_i is set
    (or if the magnitude is smaller than d), else toward zero.  Returns the
    perturbed indices."""
    u = a.view(np.uint32 if a.dtype == np.float32 else np.uint64)
    n = a.size
    r = rand_u64(seed, stream, np.arange(n, dtype=np.uint64))
    hit = np.nonzero((r >> np.uint64(40)) < np.uint64(thresh24))[0]
    if hit.size == 0:
        return hit
    rh = r[hit]
    d = np.uint64(1) + ((rh >> np.uint64(1)) % np.uint64(maxd))
    up = (rh & np.uint64(1)) == np.uint64(1)
    if a.dtype == np.float32:
        sign = u[hit] & np.uint32(0x80000000)
        mag = (u[hit] & np.uint32(0x7FFFFFFF)).astype(np.uint64)
        up = up | (mag < d)
        mag = np.where(up, mag + d, mag - d)
        u[hit] = sign | mag.astype(np.uint32)
    else:
        sign = u[hit] & np.uint64(0x8000000000000000)
        mag = u[hit] & np.uint64(0x7FFFFFFFFFFFFFFF)
        up = up | (mag < d)
        mag = np.where(up, mag + d, mag - d)
        u[hit] = sign | mag
    return hit


def distinct_positions(n: int, count: int, seed: int, stream: int) -> np.ndarray:
    """`count` distinct indices in [0, n): candidates rand % n in stream order,
    duplicates skipped."""
    if count > n:
        raise ValueError("more positions than elements")
    out, seen, j = [], set(), 0
    while len(out) < count:
        batch = rand_u64(seed, stream, np.arange(j, j + 2 * count + 8, dtype=np.uint64))
        j += 2 * count + 8
        for v in (batch % np.uint64(n)).tolist():
            if v not in seen:
                seen.add(v)
                out.append(v)
                if len(out) == count:
                    break
    return np.array(out, dtype=np.uint64)


def flip_plan(n: int, count: int, width: int, seed: int, stream: int):
    """Distinct positions and one bit index in [0, width) for each."""
    pos = distinct_positions(n, count, seed, stream)
    bits = (rand_u64(seed, stream ^ 0x5A5A, np.arange(count, dtype=np.uint64))
            % np.uint64(width)).astype(np.uint32)
    return pos, bits


def flip_bits(a: np.ndarray, pos: np.ndarray, bits: np.ndarray) -> None:
    u = a.view(np.uint32 if a.itemsize == 4 else np.uint64)
    one = np.uint32(1) if a.itemsize == 4 else np.uint64(1)
    shift = bits.astype(u.dtype)
    u[pos.astype(np.int64)] ^= (one << shift)


# --------------------------------------------------------------------------
# replica-set recipes at host scale (the device twin builds the large ones)
# --------------------------------------------------------------------------
def small_task_set(n: int = 1 << 20, seed: int = SEED_BASE + 1):
    """k=3 fp32: replica 1 has +-1..2 ULP on 10% of elements, replica 2 has 16
    single-bit flips.  Tolerance 4 ULP."""
    base = values("f32", UNIFORM, seed, 0, n)
    r1 = base.copy()
    ulp_noise(r1, seed, 1, round(0.10 * (1 << 24)), 2)
    r2 = base.copy()
    pos, bits = flip_plan(n, min(16, n), 32, seed, 2)
    flip_bits(r2, pos, bits)
    return [base, r1, r2]


def large_task_set(n: int, dtype: str = "f32", seed: int = SEED_BASE + 2, flip_rate: float = 1e-7,
            zero_block_elems: int = None):
    """k=3: replica 1 has +-1 ULP on 30%; replica 2 has one 4 KiB block set to
    +0 and round(rate*n) single-bit flips."""
    base = values(dtype, NORMAL, seed, 0, n)
    r1 = base.copy()
    ulp_noise(r1, seed, 1, round(0.30 * (1 << 24)), 1)
    r2 = base.copy()
    es = base.itemsize
    zb = zero_block_elems if zero_block_elems is not None else 4096 // es
    nzb = max(1, n // zb)
    b = int(rand_u64(seed, 3, 0) % np.uint64(nzb))
    r2[b * zb:min(n, (b + 1) * zb)] = 0
    nflip = max(1, int(round(flip_rate * n)))
    pos, bits = flip_plan(n, nflip, 8 * es, seed, 2)
    flip_bits(r2, pos, bits)
    return [base, r1, r2]


def checkpoint_set(n: int, seed: int = SEED_BASE + 5, nstuck: int = 256, nflip: int = None,
            flip_rate: float = 1e-7):
    """k=5 fp64 checkpoint: r0, r4 clean; r1 with stuck-at-0 words; r2 with bit
    flips; r3 rotated right by one element."""
    base = values("f64", NORMAL, seed, 0, n)
    r1 = base.copy()
    r1[distinct_positions(n, min(nstuck, n), seed, 1).astype(np.int64)] = 0.0
    r2 = base.copy()
    nf = nflip if nflip is not None else max(1, int(round(flip_rate * n)))
    pos, bits = flip_plan(n, nf, 64, seed, 2)
    flip_bits(r2, pos, bits)
    r3 = np.roll(base, 1)
    return [base, r1, r2, r3, base.copy()]


# --------------------------------------------------------------------------
# planted fault patterns (exact fault counts per replica, for winner cases)
# --------------------------------------------------------------------------
_WIDTH = {"f32": 32, "f64": 64, "i32": 32, "i64": 64}


def _far_bit(dtype: str) -> int:
    # an exponent bit for floats (values of U[-1,1) stay finite), a high bit for integers
    return 30 if _WIDTH[dtype] == 32 else 62


def _split_bit(dtype: str, r: int) -> int:
    # replica r's own bit for elements where every replica holds another value
    return (20 if _WIDTH[dtype] == 32 else 49) + r


def planted_set(dtype: str, n: int, per_replica, nomaj: int = 0, seed: int = SEED_BASE + 7):
    """k = len(per_replica) replicas of one base of n elements.  Replica r is
    changed at per_replica[r] positions of its own (no position is shared by two
    replicas, so all other replicas agree there), and `nomaj` further positions
    hold a different value in every replica.  Returns (base, replicas)."""
    k = len(per_replica)
    base = values(dtype, INTFULL if dtype[0] == "i" else UNIFORM, seed, 0, n)
    pos = distinct_positions(n, int(sum(per_replica)) + nomaj, seed, 1).astype(np.int64)
    reps = [base.copy() for _ in range(k)]
    one = _u[dtype](1)
    off = 0
    for r, c in enumerate(per_replica):
        reps[r].view(_u[dtype])[pos[off:off + c]] ^= one << _u[dtype](_far_bit(dtype))
        off += c
    for r in range(k):
        reps[r].view(_u[dtype])[pos[off:]] ^= one << _u[dtype](_split_bit(dtype, r))
    return base, reps


def planted_blocks(dtype: str, nblocks: int, block_bytes: int, per_replica, unresolved_block: bool = False,
                   tail_elems: int = 0, seed: int = SEED_BASE + 8):
    """k = len(per_replica) replicas of nblocks blocks (+ tail_elems elements).
    Replica r has one changed word in per_replica[r] whole blocks of its own (no
    block is changed in two replicas).  With unresolved_block, one further block
    has element 5 set to a different value in every replica.  Returns (base,
    replicas, that block's index or -1)."""
    k = len(per_replica)
    es = _WIDTH[dtype] // 8
    per = block_bytes // es
    n = nblocks * per + tail_elems
    base = values(dtype, INTFULL if dtype[0] == "i" else UNIFORM, seed, 0, n)
    need = int(sum(per_replica)) + int(unresolved_block)
    blocks = distinct_positions(nblocks, need, seed, 1).astype(np.int64)
    inblk = distinct_positions(per, need, seed, 2).astype(np.int64)
    reps = [base.copy() for _ in range(k)]
    one = _u[dtype](1)
    off = 0
    for r, c in enumerate(per_replica):
        for j in range(off, off + c):
            reps[r].view(_u[dtype])[blocks[j] * per + inblk[j]] ^= one << _u[dtype](_far_bit(dtype))
        off += c
    ub = -1
    if unresolved_block:
        ub = int(blocks[off])
        for r in range(k):
            reps[r].view(_u[dtype])[ub * per + 5] ^= one << _u[dtype](_split_bit(dtype, r))
    return base, reps, ub
