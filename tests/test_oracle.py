"""Pins for the CPU oracle: what the paper and the mathematics fix.

Nothing here compares the oracle with a retyped copy of itself.  The pins are
published constants, closed forms, library routines that a special case reduces
to (numpy's nextafter, bit-wise TMR majority, scipy's mode, numpy's minimum),
invariants (unanimity, permutation, single-fault outvoting), brute force over
fault positions on tiny buffers, and the paper's 0.1% delta (Sec. IV-D).
"""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
F32, F64, I32 = np.float32, np.float64, np.int32


def b32(x):
    return int(np.array(x, dtype=np.float32).view(np.uint32))


def b64(x):
    return int(np.array(x, dtype=np.float64).view(np.uint64))


# ---------------------------------------------------------------- keys / eq
def _nextafter_steps(a, b, dtype, limit):
    """Number of nextafter steps from a to b (numpy), or None beyond limit."""
    x = dtype(a)
    tgt = dtype(b)
    direction = dtype(np.inf) if tgt > x else dtype(-np.inf)
    for s in range(limit + 1):
        if x == tgt and (np.signbit(x) == np.signbit(tgt) or x != 0):
            return s
        x = np.nextafter(x, direction)
    return None


def test_ulp_distance_matches_nextafter_walk():
    rng = np.random.default_rng(1)
    for dtype, bits in ((np.float32, b32), (np.float64, b64)):
        for _ in range(300):
            a = dtype(rng.uniform(-4, 4)) if rng.random() < 0.9 else dtype(rng.uniform(-1e-37, 1e-37))
            steps = int(rng.integers(0, 7))
            d = dtype(np.inf) if rng.random() < 0.5 else dtype(-np.inf)
            b = a
            for _ in range(steps):
                b = np.nextafter(b, d)
            walk = _nextafter_steps(a, b, dtype, 12)
            assert oracle.ulp_distance(dtype, bits(a), bits(b)) == walk


def test_ulp_closed_forms():
    one = b32(1.0)
    assert oracle.ulp_distance(F32, one, b32(np.nextafter(F32(1), F32(2)))) == 1
    tiny = b32(np.nextafter(F32(0), F32(1)))
    assert oracle.ulp_distance(F32, tiny | 0x80000000, tiny) == 2
    assert oracle.ulp_distance(F32, 0, 0x80000000) == 0
    dmax = b64(np.finfo(np.float64).max)
    assert oracle.ulp_distance(F64, dmax | (1 << 63), dmax) == 2 ** 64 - 2 ** 53 - 2
    fmax = b32(np.finfo(np.float32).max)
    assert oracle.ulp_distance(F32, fmax | 0x80000000, fmax) == 2 * 0x7F7FFFFF


def test_eq_special_values():
    u4 = oracle.ulp(4)
    qnan, snan, nnan = 0x7FC00000, 0x7F800001, 0xFFC00123
    inf, ninf = 0x7F800000, 0xFF800000
    fmax = b32(np.finfo(np.float32).max)
    assert oracle.eq(F32, u4, qnan, snan) and oracle.eq(F32, u4, qnan, nnan)
    assert not oracle.eq(F32, u4, qnan, inf) and not oracle.eq(F32, u4, b32(1.0), qnan)
    assert oracle.eq(F32, u4, inf, inf) and not oracle.eq(F32, u4, inf, ninf)
    assert not oracle.eq(F32, u4, inf, fmax)          # 1 key step apart, still unequal
    assert oracle.eq(F32, u4, 0, 0x80000000)          # +0 == -0
    assert oracle.eq(F32, oracle.ulp(0), 0, 0x80000000)
    assert not oracle.eq(F32, oracle.exact(), 0, 0x80000000)  # EXACT is bit-wise
    r = oracle.rel(1e-3)
    assert oracle.eq(F32, r, 0, 0x80000000) and oracle.eq(F32, r, qnan, snan)
    # integers: bit-wise only
    assert oracle.eq(I32, oracle.exact(), 5, 5) and not oracle.eq(I32, oracle.exact(), 5, 6)
    # denormals are ordinary values: smallest negative and positive are 2 apart
    tiny = b32(np.nextafter(F32(0), F32(1)))
    assert oracle.eq(F32, oracle.ulp(2), tiny | 0x80000000, tiny)
    assert not oracle.eq(F32, oracle.ulp(1), tiny | 0x80000000, tiny)


def test_paper_delta_cases():
    """Sec. IV-D: the 0.1% delta for single precision (golden fixture)."""
    with open(os.path.join(GOLDEN, "paper_delta.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    assert rows
    for a, b, delta, want in rows:
        got = oracle.eq(F32, oracle.rel(float(delta)), b32(float(a)), b32(float(b)))
        assert got == bool(int(want)), (a, b)


def test_rel_matches_exact_rational_away_from_boundary():
    """REL decided in binary64 agrees with exact rational arithmetic whenever the
    pair is not within rounding distance of the threshold."""
    rng = np.random.default_rng(2)
    delta = 1e-3
    checked = 0
    for _ in range(3000):
        a = np.float32(rng.uniform(-10, 10))
        b = np.float32(a * (1 + rng.uniform(-2.5e-3, 2.5e-3)))
        A, B = Fraction(float(a)), Fraction(float(b))
        lhs, rhs = abs(A - B), Fraction(delta) * max(abs(A), abs(B))
        if rhs != 0 and abs(lhs - rhs) / rhs < Fraction(1, 10 ** 9):
            continue
        checked += 1
        assert oracle.eq(F32, oracle.rel(delta), b32(a), b32(b)) == (lhs <= rhs)
    assert checked > 2900


def test_order_key_is_total_order():
    vals = [-np.inf, -1e30, -1.0, -1e-40, -0.0, 0.0, 1e-40, 1.0, 1e30, np.inf]
    keys = [oracle.order_key(F32, b32(v)) for v in vals]
    assert keys == sorted(keys) and len(set(keys)) == len(keys)
    assert oracle.order_key(F32, 0xFFC00000) < keys[0]      # -NaN first
    assert oracle.order_key(F32, 0x7FC00000) > keys[-1]     # +NaN last
    ints = [-(2 ** 31), -5, -1, 0, 1, 7, 2 ** 31 - 1]
    ik = [oracle.order_key(I32, v & 0xFFFFFFFF) for v in ints]
    assert ik == sorted(ik)


# ------------------------------------------------------------------- vote
def _special_f32(rng, n):
    a = rng.uniform(-3, 3, n).astype(np.float32)
    sp = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 1e-45, -1e-45], dtype=np.float32)
    idx = rng.choice(n, size=min(n, 20), replace=False)
    a[idx] = sp[rng.integers(0, sp.size, idx.size)]
    return a


def test_unanimity():
    rng = np.random.default_rng(3)
    for k in range(2, 8):
        a = _special_f32(rng, 200)
        for tol in (oracle.exact(), oracle.ulp(4), oracle.rel(1e-3)):
            r = oracle.vote([a.copy() for _ in range(k)], tol)
            assert np.array_equal(r.consensus.view(np.uint32), a.view(np.uint32))
            assert not r.mask.any() and not r.pair.any() and not r.disagree.any()
            assert r.no_majority == 0 and r.verdict == oracle.UNANIMOUS and r.winner == 0


def test_empty_task():
    r = oracle.vote([np.zeros(0, np.float32)] * 3, oracle.ulp(4))
    assert r.verdict == oracle.UNANIMOUS and r.consensus.size == 0


def test_tmr_textbook_bitwise_majority():
    """EXACT, k=3: wherever two replicas agree the vote is textbook TMR,
    consensus = (a&b)|(a&c)|(b&c) per bit."""
    rng = np.random.default_rng(4)
    n = 5000
    base = rng.integers(-2 ** 31, 2 ** 31, n, dtype=np.int64).astype(np.int32)
    reps = [base.copy() for _ in range(3)]
    for r in range(3):
        idx = rng.choice(n, 600, replace=False)
        reps[r][idx] ^= (1 << rng.integers(0, 32, 600)).astype(np.int64).astype(np.uint32).view(np.int32)
    res = oracle.vote(reps, oracle.exact())
    a, b, c = (x.view(np.uint32) for x in reps)
    tmr = (a & b) | (a & c) | (b & c)
    has_maj = (a == b) | (a == c) | (b == c)
    assert np.array_equal(res.consensus.view(np.uint32)[has_maj], tmr[has_maj])
    assert np.array_equal((res.mask & 0x80) != 0, ~has_maj)
    # no majority: all three differ; consensus is the median integer (numpy sort)
    med = np.sort(np.stack(reps), axis=0)[1]
    assert np.array_equal(res.consensus[~has_maj], med[~has_maj])
    for r, x in enumerate((a, b, c)):
        assert np.array_equal(((res.mask >> r) & 1).astype(bool), x != res.consensus.view(np.uint32))
    # EXACT pair counts are plain inequality counts
    for i, j in itertools.permutations(range(3), 2):
        assert res.pair[i, j] == np.count_nonzero(reps[i] != reps[j])


def test_k5_exact_majority_is_the_mode():
    from scipy import stats
    rng = np.random.default_rng(5)
    n = 3000
    reps = np.stack([rng.integers(0, 4, n).astype(np.int32) for _ in range(5)])
    res = oracle.vote(list(reps), oracle.exact())
    mode, cnt = stats.mode(reps, axis=0, keepdims=False)
    strict = cnt >= 3
    assert np.array_equal(res.consensus[strict], mode[strict])
    assert np.array_equal((res.mask & 0x80) == 0, strict)
    assert res.no_majority == np.count_nonzero(~strict)


def test_dmr_disagreement_undecidable():
    """k = 2 (DMR, Sec. IV-D): a disagreement is detected but not decided; the
    consensus is then the smaller value (numeric order for non-zero finite)."""
    rng = np.random.default_rng(6)
    a = rng.uniform(-5, 5, 1000).astype(np.float32)
    b = a.copy()
    idx = rng.choice(1000, 50, replace=False)
    b[idx] = rng.uniform(-5, 5, 50).astype(np.float32)
    res = oracle.vote([a, b], oracle.ulp(4))
    dif = a.view(np.uint32) != b.view(np.uint32)
    assert np.array_equal(res.consensus, np.minimum(a, b))
    assert np.array_equal((res.mask & 0x80) != 0, dif)
    assert res.verdict == oracle.UNRESOLVED
    r2 = oracle.vote([a, a.copy()], oracle.ulp(4))
    assert r2.verdict == oracle.UNANIMOUS


def test_single_corrupted_replica_outvoted():
    rng = np.random.default_rng(7)
    n = 4000
    base = _special_f32(rng, n)
    bad = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32).view(np.float32)
    for tol in (oracle.exact(), oracle.ulp(4), oracle.rel(1e-3)):
        for pos in range(3):
            reps = [base.copy(), base.copy(), base.copy()]
            reps[pos] = bad.copy()
            res = oracle.vote(reps, tol)
            assert np.array_equal(res.consensus.view(np.uint32), base.view(np.uint32))
            assert res.no_majority == 0
            others = [r for r in range(3) if r != pos]
            assert not (res.mask & sum(1 << r for r in others)).any()


def test_permutation_invariance():
    rng = np.random.default_rng(8)
    n = 2000
    for k in (3, 4, 5, 7):
        base = _special_f32(rng, n)
        reps = []
        for r in range(k):
            x = base.copy()
            synth.ulp_noise(x, 99, r, round(0.3 * (1 << 24)), 6)
            idx = rng.choice(n, 100, replace=False)
            x[idx] = rng.uniform(-3, 3, 100).astype(np.float32)
            reps.append(x)
        tol = oracle.ulp(4)
        ref = oracle.vote(reps, tol)
        for _ in range(4):
            perm = rng.permutation(k)
            res = oracle.vote([reps[p] for p in perm], tol)
            assert np.array_equal(res.consensus.view(np.uint32), ref.consensus.view(np.uint32))
            assert np.array_equal(res.mask & 0x80, ref.mask & 0x80)
            for new, old in enumerate(perm):
                assert np.array_equal((res.mask >> new) & 1, (ref.mask >> old) & 1)
                assert res.disagree[new] == ref.disagree[old]
                for new2, old2 in enumerate(perm):
                    assert res.pair[new, new2] == ref.pair[old, old2]
            assert res.verdict == ref.verdict


def test_brute_force_fault_positions():
    """Every subset of positions of a tiny buffer corrupted in one replica:
    the fault is outvoted, localised exactly, and counted exactly."""
    rng = np.random.default_rng(9)
    n = 6
    for k in (3, 5):
        base = rng.uniform(-2, 2, n).astype(np.float32)
        for victim in range(k):
            for subset in range(1 << n):
                reps = [base.copy() for _ in range(k)]
                pos = [i for i in range(n) if subset >> i & 1]
                reps[victim][pos] = -reps[victim][pos] - 7.0   # far beyond any tolerance
                res = oracle.vote(reps, oracle.ulp(4))
                assert np.array_equal(res.consensus, base)
                expect = np.zeros(n, np.uint8)
                expect[pos] = 1 << victim
                assert np.array_equal(res.mask, expect)
                assert res.disagree[victim] == len(pos) and res.disagree.sum() == len(pos)
                for j in range(k):
                    if j != victim:
                        assert res.pair[victim, j] == len(pos) == res.pair[j, victim]
                if pos:
                    assert res.verdict == oracle.TASK_MAJORITY and res.winner == (1 if victim == 0 else 0)
                else:
                    assert res.verdict == oracle.UNANIMOUS


def test_non_transitive_chain():
    """a ~ b ~ c but a !~ c (tolerance 4 ULP, steps of 3): b is the only value
    supported by all three replicas."""
    a = np.float32(1.5)
    ab = b32(a)
    vals = [ab, ab + 3, ab + 6]
    reps = [np.array([v], dtype=np.uint32).view(np.float32) for v in vals]
    res = oracle.vote(reps, oracle.ulp(4))
    assert int(res.consensus.view(np.uint32)[0]) == ab + 3
    assert res.mask[0] == 0 and res.pair[0, 2] == 1 and res.pair[0, 1] == 0
    assert res.verdict == oracle.TASK_MAJORITY and res.winner == 1


def test_count_identities_and_ulp_pairs_by_walk():
    reps = synth.small_task_set(n=4096)
    res = oracle.vote(reps, oracle.ulp(4))
    pop = np.unpackbits((res.mask & 0x7F)[:, None], axis=1).sum()
    assert res.disagree.sum() == pop
    assert res.no_majority == np.count_nonzero(res.mask & 0x80)
    assert np.array_equal(res.pair, res.pair.T) and not np.diag(res.pair).any()
    # pairwise "not within 4 ULP", decided by walking nextafter (numpy)
    for i, j in itertools.combinations(range(3), 2):
        a, b = reps[i], reps[j]
        far = 0
        for x, y in zip(a[a.view(np.uint32) != b.view(np.uint32)], b[a.view(np.uint32) != b.view(np.uint32)]):
            far += _nextafter_steps(x, y, np.float32, 4) is None
        assert res.pair[i, j] == far
    # small-task-set faults: every flip that left the 4-ULP window is flagged in replica 2
    assert res.disagree[0] == 0 and res.disagree[1] == 0
    assert res.verdict == oracle.TASK_MAJORITY and res.winner == 0


def test_verdict_ladder():
    x = np.arange(8, dtype=np.float32)
    far = x + 100
    # element majority only: each replica wrong somewhere, never two at once
    r0, r1, r2 = x.copy(), x.copy(), x.copy()
    r0[0] = 50
    r1[1] = 50
    r2[2] = 50
    res = oracle.vote([r0, r1, r2], oracle.ulp(4))
    assert res.verdict == oracle.ELEMENT_MAJORITY and np.array_equal(res.consensus, x)
    assert res.winner == 0
    # unresolved: all three differ at one element
    r2b = r2.copy()
    r2b[0] = 60
    r1b = r1.copy()
    r1b[0] = 70
    res = oracle.vote([r0, r1b, r2b], oracle.ulp(4))
    assert res.verdict == oracle.UNRESOLVED and res.no_majority == 1
    res = oracle.vote([x, far, x.copy()], oracle.ulp(4))
    assert res.verdict == oracle.TASK_MAJORITY and res.winner == 0


def _plant_k5(per_replica, no_majority_element=False, n=64):
    """k = 5 fp32 replicas of arange(n) with replica r wrong (value 1000 + r) on
    per_replica[r] elements of its own, no element shared by two replicas, so
    that every element keeps a 4-of-5 majority.  With no_majority_element,
    element n-1 holds a, a, b, b, c (support 2, 2, 2, 2, 1): no strict majority,
    candidates {a, a, b, b}, lower median a = replicas 0 and 1, so replicas
    2, 3 and 4 are flagged there."""
    x = np.arange(n, dtype=np.float32)
    reps = [x.copy() for _ in range(5)]
    pos = 0
    for r, cnt in enumerate(per_replica):
        for _ in range(cnt):
            reps[r][pos] = 1000.0 + r
            pos += 1
    assert pos < n - 1
    if no_majority_element:
        for r, v in enumerate((-5.0, -5.0, 7.0, 7.0, 9.0)):
            reps[r][n - 1] = v
    return x, reps


def test_winner_is_argmin_of_disagree_element_majority():
    """Sec. IV-D winner rule outside TASK_MAJORITY: the replica with the fewest
    disagreements, the lowest index on ties.  Disagree counts (3,1,2,1,4) make
    argmin-lowest = 1, argmin-highest = 3, argmax = 4, and replica 0 (the
    default) a loser; every replica has a fault of its own, so no replica
    agrees with another over the whole task (support 1 each: no TASK_MAJORITY)."""
    x, reps = _plant_k5((3, 1, 2, 1, 4))
    res = oracle.vote(reps, oracle.ulp(4))
    assert list(res.disagree) == [3, 1, 2, 1, 4]
    assert res.no_majority == 0 and np.array_equal(res.consensus, x)
    assert res.verdict == oracle.ELEMENT_MAJORITY
    assert res.winner == 1


def test_winner_is_argmin_of_disagree_unresolved():
    """The same counts reached with one element that has no majority: planted
    faults (3,1,1,0,3) plus the a,a,b,b,c element adding one to replicas 2, 3, 4."""
    x, reps = _plant_k5((3, 1, 1, 0, 3), no_majority_element=True)
    res = oracle.vote(reps, oracle.ulp(4))
    assert list(res.disagree) == [3, 1, 2, 1, 4]
    assert res.no_majority == 1 and res.mask[-1] == 0x80 | 0b11100
    assert res.consensus[-1] == np.float32(-5.0)
    assert res.verdict == oracle.UNRESOLVED
    assert res.winner == 1


def test_task_majority_needs_a_strict_majority_of_replicas():
    """k = 4: replicas 0 and 1 agree everywhere, 2 and 3 each have faults of
    their own.  Task support T = (2, 2, 1, 1) and 2*2 > 4 is false: no replica
    is a valid result alone, the consensus is (ELEMENT_MAJORITY, winner = the
    lowest replica with no disagreement)."""
    x = np.arange(16, dtype=np.float32)
    reps = [x.copy(), x.copy(), x.copy(), x.copy()]
    reps[2][3] = 100.0
    reps[3][5] = 200.0
    reps[3][6] = 300.0
    res = oracle.vote(reps, oracle.ulp(4))
    assert list(res.disagree) == [0, 0, 1, 2]
    assert res.verdict == oracle.ELEMENT_MAJORITY and res.winner == 0
    # k = 5 with three replicas clean: T = 3 for them, 2*3 > 5 -> TASK_MAJORITY,
    # lowest such replica; replica 0 is faulty so the winner is 1
    reps = [x.copy() for _ in range(5)]
    reps[0][1] = 50.0
    reps[3][2] = 60.0
    res = oracle.vote(reps, oracle.ulp(4))
    assert res.verdict == oracle.TASK_MAJORITY and res.winner == 1


def test_fp64_and_int64_paths():
    rng = np.random.default_rng(10)
    a = rng.standard_normal(500)
    b = a.copy()
    b.view(np.uint64)[::7] += np.uint64(2)
    c = a.copy()
    c[3] = 1e300
    res = oracle.vote([a, b, c], oracle.ulp(2))
    assert np.array_equal(res.consensus, a) and res.disagree[2] == 1 and res.disagree[1] == 0
    res = oracle.vote([a, b, c], oracle.ulp(1))
    assert res.pair[0, 1] == len(range(0, 500, 7))
    ia = rng.integers(-2 ** 62, 2 ** 62, 300)
    ib = ia.copy()
    ib[5] += 1
    res = oracle.vote([ia, ib, ia.copy()], oracle.exact())
    assert np.array_equal(res.consensus, ia) and res.mask[5] == 2


def test_invalid_arguments():
    a = np.zeros(4, np.int32)
    with pytest.raises(ValueError):
        oracle.vote([a, a, a], oracle.ulp(2))       # ULP on an integer type
    with pytest.raises(ValueError):
        oracle.vote([a], oracle.exact())            # k < 2
    with pytest.raises(ValueError):
        oracle.vote([a] * 8, oracle.exact())        # k > 7


# ------------------------------------------------------------ fingerprints
def test_fnv_published_vectors():
    with open(os.path.join(GOLDEN, "fnv1a64_vectors.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for text, want in rows:
        s = text.strip('"').encode()
        # word-wise FNV-1a over words < 256 is byte-wise FNV-1a over those bytes
        assert oracle.fnv1a_words(list(s)) == int(want, 16)


def test_fingerprint_single_leaf_is_fnv_over_eight_words():
    rng = np.random.default_rng(11)
    w = rng.integers(0, 2 ** 63, 8, dtype=np.uint64)
    assert oracle.fingerprint(w.view(np.uint8), 64)[0] == oracle.fnv1a_words(w)


def test_fingerprint_complete_tree_closed_form():
    """All 1024 leaves identical: a complete binary tree of depth 10 gives the
    leaf value pushed through h <- node(h, h) ten times."""
    pattern = np.arange(1, 9, dtype=np.uint64)
    block = np.tile(pattern, 8192 // 8)
    h = oracle.fnv1a_words(pattern)
    for _ in range(10):
        h = oracle.fnv1a_words([h, h])
    assert oracle.fingerprint(block.view(np.uint8), 65536)[0] == h


def test_fingerprint_halves_recursion():
    rng = np.random.default_rng(12)
    buf = rng.integers(0, 2 ** 63, 8192, dtype=np.uint64).view(np.uint8)
    for bb in (128, 1024, 8192, 65536):
        whole = oracle.fingerprint(buf, bb)
        halves = oracle.fingerprint(buf, bb // 2)
        for b in range(whole.size):
            assert whole[b] == oracle.fnv1a_words([halves[2 * b], halves[2 * b + 1]])


def test_fingerprint_every_single_word_change_detected():
    rng = np.random.default_rng(13)
    words = rng.integers(0, 2 ** 63, 64, dtype=np.uint64)   # 512 B block
    ref = oracle.fingerprint(words.view(np.uint8), 512)[0]
    seen = {int(ref)}
    for i in range(64):
        for delta in (1, 1 << 17, 1 << 63, 0xFFFFFFFFFFFFFFFF):
            w = words.copy()
            w[i] ^= np.uint64(delta)
            fp = int(oracle.fingerprint(w.view(np.uint8), 512)[0])
            assert fp != ref
            seen.add(fp)
            if delta == 1 << 63:
                # xoring bit 63 adds 2^63 mod 2^64, and 2^63 * (odd prime) = 2^63:
                # the flip survives every later step unchanged (closed form)
                assert fp == int(ref) ^ (1 << 63)
    assert len(seen) == 1 + 64 * 3 + 1


def test_fingerprint_leaf_order_and_zero_padding():
    rng = np.random.default_rng(14)
    words = rng.integers(0, 2 ** 63, 32, dtype=np.uint64)
    swapped = words.copy()
    swapped[0:8], swapped[8:16] = words[8:16].copy(), words[0:8].copy()
    assert oracle.fingerprint(words.view(np.uint8), 256)[0] != oracle.fingerprint(swapped.view(np.uint8), 256)[0]
    raw = rng.integers(0, 256, 1000, dtype=np.uint8)
    padded = np.zeros(1024, np.uint8)
    padded[:1000] = raw
    assert np.array_equal(oracle.fingerprint(raw, 512), oracle.fingerprint(padded, 512))
    assert oracle.fingerprint(np.zeros(0, np.uint8), 512).size == 0


# -------------------------------------------------------------- block vote
def test_block_vote_identical_replicas():
    a = synth.values("f64", synth.NORMAL, 5, 0, 4096)
    res = oracle.vote_blocks([a.copy() for _ in range(5)], oracle.exact(), 4096)
    assert res.verdict == oracle.UNANIMOUS and not res.blockmap.any()
    assert np.array_equal(res.consensus.view(np.uint64), a.view(np.uint64))


def test_block_vote_checkpoint_shape():
    n = 64 * 512   # 64 blocks of 4 KiB
    reps = synth.checkpoint_set(n, nstuck=9, nflip=7)
    base = reps[0]
    res = oracle.vote_blocks(reps, oracle.exact(), 4096)
    per = 4096 // 8
    stuck = set((np.nonzero(reps[1].view(np.uint64) != base.view(np.uint64))[0] // per).tolist())
    flips = set((np.nonzero(reps[2].view(np.uint64) != base.view(np.uint64))[0] // per).tolist())
    for b in range(res.blocks):
        m = int(res.blockmap[b])
        assert bool(m & 2) == (b in stuck) and bool(m & 4) == (b in flips)
        assert m & 8            # rotated replica differs in every block of random data
        assert not m & 1 and not m & 16
    assert np.array_equal(res.consensus.view(np.uint64), base.view(np.uint64))
    assert res.fallback_blocks == 0 and res.verdict == oracle.TASK_MAJORITY and res.winner == 0


def test_block_vote_no_majority_falls_back_to_element_vote():
    n = 8 * 512
    reps = synth.checkpoint_set(n, nstuck=1, nflip=1)
    base = reps[0]
    # force a stuck word (r1) and a flip (r2) into block 3 -> 2 of 5 agree there
    reps[1] = base.copy()
    reps[2] = base.copy()
    reps[1][3 * 512 + 10] = 0.0
    reps[2].view(np.uint64)[3 * 512 + 400] ^= np.uint64(1 << 40)
    res = oracle.vote_blocks(reps, oracle.exact(), 4096)
    assert res.blockmap[3] & 0x80 and res.fallback_blocks == 1
    assert np.array_equal(res.consensus.view(np.uint64), base.view(np.uint64))
    assert res.unresolved_elems == 0 and res.verdict == oracle.ELEMENT_MAJORITY
    assert res.mask[3 * 512 + 10] & 2 and res.mask[3 * 512 + 400] & 4
    assert res.mask[3 * 512 + 11] == 8   # the rotated replica, flagged element-wise
    assert not res.mask[:3 * 512].any()


def _block_reps_k5(n_blocks, per=512):
    """k = 5 fp64 replicas of distinct random words, n_blocks blocks of 4 KiB."""
    base = synth.values("f64", synth.NORMAL, 21, 0, n_blocks * per)
    return base, [base.copy() for _ in range(5)]


def _corrupt_blocks(reps, plan, per=512):
    """plan: list of (replica, block): one word of that block changed in that
    replica; each block is corrupted in at most one replica, so every block keeps
    a 4-of-5 fingerprint majority."""
    for r, b in plan:
        reps[r].view(np.uint64)[b * per + 7] ^= np.uint64(1 << 33)


def test_block_vote_winner_is_argmin_element_majority():
    """Replica blocks (3,1,2,1,4): every replica differs somewhere, no fallback
    block -> ELEMENT_MAJORITY with winner = the lowest index of the fewest
    differing blocks (1; argmax would give 4, highest-index ties 3)."""
    base, reps = _block_reps_k5(16)
    plan = [(0, 0), (0, 1), (0, 2), (1, 3), (2, 4), (2, 5), (3, 6), (4, 7), (4, 8), (4, 9), (4, 10)]
    _corrupt_blocks(reps, plan)
    res = oracle.vote_blocks(reps, oracle.exact(), 4096)
    assert list(res.replica_blocks) == [3, 1, 2, 1, 4]
    assert res.fallback_blocks == 0 and res.disagree_blocks == 11
    assert np.array_equal(res.consensus.view(np.uint64), base.view(np.uint64))
    for r, b in plan:
        assert res.blockmap[b] == 1 << r
    assert res.verdict == oracle.ELEMENT_MAJORITY and res.winner == 1


def test_block_vote_unresolved_and_its_winner():
    """One block with fingerprints a,a,b,b,c (support 2,2,2,2,1: no strict
    majority) falls back to the element vote, whose element 9 also has no
    majority (replicas 2 and 3 agree on another value, replica 4 on a third):
    UNRESOLVED.  The source of that block is replica 0 (the lowest of maximal
    support), so replicas 2, 3, 4 are counted as differing there; with the
    majority-block faults (3,1,1,0,3) the replica blocks are (3,1,2,1,4) and the
    winner is replica 1."""
    per = 512
    base, reps = _block_reps_k5(16)
    plan = [(0, 0), (0, 1), (0, 2), (1, 3), (2, 4), (4, 7), (4, 8), (4, 10)]
    _corrupt_blocks(reps, plan)
    fb = 12
    w = [r.view(np.uint64) for r in reps]
    w[2][fb * per + 9] = w[3][fb * per + 9] = np.uint64(0x3FF0000000000000)   # 1.0
    w[4][fb * per + 9] = np.uint64(0x4000000000000000)                        # 2.0
    res = oracle.vote_blocks(reps, oracle.exact(), 4096)
    assert res.blockmap[fb] == 0x80 | 0b11100
    assert res.fallback_blocks == 1 and res.unresolved_elems == 1
    assert list(res.replica_blocks) == [3, 1, 2, 1, 4]
    assert res.mask[fb * per + 9] == 0x80 | 0b11100
    # element 9 has candidates {base, base, 1.0, 1.0}; the lower median under
    # totalOrder is the smaller of base[9] and 1.0
    lo = min(float(base[fb * per + 9]), 1.0)
    assert res.consensus[fb * per + 9] == lo
    assert res.verdict == oracle.UNRESOLVED and res.winner == 1


def test_block_vote_task_majority_winner_is_lowest_clean_replica():
    """Replica 0 differs in one block and replica 1 nowhere: TASK_MAJORITY with
    winner 1 (not the default 0), and the consensus is restored from replica 1
    in the block where replica 0 is the outlier."""
    base, reps = _block_reps_k5(8)
    _corrupt_blocks(reps, [(0, 2), (2, 5)])
    res = oracle.vote_blocks(reps, oracle.exact(), 4096)
    assert res.verdict == oracle.TASK_MAJORITY and res.winner == 1
    assert np.array_equal(res.consensus.view(np.uint64), base.view(np.uint64))


def test_threaded_vote_is_the_sequential_vote():
    """The host-core timing leg (the element loop split over OpenMP threads,
    counters summed per thread) gives the sequential oracle's bits and counts,
    for every thread count, on a set with every kind of fault and ragged
    per-thread ranges."""
    cases = [(synth.small_task_set(n=100003), oracle.ulp(4)),
             (synth.planted_set("f64", 77777, [40, 10, 30, 10, 50], 3)[1], oracle.ulp(2)),
             (synth.planted_set("i32", 5001, [5, 1, 3], 1)[1], oracle.exact()),
             (synth.large_task_set(65536, "f32", flip_rate=1e-4), oracle.rel(1e-3))]
    for reps, tol in cases:
        ref = oracle.vote(reps, tol)
        u = np.uint32 if reps[0].itemsize == 4 else np.uint64
        for nt in (1, 2, 3, 7, 16):
            got, used = oracle.vote_threads(reps, tol, nt)
            assert used == nt
            assert np.array_equal(got.consensus.view(u), ref.consensus.view(u))
            assert np.array_equal(got.mask, ref.mask)
            assert np.array_equal(got.pair, ref.pair) and np.array_equal(got.disagree, ref.disagree)
            assert (got.no_majority, got.verdict, got.winner) == (ref.no_majority, ref.verdict, ref.winner)
    got, used = oracle.vote_threads([np.zeros(0, np.float32)] * 3, oracle.ulp(4), 4)
    assert got.verdict == oracle.UNANIMOUS and got.mask.size == 0
