/*
 * ftv_oracle.c -- plain, slow CPU oracle for the heterogeneity-aware majority
 * voter (Kicherer & Karl, "Heterogeneity-aware Fault Tolerance using a
 * Self-Organizing Runtime System", Sec. IV-D) and for the block fingerprints
 * used to validate checkpoints.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the GPU library: every definition below is
 * written out again from the paper's statement of the problem.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 * (no FMA contraction, no flush-to-zero: the relative test must round exactly
 * as IEEE-754 binary64 with round-to-nearest-even prescribes).  OpenMP is only
 * used by fto_vote_threads, the host-core timing leg; every other function is
 * sequential.
 *
 * Everything is scalar and sequential, one element at a time, in the order the
 * definitions are stated.  Element values are handled as raw bit patterns
 * (uint64_t holding 32- or 64-bit words) so that NaN payloads and signed zeros
 * are never altered by a load.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* value types: the type a buffer is registered with selects how its values are
 * compared (Sec. IV-E: buffers are registered together with their value type). */
#define O_F32 0
#define O_F64 1
#define O_I32 2
#define O_I64 3

/* tolerance kinds (Sec. IV-D) */
#define O_EXACT 0 /* bit-wise comparison, the rule for integer types      */
#define O_ULP 1   /* float: integer distance between ordered bit keys      */
#define O_REL 2   /* float: relative delta, the paper's 0.1% for fp32       */

/* verdicts */
#define O_UNANIMOUS 0
#define O_TASK_MAJORITY 1
#define O_ELEMENT_MAJORITY 2
#define O_UNRESOLVED 3

#define O_MAXK 7
#define O_NOMAJ_BIT 0x80u

/* counter layout shared by the Python wrapper: pair[7][7], disagree[7], no_majority */
#define O_NCOUNT (49 + 7 + 1)

typedef struct {
  int kind;
  uint64_t max_ulp;
  double delta;
  double abs_floor;
} otol;

static int o_valid_dtype(int dt) { return dt >= O_F32 && dt <= O_I64; }
static int o_is_float(int dt) { return dt == O_F32 || dt == O_F64; }
static int o_size(int dt) { return (dt == O_F32 || dt == O_I32) ? 4 : 8; }

static uint64_t o_load(const void *p, int dt, uint64_t i) {
  if (o_size(dt) == 4) {
    uint32_t v;
    memcpy(&v, (const unsigned char *)p + 4 * i, 4);
    return v;
  }
  uint64_t v;
  memcpy(&v, (const unsigned char *)p + 8 * i, 8);
  return v;
}

static void o_store(void *p, int dt, uint64_t i, uint64_t bits) {
  if (o_size(dt) == 4) {
    uint32_t v = (uint32_t)bits;
    memcpy((unsigned char *)p + 4 * i, &v, 4);
  } else {
    memcpy((unsigned char *)p + 8 * i, &bits, 8);
  }
}

/* IEEE-754 field views of a raw float pattern */
static uint64_t o_sign(int dt, uint64_t u) { return dt == O_F32 ? (u >> 31) & 1u : u >> 63; }
static uint64_t o_mag(int dt, uint64_t u) {
  return dt == O_F32 ? (u & 0x7fffffffULL) : (u & 0x7fffffffffffffffULL);
}
static uint64_t o_inf_mag(int dt) { return dt == O_F32 ? 0x7f800000ULL : 0x7ff0000000000000ULL; }
static int o_isnan(int dt, uint64_t u) { return o_mag(dt, u) > o_inf_mag(dt); }
static int o_isinf(int dt, uint64_t u) { return o_mag(dt, u) == o_inf_mag(dt); }

/* Signed-magnitude -> two's-complement key: adjacent finite floats have keys
 * that differ by exactly one, and +0 / -0 both map to 0. */
static int64_t o_ulp_key(int dt, uint64_t u) {
  int64_t m = (int64_t)o_mag(dt, u);
  return o_sign(dt, u) ? -m : m;
}

/* |a - b| of two keys, exact: the difference of two 64-bit keys can exceed
 * INT64_MAX, so it is taken in unsigned arithmetic, larger minus smaller. */
static uint64_t o_key_dist(int64_t a, int64_t b) {
  return a >= b ? (uint64_t)a - (uint64_t)b : (uint64_t)b - (uint64_t)a;
}

static double o_as_double(int dt, uint64_t u) {
  if (dt == O_F32) {
    uint32_t w = (uint32_t)u;
    float f;
    memcpy(&f, &w, 4);
    return (double)f; /* exact widening */
  }
  double d;
  memcpy(&d, &u, 8);
  return d;
}

/* The voter's notion of "equal" (Sec. IV-D): bit-wise for integer types; for
 * floating point, values that differ by no more than a programmer-set maximum
 * are equal.  NaN equals any NaN (payloads differ between processing units),
 * an infinity equals only the same infinity, +0 equals -0. */
static int o_eq(int dt, const otol *t, uint64_t a, uint64_t b) {
  if (!o_is_float(dt) || t->kind == O_EXACT) return a == b;
  int an = o_isnan(dt, a), bn = o_isnan(dt, b);
  if (an || bn) return an && bn;
  if (o_isinf(dt, a) || o_isinf(dt, b)) return a == b;
  int64_t ka = o_ulp_key(dt, a), kb = o_ulp_key(dt, b);
  if (ka == kb) return 1;
  if (t->kind == O_ULP) return o_key_dist(ka, kb) <= t->max_ulp;
  /* relative test in binary64: |A-B| <= delta * max(|A|,|B|), or an absolute floor */
  double A = o_as_double(dt, a), B = o_as_double(dt, b);
  double d = fabs(A - B);
  double m = fmax(fabs(A), fabs(B));
  double lim = t->delta * m;
  return d <= lim || d <= t->abs_floor;
}

/* Order used to break ties among equally supported candidates: IEEE-754
 * totalOrder for floats (-NaN < -inf < ... < -0 < +0 < ... < +inf < +NaN),
 * two's-complement order for integers.  Mapped to an unsigned key. */
static uint64_t o_order_key(int dt, uint64_t u) {
  switch (dt) {
  case O_F32: return (u >> 31) ? (~u & 0xffffffffULL) : (u | 0x80000000ULL);
  case O_F64: return (u >> 63) ? ~u : (u | 0x8000000000000000ULL);
  case O_I32: return (u ^ 0x80000000ULL) & 0xffffffffULL;
  default: return u ^ 0x8000000000000000ULL;
  }
}

static int o_check(int dt, int k, const otol *t) {
  if (!o_valid_dtype(dt)) return -2;
  if (k < 2 || k > O_MAXK) return -3;
  if (t->kind < O_EXACT || t->kind > O_REL) return -1;
  if (!o_is_float(dt) && t->kind != O_EXACT) return -1;
  return 0;
}

/* One element of the majority vote.  x[0..k-1] are the replicas' bit patterns.
 * Writes the consensus pattern and the mask byte, and adds the element's
 * contribution to the counters. */
static void o_vote_element(int dt, int k, const otol *t, const uint64_t *x, uint64_t *cons,
                           uint8_t *maskbyte, uint64_t *cnt) {
  int e[O_MAXK][O_MAXK];
  int s[O_MAXK];
  for (int r = 0; r < k; ++r)
    for (int j = 0; j < k; ++j) e[r][j] = o_eq(dt, t, x[r], x[j]);

  /* support of each replica's value, counting itself */
  int M = 0;
  for (int r = 0; r < k; ++r) {
    s[r] = 0;
    for (int j = 0; j < k; ++j) s[r] += e[r][j];
    if (s[r] > M) M = s[r];
  }
  int majority = 2 * M > k;

  /* candidates: the replicas of maximal support, in replica order */
  int cand[O_MAXK] = {0}, nc = 0;
  for (int r = 0; r < k; ++r)
    if (s[r] == M) cand[nc++] = r;
  /* sort candidates by (order key, replica index) -- insertion sort */
  for (int a = 1; a < nc; ++a) {
    int v = cand[a];
    int b = a - 1;
    while (b >= 0) {
      uint64_t kb = o_order_key(dt, x[cand[b]]), kv = o_order_key(dt, x[v]);
      if (kb > kv || (kb == kv && cand[b] > v)) {
        cand[b + 1] = cand[b];
        --b;
      } else {
        break;
      }
    }
    cand[b + 1] = v;
  }
  int c = cand[(nc - 1) / 2]; /* lower median */
  *cons = x[c];

  uint8_t m = 0;
  for (int r = 0; r < k; ++r)
    if (!o_eq(dt, t, x[r], x[c])) m |= (uint8_t)(1u << r);
  if (!majority) m |= O_NOMAJ_BIT;
  *maskbyte = m;

  uint64_t *pair = cnt, *dis = cnt + 49, *nomaj = cnt + 56;
  for (int r = 0; r < k; ++r)
    for (int j = 0; j < k; ++j)
      if (r != j && !e[r][j]) pair[r * 7 + j] += 1;
  for (int r = 0; r < k; ++r)
    if (m & (1u << r)) dis[r] += 1;
  if (!majority) *nomaj += 1;
}

/* Task verdict from the counters.  Replica r agrees with replica j over the
 * whole task iff pair[r][j] == 0; a replica agreeing with a strict majority of
 * the replicas over the whole task is a valid result on its own. */
static void o_verdict(int k, const uint64_t *cnt, int32_t *verdict, int32_t *winner) {
  const uint64_t *pair = cnt, *dis = cnt + 49, nomaj = cnt[56];
  int all_zero = 1;
  for (int r = 0; r < k; ++r)
    for (int j = 0; j < k; ++j)
      if (pair[r * 7 + j] != 0) all_zero = 0;
  int best = -1, bestT = -1;
  for (int r = 0; r < k; ++r) {
    int T = 0;
    for (int j = 0; j < k; ++j) T += pair[r * 7 + j] == 0;
    if (T > bestT) {
      bestT = T;
      best = r;
    }
  }
  int argmin = 0;
  for (int r = 1; r < k; ++r)
    if (dis[r] < dis[argmin]) argmin = r;
  if (all_zero) {
    *verdict = O_UNANIMOUS;
    *winner = 0;
  } else if (2 * bestT > k) {
    *verdict = O_TASK_MAJORITY;
    *winner = best;
  } else if (nomaj == 0) {
    *verdict = O_ELEMENT_MAJORITY;
    *winner = argmin;
  } else {
    *verdict = O_UNRESOLVED;
    *winner = argmin;
  }
}

/* ---- exported: single compare ------------------------------------------ */
int fto_eq(int dt, int kind, uint64_t max_ulp, double delta, double abs_floor, uint64_t a,
           uint64_t b) {
  otol t = {kind, max_ulp, delta, abs_floor};
  return o_eq(dt, &t, a, b);
}

uint64_t fto_ulp_distance(int dt, uint64_t a, uint64_t b) {
  return o_key_dist(o_ulp_key(dt, a), o_ulp_key(dt, b));
}

uint64_t fto_order_key(int dt, uint64_t u) { return o_order_key(dt, u); }

/* ---- exported: the vote over one task ----------------------------------- *
 * reps[r] : replica r, n elements of dtype dt (host memory)
 * consensus : n elements (may be NULL); mask : n bytes (may be NULL)
 * counts  : O_NCOUNT uint64 (pair[7][7], disagree[7], no_majority), overwritten
 * vw      : int32[2] = {verdict, winner}
 * returns 0, or a negative code for invalid arguments. */
int fto_vote(int dt, int k, uint64_t n, const void *const *reps, int kind, uint64_t max_ulp,
             double delta, double abs_floor, void *consensus, uint8_t *mask, uint64_t *counts,
             int32_t *vw) {
  otol t = {kind, max_ulp, delta, abs_floor};
  int rc = o_check(dt, k, &t);
  if (rc) return rc;
  for (int i = 0; i < O_NCOUNT; ++i) counts[i] = 0;
  uint64_t x[O_MAXK];
  for (uint64_t i = 0; i < n; ++i) {
    for (int r = 0; r < k; ++r) x[r] = o_load(reps[r], dt, i);
    uint64_t c;
    uint8_t m;
    o_vote_element(dt, k, &t, x, &c, &m, counts);
    if (consensus) o_store(consensus, dt, i, c);
    if (mask) mask[i] = m;
  }
  o_verdict(k, counts, &vw[0], &vw[1]);
  return 0;
}

/* ---- exported: the same vote on several host threads ----------------------
 * The element loop of fto_vote with the elements split into one contiguous
 * range per thread (OpenMP), each thread adding to counters of its own; the
 * per-thread counters are summed afterwards (integer sums: the order does not
 * matter) and the verdict is taken from the totals.  Consensus, mask, counts
 * and verdict are those of fto_vote.  nthreads <= 0: OpenMP's default.
 * *used receives the number of threads that ran. */
#ifdef _OPENMP
#include <omp.h>
#endif
int fto_vote_threads(int dt, int k, uint64_t n, const void *const *reps, int kind, uint64_t max_ulp,
                     double delta, double abs_floor, void *consensus, uint8_t *mask, uint64_t *counts,
                     int32_t *vw, int nthreads, int *used) {
  otol t = {kind, max_ulp, delta, abs_floor};
  int rc = o_check(dt, k, &t);
  if (rc) return rc;
  int T = 1;
#ifdef _OPENMP
  T = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
  uint64_t *per = (uint64_t *)calloc((size_t)T * O_NCOUNT, sizeof(uint64_t));
  if (!per) return -6;
  int ran = 1;
#ifdef _OPENMP
#pragma omp parallel num_threads(T)
#endif
  {
    int me = 0, nt = 1;
#ifdef _OPENMP
    me = omp_get_thread_num();
    nt = omp_get_num_threads();
#pragma omp single
    ran = nt;
#endif
    uint64_t lo = n * (uint64_t)me / (uint64_t)nt, hi = n * (uint64_t)(me + 1) / (uint64_t)nt;
    uint64_t *cnt = per + (size_t)me * O_NCOUNT;
    uint64_t x[O_MAXK];
    for (uint64_t i = lo; i < hi; ++i) {
      for (int r = 0; r < k; ++r) x[r] = o_load(reps[r], dt, i);
      uint64_t c;
      uint8_t m;
      o_vote_element(dt, k, &t, x, &c, &m, cnt);
      if (consensus) o_store(consensus, dt, i, c);
      if (mask) mask[i] = m;
    }
  }
  for (int i = 0; i < O_NCOUNT; ++i) {
    counts[i] = 0;
    for (int j = 0; j < T; ++j) counts[i] += per[(size_t)j * O_NCOUNT + i];
  }
  free(per);
  o_verdict(k, counts, &vw[0], &vw[1]);
  if (used) *used = ran;
  return 0;
}

/* ---- exported: 64-bit FNV-1a over 64-bit words ----------------------------
 * The FNV-1a step xors the next input unit into the state and multiplies by
 * the FNV prime modulo 2^64; here the unit is a whole little-endian 64-bit
 * word.  With every word below 256 this is the published byte-wise FNV-1a. */
#define O_FNV_BASIS 0xcbf29ce484222325ULL
#define O_FNV_PRIME 0x00000100000001b3ULL

static uint64_t o_fnv_step(uint64_t h, uint64_t w) { return (h ^ w) * O_FNV_PRIME; }

uint64_t fto_fnv1a_words(const uint64_t *w, uint64_t count) {
  uint64_t h = O_FNV_BASIS;
  for (uint64_t i = 0; i < count; ++i) h = o_fnv_step(h, w[i]);
  return h;
}

/* word i of a byte buffer of nbytes, little-endian, zero beyond the end */
static uint64_t o_word(const unsigned char *p, uint64_t nbytes, uint64_t i) {
  uint64_t w = 0;
  for (int b = 0; b < 8; ++b) {
    uint64_t off = 8 * i + (uint64_t)b;
    uint64_t byte = off < nbytes ? p[off] : 0;
    w |= byte << (8 * b);
  }
  return w;
}

static int o_pow2(uint64_t x) { return x && !(x & (x - 1)); }

/* Fingerprint of one block: leaves are FNV-1a over 8 consecutive words (64 B);
 * the leaves are then combined pairwise -- (0,1), (2,3), ... -- level by level,
 * a node being FNV-1a over the two words (left, right), until one remains. */
static uint64_t o_block_fp(const unsigned char *p, uint64_t nbytes, uint64_t first_word,
                           uint64_t block_bytes, uint64_t *level) {
  uint64_t leaves = block_bytes / 64;
  for (uint64_t j = 0; j < leaves; ++j) {
    uint64_t w[8];
    for (int q = 0; q < 8; ++q) w[q] = o_word(p, nbytes, first_word + 8 * j + (uint64_t)q);
    level[j] = fto_fnv1a_words(w, 8);
  }
  for (uint64_t len = leaves; len > 1; len /= 2) {
    for (uint64_t j = 0; j < len / 2; ++j) {
      uint64_t pr[2] = {level[2 * j], level[2 * j + 1]};
      level[j] = fto_fnv1a_words(pr, 2);
    }
  }
  return level[0];
}

/* fp_out[b] for b < ceil(nbytes / block_bytes); block_bytes a power of two >= 64 */
int fto_fingerprint(const void *buf, uint64_t nbytes, uint64_t block_bytes, uint64_t *fp_out) {
  if (!o_pow2(block_bytes) || block_bytes < 64) return -1;
  uint64_t nblocks = (nbytes + block_bytes - 1) / block_bytes;
  uint64_t *level = (uint64_t *)malloc(sizeof(uint64_t) * (block_bytes / 64));
  if (!level) return -6;
  for (uint64_t b = 0; b < nblocks; ++b)
    fp_out[b] = o_block_fp((const unsigned char *)buf, nbytes, b * (block_bytes / 8), block_bytes,
                           level);
  free(level);
  return 0;
}

/* ---- exported: block vote with consensus restore ---------------------------
 * Per block: the fingerprints of the k replicas are voted by exact equality;
 * with a strict majority the block of the lowest-indexed replica holding the
 * majority fingerprint is copied to the consensus (recopy from a valid copy,
 * Sec. IV-A); without one, the block falls back to the element vote.
 * fps      : k * nblocks (replica-major), written
 * blockmap : nblocks bytes: bit r = replica r's fingerprint differs from the
 *            source's; bit 7 = no fingerprint majority (element fallback)
 * consensus: nbytes; mask: n bytes (0 outside fallback blocks) or NULL
 * bstats   : uint64[4 + 7]: blocks, disagree_blocks, fallback_blocks,
 *            unresolved_elems, replica_blocks[7]
 * vw       : {verdict, winner} */
int fto_vote_blocks(int dt, int k, uint64_t nbytes, const void *const *reps, int kind,
                    uint64_t max_ulp, double delta, double abs_floor, uint64_t block_bytes,
                    uint64_t *fps, uint8_t *blockmap, void *consensus, uint8_t *mask,
                    uint64_t *bstats, int32_t *vw) {
  otol t = {kind, max_ulp, delta, abs_floor};
  int rc = o_check(dt, k, &t);
  if (rc) return rc;
  uint64_t es = (uint64_t)o_size(dt);
  if (!o_pow2(block_bytes) || block_bytes < 64 || nbytes % es) return -1;
  uint64_t nblocks = (nbytes + block_bytes - 1) / block_bytes;
  for (int r = 0; r < k; ++r) {
    rc = fto_fingerprint(reps[r], nbytes, block_bytes, fps + (uint64_t)r * nblocks);
    if (rc) return rc;
  }
  for (int i = 0; i < 11; ++i) bstats[i] = 0;
  bstats[0] = nblocks;
  uint64_t cnt[O_NCOUNT];
  uint64_t x[O_MAXK];
  for (uint64_t b = 0; b < nblocks; ++b) {
    int s[O_MAXK], M = 0, src = 0;
    for (int r = 0; r < k; ++r) {
      s[r] = 0;
      for (int j = 0; j < k; ++j) s[r] += fps[(uint64_t)r * nblocks + b] == fps[(uint64_t)j * nblocks + b];
      if (s[r] > M) {
        M = s[r];
        src = r;
      }
    }
    uint8_t bm = 0;
    for (int r = 0; r < k; ++r)
      if (fps[(uint64_t)r * nblocks + b] != fps[(uint64_t)src * nblocks + b]) {
        bm |= (uint8_t)(1u << r);
        bstats[4 + r] += 1;
      }
    uint64_t lo = b * block_bytes;
    uint64_t hi = lo + block_bytes < nbytes ? lo + block_bytes : nbytes;
    if (2 * M > k) {
      memcpy((unsigned char *)consensus + lo, (const unsigned char *)reps[src] + lo, hi - lo);
      if (mask)
        for (uint64_t i = lo / es; i < hi / es; ++i) mask[i] = 0;
    } else {
      bm |= O_NOMAJ_BIT;
      bstats[2] += 1;
      for (int q = 0; q < O_NCOUNT; ++q) cnt[q] = 0;
      for (uint64_t i = lo / es; i < hi / es; ++i) {
        for (int r = 0; r < k; ++r) x[r] = o_load(reps[r], dt, i);
        uint64_t c;
        uint8_t m;
        o_vote_element(dt, k, &t, x, &c, &m, cnt);
        o_store(consensus, dt, i, c);
        if (mask) mask[i] = m;
      }
      bstats[3] += cnt[56];
    }
    if (bm & 0x7f) bstats[1] += 1;
    blockmap[b] = bm;
  }
  /* verdict */
  int clean = -1;
  for (int r = 0; r < k; ++r)
    if (bstats[4 + r] == 0) {
      clean = r;
      break;
    }
  int argmin = 0;
  for (int r = 1; r < k; ++r)
    if (bstats[4 + r] < bstats[4 + argmin]) argmin = r;
  if (bstats[1] == 0) {
    vw[0] = O_UNANIMOUS;
    vw[1] = 0;
  } else if (bstats[2] == 0 && clean >= 0) {
    vw[0] = O_TASK_MAJORITY;
    vw[1] = clean;
  } else if (bstats[3] == 0) {
    vw[0] = O_ELEMENT_MAJORITY;
    vw[1] = argmin;
  } else {
    vw[0] = O_UNRESOLVED;
    vw[1] = argmin;
  }
  return 0;
}

/* ---- exported: fault-aware runtime (Sec. IV-B) -----------------------------
 * p = 1 - v/t is the fault probability of a unit with v valid runs out of t;
 * F = R / (1 - p) = R * (t / v): the fault-free runtime scaled by the
 * expected number of runs until one is valid.  No history (t = 0): F = R.
 * v = 0 < t: p = 1, F = +infinity. */
double fto_fault_aware_runtime(double R, uint64_t v, uint64_t t) {
  if (t == 0) return R;
  if (v == 0) return INFINITY;
  return R * ((double)t / (double)v);
}
