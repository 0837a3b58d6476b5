// ftv_host.cpp -- the voter on the host's cores.
//
// The paper's runtime holds the voter as kernels for several processing
// units -- a single-threaded one, an OpenMP one and a GPU one -- and picks
// among them by data size and by where the results lie (Kicherer & Karl,
// Sec. V-A, Fig. 3; the voter is a task like any other, Sec. IV-D).  This is
// the host side of that set: the same element vote as the MI355X kernels
// (same tolerance test, majority rule, tie-break, mask, counts and verdict),
// written for a CPU core, on one thread or split over OpenMP threads.  Its
// results are bit-identical to the device voter's; it is a unit that the
// placement below chooses by measured time, never a stand-in for a missing
// GPU.
//
// Per element the common case is that every replica holds the same bit
// pattern: one compare per replica, the pattern is the consensus, nothing is
// counted.  Otherwise the k x k tolerance relation is built as one bit row
// per replica; supports are the rows' popcounts, the candidates are the
// replicas of maximal support and the consensus is their lower median under
// the total order of the raw bits.  Counts are per thread and summed after
// the parallel region (integers, so the order of the sum does not matter).
#include <omp.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "ftv.h"
#include "ftv_common.hpp"

using namespace ftv;

namespace {

template <int DT>
struct HT;
template <>
struct HT<FTV_F32> {
  using W = uint32_t;
  static constexpr bool FL = true;
  static constexpr W SIGN = 0x80000000u, MAG = 0x7fffffffu, INF = 0x7f800000u;
  static double value(W x) {
    float f;
    memcpy(&f, &x, 4);
    return (double)f;
  }
};
template <>
struct HT<FTV_F64> {
  using W = uint64_t;
  static constexpr bool FL = true;
  static constexpr W SIGN = 0x8000000000000000ull, MAG = 0x7fffffffffffffffull, INF = 0x7ff0000000000000ull;
  static double value(W x) {
    double d;
    memcpy(&d, &x, 8);
    return d;
  }
};
template <>
struct HT<FTV_I32> {
  using W = uint32_t;
  static constexpr bool FL = false;
  static constexpr W SIGN = 0x80000000u;
};
template <>
struct HT<FTV_I64> {
  using W = uint64_t;
  static constexpr bool FL = false;
  static constexpr W SIGN = 0x8000000000000000ull;
};

struct HTol {
  uint64_t max_ulp;  // clamped to the width of the value type
  double delta;
  double abs_floor;
};

// Tolerance relation between two bit patterns.
template <int DT, int TOL>
inline bool host_eq(typename HT<DT>::W a, typename HT<DT>::W b, const HTol &t) {
  using T = HT<DT>;
  using W = typename T::W;
  if (a == b) return true;
  if constexpr (!T::FL || TOL == FTV_TOL_EXACT) {
    return false;
  } else {
    const W ma = a & T::MAG, mb = b & T::MAG;
    if (ma > T::INF || mb > T::INF) return ma > T::INF && mb > T::INF;  // NaN equals only NaN
    if (ma == T::INF || mb == T::INF) return false;  // an infinity only itself (a != b here)
    if constexpr (TOL == FTV_TOL_ULP) {
      // the ordered line of finite values: -max .. -0 = +0 .. +max, shifted to unsigned
      const W ka = (a & T::SIGN) ? (W)(T::SIGN - ma) : (W)(ma | T::SIGN);
      const W kb = (b & T::SIGN) ? (W)(T::SIGN - mb) : (W)(mb | T::SIGN);
      const W dist = ka > kb ? ka - kb : kb - ka;
      return (uint64_t)dist <= t.max_ulp;
    } else {
      if ((ma | mb) == 0) return true;  // +0 and -0
      const double x = T::value(a), y = T::value(b);
      double diff = x - y;
      if (diff < 0) diff = -diff;
      const double ax = x < 0 ? -x : x, ay = y < 0 ? -y : y;
      const double big = ax > ay ? ax : ay;
      const double lim = t.delta * big;
      return diff <= lim || diff <= t.abs_floor;
    }
  }
}

// Unsigned key of the total order of bit patterns (IEEE-754 totalOrder for
// floats, two's-complement order for integers).
template <int DT>
inline typename HT<DT>::W host_order(typename HT<DT>::W x) {
  using T = HT<DT>;
  if constexpr (T::FL) return (x & T::SIGN) ? (typename T::W)~x : (typename T::W)(x | T::SIGN);
  else return x ^ T::SIGN;
}

// Counts of one thread: pairs (i < j) in row-major upper-triangle order, then
// per-replica disagreements, then elements without a majority.
struct HCounts {
  uint64_t pair[FTV_MAX_K][FTV_MAX_K];
  uint64_t disagree[FTV_MAX_K];
  uint64_t nomaj;
};

template <int DT, int TOL, int K>
void host_range(const ftv_vote_desc &d, const HTol &t, uint64_t lo, uint64_t hi, HCounts &c) {
  using W = typename HT<DT>::W;
  const W *rep[K];
  for (int r = 0; r < K; ++r) rep[r] = static_cast<const W *>(d.replicas[r]);
  W *cons = static_cast<W *>(d.consensus);
  uint8_t *mask = d.mask;
  constexpr uint32_t ALL = (1u << K) - 1u;
  for (uint64_t i = lo; i < hi; ++i) {
    W x[K];
    bool same = true;
    for (int r = 0; r < K; ++r) {
      x[r] = rep[r][i];
      same &= x[r] == x[0];
    }
    if (same) {
      if (cons) cons[i] = x[0];
      if (mask) mask[i] = 0;
      continue;
    }
    uint32_t row[K];
    for (int r = 0; r < K; ++r) row[r] = 1u << r;
    for (int a = 0; a < K; ++a)
      for (int b = a + 1; b < K; ++b) {
        if (host_eq<DT, TOL>(x[a], x[b], t)) {
          row[a] |= 1u << b;
          row[b] |= 1u << a;
        } else {
          c.pair[a][b]++;
        }
      }
    int best = 0;
    for (int r = 0; r < K; ++r) best = std::max(best, __builtin_popcount(row[r]));
    // candidates ordered by their key; the lower median is the consensus
    int cand[K];
    W ckey[K];
    int nc = 0;
    for (int r = 0; r < K; ++r) {
      if (__builtin_popcount(row[r]) != best) continue;
      const W key = host_order<DT>(x[r]);
      int p = nc++;
      while (p > 0 && ckey[p - 1] > key) {
        ckey[p] = ckey[p - 1];
        cand[p] = cand[p - 1];
        --p;
      }
      ckey[p] = key;
      cand[p] = r;
    }
    const int pick = cand[(nc - 1) / 2];
    const uint32_t off = ~row[pick] & ALL;  // replicas outside the tolerance of the consensus
    const bool nomaj = 2 * best <= K;
    if (cons) cons[i] = x[pick];
    if (mask) mask[i] = (uint8_t)(off | (nomaj ? 0x80u : 0u));
    for (int r = 0; r < K; ++r) c.disagree[r] += (off >> r) & 1u;
    c.nomaj += nomaj;
  }
}

// Stats record from the summed counts: the verdict ladder and its winner.
void host_finish(const HCounts &c, uint32_t k, uint64_t n, ftv_stats *st) {
  memset(st, 0, sizeof(*st));
  bool unanimous = true;
  for (uint32_t a = 0; a < k; ++a)
    for (uint32_t b = a + 1; b < k; ++b) {
      st->pair[a][b] = st->pair[b][a] = c.pair[a][b];
      unanimous &= c.pair[a][b] == 0;
    }
  int top = 0, topT = -1, fewest = 0;
  for (uint32_t r = 0; r < k; ++r) {
    st->disagree[r] = c.disagree[r];
    int T = 0;  // replicas agreeing with r on every element, r included
    for (uint32_t j = 0; j < k; ++j) T += st->pair[r][j] == 0;
    if (T > topT) {
      topT = T;
      top = (int)r;
    }
    if (c.disagree[r] < c.disagree[fewest]) fewest = (int)r;
  }
  st->no_majority = c.nomaj;
  st->n = n;
  if (unanimous) {
    st->verdict = FTV_UNANIMOUS;
    st->winner = 0;
  } else if (2 * topT > (int)k) {
    st->verdict = FTV_TASK_MAJORITY;
    st->winner = top;
  } else {
    st->verdict = c.nomaj == 0 ? FTV_ELEMENT_MAJORITY : FTV_UNRESOLVED;
    st->winner = fewest;
  }
}

// Elements per thread at least: a thread then votes for about 6 us (4096 fp32
// elements of k = 3 on one core), more than the fork and join of the team;
// with fewer, a team of one thread per core costs more than it saves and is
// exposed to the scheduler time slices of the process's other threads (a
// 16 KiB vote on 16 threads once measured about 1 ms, against 6 us on one).
constexpr uint64_t kMinPerThread = 4096;

template <int DT, int TOL, int K>
void host_vote_k(const ftv_vote_desc &d, const HTol &t, int threads, HCounts &total) {
  memset(&total, 0, sizeof(total));
  const uint64_t most = (d.n + kMinPerThread - 1) / kMinPerThread;
  if ((uint64_t)threads > most) threads = (int)most;
  if (threads <= 1 || d.n < 2) {
    host_range<DT, TOL, K>(d, t, 0, d.n, total);
    return;
  }
  std::vector<HCounts> per((size_t)threads);
  memset(per.data(), 0, per.size() * sizeof(HCounts));
  int used = 1;
#pragma omp parallel num_threads(threads)
  {
    const int me = omp_get_thread_num(), nt = omp_get_num_threads();
#pragma omp single
    used = nt;
    // contiguous ranges, split at 64-element boundaries
    const uint64_t units = (d.n + 63) / 64;
    const uint64_t lo = std::min(d.n, units * (uint64_t)me / (uint64_t)nt * 64);
    const uint64_t hi = std::min(d.n, units * (uint64_t)(me + 1) / (uint64_t)nt * 64);
    host_range<DT, TOL, K>(d, t, lo, hi, per[(size_t)me]);
  }
  for (int q = 0; q < used; ++q) {
    const HCounts &p = per[(size_t)q];
    for (int a = 0; a < FTV_MAX_K; ++a)
      for (int b = 0; b < FTV_MAX_K; ++b) total.pair[a][b] += p.pair[a][b];
    for (int r = 0; r < FTV_MAX_K; ++r) total.disagree[r] += p.disagree[r];
    total.nomaj += p.nomaj;
  }
}

template <int DT, int TOL>
void host_vote_tol(const ftv_vote_desc &d, const HTol &t, int threads, HCounts &c) {
  switch (d.k) {
    case 2: return host_vote_k<DT, TOL, 2>(d, t, threads, c);
    case 3: return host_vote_k<DT, TOL, 3>(d, t, threads, c);
    case 4: return host_vote_k<DT, TOL, 4>(d, t, threads, c);
    case 5: return host_vote_k<DT, TOL, 5>(d, t, threads, c);
    case 6: return host_vote_k<DT, TOL, 6>(d, t, threads, c);
    default: return host_vote_k<DT, TOL, 7>(d, t, threads, c);
  }
}

}  // namespace

namespace ftv {

// Threads the host voter uses for `threads` (0 = every core the process may use).
int host_threads(uint32_t threads) {
  if (threads == 0) return std::max(1, omp_get_num_procs());
  return (int)std::min<uint32_t>(threads, 1024);
}

}  // namespace ftv

extern "C" {

int ftv_vote_host(const ftv_vote_desc *d, uint32_t threads) {
  if (!d) return fail(FTV_E_INVALID, "NULL descriptor");
  if (d->k < 2 || d->k > FTV_MAX_K) return fail(FTV_E_K, "k must be in [2, 7]");
  int rc = check_tol(d->dtype, d->tol);
  if (rc) return rc;
  if (!d->stats) return fail(FTV_E_INVALID, "stats pointer is NULL");
  const uint64_t es = (uint64_t)elem_size(d->dtype);
  if ((uintptr_t)d->stats % 8) return fail(FTV_E_ALIGN, "stats must be 8-byte aligned");
  for (uint32_t r = 0; r < d->k; ++r) {
    if (!d->replicas[r] && d->n) return fail(FTV_E_INVALID, "replica pointer is NULL");
    if ((uintptr_t)d->replicas[r] % es) return fail(FTV_E_ALIGN, "replica not element-aligned");
  }
  if (d->consensus && (uintptr_t)d->consensus % es) return fail(FTV_E_ALIGN, "consensus not element-aligned");
  rc = check_vote_overlaps(d);  // the same rule as the device voter's
  if (rc) return rc;
  const TolD td = to_tol_d(d->dtype, d->tol);
  const HTol t{td.max_ulp, td.delta, td.abs_floor};
  const int T = host_threads(threads);
  HCounts c;
  switch (d->dtype * 3 + d->tol.kind) {
    case FTV_F32 * 3 + FTV_TOL_EXACT: host_vote_tol<FTV_F32, FTV_TOL_EXACT>(*d, t, T, c); break;
    case FTV_F32 * 3 + FTV_TOL_ULP: host_vote_tol<FTV_F32, FTV_TOL_ULP>(*d, t, T, c); break;
    case FTV_F32 * 3 + FTV_TOL_REL: host_vote_tol<FTV_F32, FTV_TOL_REL>(*d, t, T, c); break;
    case FTV_F64 * 3 + FTV_TOL_EXACT: host_vote_tol<FTV_F64, FTV_TOL_EXACT>(*d, t, T, c); break;
    case FTV_F64 * 3 + FTV_TOL_ULP: host_vote_tol<FTV_F64, FTV_TOL_ULP>(*d, t, T, c); break;
    case FTV_F64 * 3 + FTV_TOL_REL: host_vote_tol<FTV_F64, FTV_TOL_REL>(*d, t, T, c); break;
    case FTV_I32 * 3 + FTV_TOL_EXACT: host_vote_tol<FTV_I32, FTV_TOL_EXACT>(*d, t, T, c); break;
    case FTV_I64 * 3 + FTV_TOL_EXACT: host_vote_tol<FTV_I64, FTV_TOL_EXACT>(*d, t, T, c); break;
    default: return fail(FTV_E_DTYPE, "tolerance kind not valid for this type");
  }
  host_finish(c, d->k, d->n, d->stats);
  return FTV_OK;
}

}  // extern "C"
