// ftv_vote_dev.hpp -- device-side element vote for gfx950 (wave64).
//
// The voter compares the k results of a duplicated task element by element
// (Kicherer & Karl, Sec. IV-D): integer values bit-wise, floating-point values
// within a programmer-set tolerance.  Each element's consensus is chosen among
// the replicas of maximal support (a strict majority when 2M > k), ties broken
// by the lower median under IEEE-754 totalOrder of the raw bits, so the result
// does not depend on the order of the replicas.
//
// Layout of the hot loop: every lane streams one 16-byte vector of each of the
// k replicas per step (global_load_dwordx4, non-temporal), votes the 4 (fp32,
// i32) or 2 (fp64, i64) elements in registers, and writes one 16-byte
// consensus vector and 4 or 2 mask bytes.  Mismatch counting is done only in
// waves where some lane saw a disagreement: into per-lane counters folded once
// per workgroup (the per-task kernel) or with ballots into wave-uniform
// (scalar) accumulators (the batched and block kernels, where registers are
// scarcer and disagreements rare).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ftv_internal.hpp"

namespace ftv {
namespace dev {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int DT>
struct VT;
template <>
struct VT<FTV_F32> {
  using W = uint32_t;
  using S = int32_t;
  static constexpr bool FL = true;
  static constexpr W SIGN = 0x80000000u;
  static constexpr W MAG = 0x7fffffffu;
  static constexpr W INF = 0x7f800000u;
};
template <>
struct VT<FTV_F64> {
  using W = uint64_t;
  using S = int64_t;
  static constexpr bool FL = true;
  static constexpr W SIGN = 0x8000000000000000ull;
  static constexpr W MAG = 0x7fffffffffffffffull;
  static constexpr W INF = 0x7ff0000000000000ull;
};
template <>
struct VT<FTV_I32> {
  using W = uint32_t;
  using S = int32_t;
  static constexpr bool FL = false;
  static constexpr W SIGN = 0x80000000u;
  static constexpr W MAG = 0x7fffffffu;
  static constexpr W INF = 0;
};
template <>
struct VT<FTV_I64> {
  using W = uint64_t;
  using S = int64_t;
  static constexpr bool FL = false;
  static constexpr W SIGN = 0x8000000000000000ull;
  static constexpr W MAG = 0x7fffffffffffffffull;
  static constexpr W INF = 0;
};

template <typename W>
__device__ __forceinline__ W umin(W a, W b) { return a < b ? a : b; }
template <typename W>
__device__ __forceinline__ W umax(W a, W b) { return a < b ? b : a; }

__device__ __forceinline__ double as_double(uint32_t x) { return (double)__uint_as_float(x); }
__device__ __forceinline__ double as_double(uint64_t x) { return __longlong_as_double((long long)x); }

// Per-replica quantities reused by every pair that replica is part of.
template <int DT, int TOL>
struct Pre {
  using W = typename VT<DT>::W;
  using S = typename VT<DT>::S;
  W bits;
  W mag;
  S key;       // signed-magnitude bits as two's complement: adjacent floats differ by 1
  double val;  // REL only
};

template <int DT, int TOL>
__device__ __forceinline__ Pre<DT, TOL> prep(typename VT<DT>::W x) {
  using T = VT<DT>;
  using S = typename T::S;
  Pre<DT, TOL> p;
  p.bits = x;
  if constexpr (T::FL && TOL != FTV_TOL_EXACT) {
    p.mag = x & T::MAG;
    p.key = (x & T::SIGN) ? -(S)p.mag : (S)p.mag;
    if constexpr (TOL == FTV_TOL_REL) p.val = as_double(x);
  }
  return p;
}

// The voter's equality: bit-wise for integers and EXACT; otherwise NaN equals
// any NaN, an infinity only the same infinity, and finite values within the
// tolerance (ULP: key distance; REL: binary64 relative test, no FMA).  Written
// without early exits so that it compiles to selects, not branches.
template <int DT, int TOL>
__device__ __forceinline__ bool eqp(const Pre<DT, TOL> &a, const Pre<DT, TOL> &b, const TolD &t) {
  using T = VT<DT>;
  using W = typename T::W;
  if constexpr (!T::FL || TOL == FTV_TOL_EXACT) {
    return a.bits == b.bits;
  } else {
    const bool an = a.mag > T::INF, bn = b.mag > T::INF;
    const bool fin = (a.mag < T::INF) & (b.mag < T::INF);
    bool within;
    if constexpr (TOL == FTV_TOL_ULP) {
      // keys biased by 2^(w-1) into unsigned range: the distance is |ua - ub|
      const W ua = (a.bits & T::SIGN) ? (W)(T::SIGN - a.mag) : (a.mag | T::SIGN);
      const W ub = (b.bits & T::SIGN) ? (W)(T::SIGN - b.mag) : (b.mag | T::SIGN);
      within = (umax(ua, ub) - umin(ua, ub)) <= (W)t.max_ulp;
    } else {
      const double d = __builtin_fabs(__dsub_rn(a.val, b.val));
      const double m = __builtin_fmax(__builtin_fabs(a.val), __builtin_fabs(b.val));
      const double lim = __dmul_rn(t.delta, m);
      within = ((a.mag | b.mag) == 0) | (d <= lim) | (d <= t.abs_floor);
    }
    return (a.bits == b.bits) | (an & bn) | (fin & within);
  }
}

template <int DT, int TOL>
__device__ __forceinline__ bool eqv(typename VT<DT>::W a, typename VT<DT>::W b, const TolD &t) {
  return eqp<DT, TOL>(prep<DT, TOL>(a), prep<DT, TOL>(b), t);
}

// Unsigned key of IEEE-754 totalOrder (floats) or two's-complement order
// (integers), and its inverse.
template <int DT>
__device__ __forceinline__ typename VT<DT>::W okey(typename VT<DT>::W x) {
  using T = VT<DT>;
  if constexpr (T::FL) return (x & T::SIGN) ? ~x : (x | T::SIGN);
  else return x ^ T::SIGN;
}
template <int DT>
__device__ __forceinline__ typename VT<DT>::W okey_inv(typename VT<DT>::W k) {
  using T = VT<DT>;
  if constexpr (T::FL) return (k & T::SIGN) ? (k ^ T::SIGN) : ~k;
  else return k ^ T::SIGN;
}


// Result of voting one element: consensus bits, mask byte, and the set of
// unequal replica pairs (bit p for pair p in (0,1),(0,2),..,(1,2),.. order).
template <typename W>
struct ElemOut {
  W cons;
  uint32_t mb;
  uint32_t ne;
};

template <int K>
struct NPair {
  static constexpr int value = K * (K - 1) / 2;
};

// k = 3 when the three bit patterns may all differ: the case analysis on the
// number of agreeing pairs (3 or 0: median; 2: the replica agreeing with both;
// 1: the smaller key of the agreeing pair).
template <int DT>
__device__ __forceinline__ typename VT<DT>::W vote3_general(const typename VT<DT>::W (&x)[3],
                                                            uint32_t ne, uint32_t &mb_out) {
  using W = typename VT<DT>::W;
  const bool e01 = !(ne & 1u), e02 = !(ne & 2u), e12 = !(ne & 4u);
  const int cnt = (int)e01 + (int)e02 + (int)e12;
  const W k0 = okey<DT>(x[0]), k1 = okey<DT>(x[1]), k2 = okey<DT>(x[2]);
  const W med = umax(umin(k0, k1), umin(umax(k0, k1), k2));
  const W pairmin = e01 ? umin(k0, k1) : (e02 ? umin(k0, k2) : umin(k1, k2));
  const W vertex = !e01 ? k2 : (!e02 ? k1 : k0);
  const W kc = cnt == 1 ? pairmin : (cnt == 2 ? vertex : med);
  const uint32_t cmed = (k0 == med) ? 0u : ((k1 == med) ? 1u : 2u);
  const uint32_t odd = e01 ? 4u : (e02 ? 2u : 1u);
  mb_out = cnt == 1 ? odd : (cnt == 0 ? (0x80u | (7u & ~(1u << cmed))) : 0u);
  return okey_inv<DT>(kc);
}

// Bit mask of the replica pairs (0,1),(0,2),..,(1,2),.. that involve replica r.
template <int K>
__device__ __forceinline__ uint32_t pairs_of(uint32_t r) {
  uint32_t m = 0;
  int q = 0;
#pragma unroll
  for (int i = 0; i < K; ++i)
#pragma unroll
    for (int j = i + 1; j < K; ++j, ++q) m |= (uint32_t)((uint32_t)i == r || (uint32_t)j == r) << q;
  return m;
}

template <int DT, int TOL, int K>
__device__ __forceinline__ ElemOut<typename VT<DT>::W> vote_general(const typename VT<DT>::W (&x)[K],
                                                                    const TolD &t);

// k >= 3.  If all replicas but at most one hold the same bit pattern m, then m
// is the consensus whatever the odd replica holds: with the odd one equal to m
// (under the tolerance) all k replicas are candidates and k-1 of them hold m,
// so the lower median is m; otherwise the k-1 copies of m are the only
// candidates.  Either way 2(k-1) > k is a majority.  One tolerance test, odd
// replica against m, decides the element; elements with two or more differing
// bit patterns take the general computation.
template <int DT, int TOL, int K>
__device__ __forceinline__ ElemOut<typename VT<DT>::W> vote_fast(const typename VT<DT>::W (&x)[K],
                                                                 const TolD &t, bool &general) {
  using W = typename VT<DT>::W;
  ElemOut<W> o;
  // with at most one outlier, two of the first three replicas hold m
  const W m = (x[0] == x[1] || x[0] == x[2]) ? x[0] : x[1];
  uint32_t nd = 0, odd = 0;
  W xo = m;
#pragma unroll
  for (int r = 0; r < K; ++r) {
    const bool d = x[r] != m;
    nd += d ? 1u : 0u;
    odd = d ? (uint32_t)r : odd;
    xo = d ? x[r] : xo;
  }
  const bool e = eqv<DT, TOL>(xo, m, t);  // true when nothing differs
  o.cons = m;
  o.mb = e ? 0u : (1u << odd);
  o.ne = e ? 0u : pairs_of<K>(odd);
  general = nd > 1u;
  return o;
}

// General k: supports, candidate set, lower median of the candidates by key.
// Recomputes keys instead of keeping per-replica arrays, to stay small in
// registers: it only runs for elements with two or more differing patterns.
template <int DT, int TOL, int K>
__device__ __forceinline__ ElemOut<typename VT<DT>::W> vote_general(const typename VT<DT>::W (&x)[K],
                                                                    const TolD &t) {
  using W = typename VT<DT>::W;
  uint32_t adj[K];
#pragma unroll
  for (int r = 0; r < K; ++r) adj[r] = 1u << r;
  uint32_t ne = 0;
  int q = 0;
#pragma unroll
  for (int r = 0; r < K; ++r) {
#pragma unroll
    for (int j = r + 1; j < K; ++j, ++q) {
      const bool e = eqv<DT, TOL>(x[r], x[j], t);
      adj[r] |= (uint32_t)e << j;
      adj[j] |= (uint32_t)e << r;
      ne |= (uint32_t)(!e) << q;
    }
  }
  ElemOut<W> o;
  o.ne = ne;
  if constexpr (K == 2) {
    // supports are 2,2 (agree) or 1,1 (disagree); either way both replicas
    // are candidates and the lower median of two is the smaller key.  On a
    // disagreement the other replica is flagged and there is no majority.
    const W k0 = okey<DT>(x[0]), k1 = okey<DT>(x[1]);
    o.cons = okey_inv<DT>(umin(k0, k1));
    o.mb = ne ? (0x80u | (k0 < k1 ? 2u : 1u)) : 0u;
  } else {
    int M = 0;
#pragma unroll
    for (int r = 0; r < K; ++r) M = __popc(adj[r]) > M ? __popc(adj[r]) : M;
    uint32_t cm = 0;
#pragma unroll
    for (int r = 0; r < K; ++r) cm |= (uint32_t)(__popc(adj[r]) == M) << r;
    const int target = (__popc(cm) - 1) >> 1;
    W cv = x[0];
    uint32_t ac = adj[0];
#pragma unroll
    for (int r = 0; r < K; ++r) {
      const W kr = okey<DT>(x[r]);
      int rank = 0;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const W kj = okey<DT>(x[j]);
        rank += (int)(((cm >> j) & 1u) && (kj < kr || (kj == kr && j < r)));
      }
      if (((cm >> r) & 1u) && rank == target) {
        cv = x[r];
        ac = adj[r];
      }
    }
    o.cons = cv;
    o.mb = (~ac & ((1u << K) - 1u)) | (2 * M > K ? 0u : 0x80u);
  }
  return o;
}

// rep[r] for a runtime r as a select chain over the seven slots: indexing a
// by-value record with a runtime index would move it to scratch memory.
__device__ __forceinline__ const void *rep_sel(const void *const (&rep)[FTV_MAX_K], int r) {
  const void *p = rep[0];
#pragma unroll
  for (int j = 1; j < FTV_MAX_K; ++j) p = (j == r) ? rep[j] : p;
  return p;
}

// General vote of element i for a runtime k (4..7): the same definition as
// vote_general, with loops that are not unrolled, the support relation packed
// into one 64-bit word (bit 8r+j = eq(x_r, x_j)) and replica values re-read
// from memory when needed, so that the rare elements that need it cost
// registers only for their own duration.
template <int DT, int TOL>
__device__ __forceinline__ ElemOut<typename VT<DT>::W> vote_general_dyn(
    const void *const (&rep)[FTV_MAX_K], int k, uint64_t i, const TolD &t) {
  using W = typename VT<DT>::W;
  auto X = [&](int r) -> W { return reinterpret_cast<const W *>(rep_sel(rep, r))[i]; };
  uint64_t A = 0;
  uint32_t ne = 0;
  int q = 0;
#pragma unroll 1
  for (int r = 0; r < k; ++r) {
    const W xr = X(r);
    A |= 1ull << (8 * r + r);
#pragma unroll 1
    for (int j = r + 1; j < k; ++j, ++q) {
      if (eqv<DT, TOL>(xr, X(j), t)) A |= (1ull << (8 * r + j)) | (1ull << (8 * j + r));
      else ne |= 1u << q;
    }
  }
  int M = 0;
#pragma unroll 1
  for (int r = 0; r < k; ++r) {
    const int sr = __popcll((A >> (8 * r)) & 0xffull);
    M = sr > M ? sr : M;
  }
  uint32_t cm = 0;
#pragma unroll 1
  for (int r = 0; r < k; ++r) cm |= (uint32_t)(__popcll((A >> (8 * r)) & 0xffull) == M) << r;
  const int target = (__popc(cm) - 1) >> 1;
  int c = 0;
#pragma unroll 1
  for (int r = 0; r < k; ++r) {
    if (!((cm >> r) & 1u)) continue;
    const W kr = okey<DT>(X(r));
    int rank = 0;
#pragma unroll 1
    for (int j = 0; j < k; ++j) {
      if (!((cm >> j) & 1u)) continue;
      const W kj = okey<DT>(X(j));
      rank += (int)(kj < kr || (kj == kr && j < r));
    }
    if (rank == target) c = r;
  }
  ElemOut<W> o;
  o.cons = X(c);
  o.mb = ((uint32_t)~(A >> (8 * c)) & ((1u << k) - 1u)) | (2 * M > k ? 0u : 0x80u);
  o.ne = ne;
  return o;
}

// k = 3 with three differing bit patterns: the three tolerance tests and the
// case analysis.
template <int DT, int TOL>
__device__ __forceinline__ ElemOut<typename VT<DT>::W> vote3_slow(const typename VT<DT>::W (&x)[3],
                                                                  const TolD &t) {
  ElemOut<typename VT<DT>::W> o;
  const uint32_t ne = (uint32_t)!eqv<DT, TOL>(x[0], x[1], t) | ((uint32_t)!eqv<DT, TOL>(x[0], x[2], t) << 1) |
                      ((uint32_t)!eqv<DT, TOL>(x[1], x[2], t) << 2);
  o.ne = ne;
  o.cons = vote3_general<DT>(x, ne, o.mb);
  return o;
}

// Elements with two or more differing bit patterns (k >= 3).
template <int DT, int TOL, int K>
__device__ __forceinline__ ElemOut<typename VT<DT>::W> vote_slow(const typename VT<DT>::W (&x)[K],
                                                                 const TolD &t,
                                                                 const void *const (&rep)[FTV_MAX_K],
                                                                 uint64_t i) {
  if constexpr (K == 3) {
    return vote3_slow<DT, TOL>(x, t);
  } else {
    return vote_general_dyn<DT, TOL>(rep, K, i, t);
  }
}

// Vote of one element.  k = 2 is one tolerance test; k >= 3 takes the
// at-most-one-outlier form and falls back to the general computation.
template <int DT, int TOL, int K>
__device__ __forceinline__ ElemOut<typename VT<DT>::W> vote_elem(const typename VT<DT>::W (&x)[K],
                                                                 const TolD &t,
                                                                 const void *const (&rep)[FTV_MAX_K],
                                                                 uint64_t i) {
  if constexpr (K == 2) {
    return vote_general<DT, TOL, 2>(x, t);
  } else {
    bool general;
    ElemOut<typename VT<DT>::W> o = vote_fast<DT, TOL, K>(x, t, general);
    if (general) o = vote_slow<DT, TOL, K>(x, t, rep, i);
    return o;
  }
}

// Wave-uniform mismatch accumulators: pair[NP], disagree[K], no_majority.
template <int K>
struct Acc {
  static constexpr int NP = NPair<K>::value;
  static constexpr int NC = NP + K + 1;
  static constexpr bool kLane = false;
  uint64_t c[NC];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < NC; ++i) c[i] = 0;
  }
  // Count one element per lane; `valid` masks lanes past the end.
  __device__ __forceinline__ void add(bool valid, uint32_t ne, uint32_t mb) {
    if (__ballot(valid && ne != 0u) == 0ull) return;  // wave-uniform
#pragma unroll
    for (int q = 0; q < NP; ++q) c[q] += __popcll(__ballot(valid && ((ne >> q) & 1u)));
#pragma unroll
    for (int r = 0; r < K; ++r) c[NP + r] += __popcll(__ballot(valid && ((mb >> r) & 1u)));
    c[NP + K] += __popcll(__ballot(valid && (mb & 0x80u)));
  }
};

// The same counts with a per-lane stage: in a wave where some lane saw a
// mismatch, each counter takes one 32-bit add per lane (no ballot, no scalar
// dependency chain), and fold() sums the lanes into the wave-uniform 64-bit
// counters once, before the workgroup total.  Waves without a mismatch skip
// the adds as in Acc.  When most elements disagree (a corrupted replica, or
// float replicas under EXACT) the ballot chain of Acc, with one wave per SIMD,
// is what limits the kernel.  A lane's 32-bit counters hold at most the
// elements that lane votes between folds.
template <int K>
struct LaneAcc {
  static constexpr int NP = NPair<K>::value;
  static constexpr int NC = NP + K + 1;
  static constexpr bool kLane = true;
  uint64_t c[NC];
  uint32_t l[NC];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      c[i] = 0;
      l[i] = 0;
    }
  }
  __device__ __forceinline__ void add(bool valid, uint32_t ne, uint32_t mb) {
    if (__ballot(valid && ne != 0u) == 0ull) return;  // wave-uniform
    const uint32_t e = valid ? ne : 0u, m = valid ? mb : 0u;
#pragma unroll
    for (int q = 0; q < NP; ++q) l[q] += (e >> q) & 1u;
#pragma unroll
    for (int r = 0; r < K; ++r) l[NP + r] += (m >> r) & 1u;
    l[NP + K] += (m >> 7) & 1u;
  }
  // Called by every lane of the wave.  A wave that counted nothing (most
  // waves of a clean task) skips the reductions: they are a chain of
  // cross-lane steps that a short kernel would otherwise wait for.
  __device__ __forceinline__ void fold() {
    uint32_t any = 0;
#pragma unroll
    for (int i = 0; i < NC; ++i) any |= l[i];
    if (__ballot(any != 0u) == 0ull) return;  // wave-uniform
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      uint32_t v = l[i];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      c[i] += v;
      l[i] = 0;
    }
  }
};

// ---- 16-byte vector <-> words ---------------------------------------------
template <typename W>
struct Vec;
template <>
struct Vec<uint32_t> {
  static constexpr int V = 4;
  __device__ __forceinline__ static void unpack(u32x4 v, uint32_t (&w)[4]) {
    w[0] = v.x;
    w[1] = v.y;
    w[2] = v.z;
    w[3] = v.w;
  }
  __device__ __forceinline__ static u32x4 pack(const uint32_t (&w)[4]) {
    u32x4 v;
    v.x = w[0];
    v.y = w[1];
    v.z = w[2];
    v.w = w[3];
    return v;
  }
};
template <>
struct Vec<uint64_t> {
  static constexpr int V = 2;
  __device__ __forceinline__ static void unpack(u32x4 v, uint64_t (&w)[2]) {
    w[0] = (uint64_t)v.x | ((uint64_t)v.y << 32);
    w[1] = (uint64_t)v.z | ((uint64_t)v.w << 32);
  }
  __device__ __forceinline__ static u32x4 pack(const uint64_t (&w)[2]) {
    u32x4 v;
    v.x = (uint32_t)w[0];
    v.y = (uint32_t)(w[0] >> 32);
    v.z = (uint32_t)w[1];
    v.w = (uint32_t)(w[1] >> 32);
    return v;
  }
};

__device__ __forceinline__ u32x4 ld16(const void *base, uint64_t vi) {
  return __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(base) + vi);
}
__device__ __forceinline__ void st16(void *base, uint64_t vi, u32x4 v, bool nt) {
  u32x4 *p = reinterpret_cast<u32x4 *>(base) + vi;
  if (nt) __builtin_nontemporal_store(v, p);
  else *p = v;
}
template <typename T>
__device__ __forceinline__ void st_nt(T *p, T v, bool nt) {
  if (nt) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Streaming output stores of the vector path: non-temporal at agent scope
// (nt sc1), so that the consensus and mask vectors, written once and never
// read back by the kernel, are written through the XCD's L2 instead of being
// written back later while the replica reads are streaming.  They are buffer
// stores against a resource based at the step's first vector, so the 32-bit
// offset covers any task size.
constexpr int kStreamStorePolicy = 2 | 16;  // nt | sc1

__device__ __forceinline__ __amdgpu_buffer_rsrc_t stream_rsrc(uintptr_t base) {
  return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void *>(base), (short)0, 0x7fffffff,
                                           0x00020000);
}
// One streaming store at byte offset `off` from a workgroup-uniform base.
__device__ __forceinline__ void stream_store16(uintptr_t base, uint32_t off, u32x4 v) {
  __builtin_amdgcn_raw_buffer_store_b128(v, stream_rsrc(base), off, 0, kStreamStorePolicy);
}
__device__ __forceinline__ void stream_store8(uintptr_t base, uint32_t off, uint64_t v) {
  typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
  const u32x2 w = {(uint32_t)v, (uint32_t)(v >> 32)};
  __builtin_amdgcn_raw_buffer_store_b64(w, stream_rsrc(base), off, 0, kStreamStorePolicy);
}

// The votes of the V elements of one vector (x[r][e]: element e of replica
// r).  k = 2: one tolerance test each.  k >= 3: the at-most-one-outlier form;
// the elements with more differing patterns are then voted in place from the
// registers (one wave-uniform branch per vector, taken only when some lane
// has such an element) for k = 3, and for k >= 4 when INL; otherwise they are
// returned as bits for the fix-up pass, which reloads each element and keeps
// the general vote out of the streaming registers (the batched kernel, whose
// register budget is that of its largest specialization).  With one replica
// corrupted and rounding noise between the others most elements have three
// patterns: the fix-up pass then took 3.7 ms for the k = 3 fp32 16384^2 task
// against 0.77 ms for the clean one, the in-place vote 1.65 ms.
template <int DT, int TOL, int K, int V, bool INL>
__device__ __forceinline__ uint32_t vote_vec(const typename VT<DT>::W (&x)[K][V], const TolD &tol, bool valid,
                                             ElemOut<typename VT<DT>::W> (&o)[V]) {
  using W = typename VT<DT>::W;
  uint32_t gen = 0;
#pragma unroll
  for (int e = 0; e < V; ++e) {
    W xe[K];
#pragma unroll
    for (int r = 0; r < K; ++r) xe[r] = x[r][e];
    if constexpr (K == 2) {
      o[e] = vote_general<DT, TOL, 2>(xe, tol);
    } else {
      bool g = false;
      o[e] = vote_fast<DT, TOL, K>(xe, tol, g);
      gen |= (uint32_t)(g && valid) << e;
    }
  }
  if constexpr (K == 3 || (K >= 4 && INL)) {
    // marked unlikely so that the general votes are laid out after the
    // streaming path instead of inside it
    if (__builtin_expect(__ballot(gen != 0u) != 0ull, 0)) {
#pragma unroll
      for (int e = 0; e < V; ++e) {
        if ((gen >> e) & 1u) {
          W xe[K];
#pragma unroll
          for (int r = 0; r < K; ++r) xe[r] = x[r][e];
          if constexpr (K == 3) o[e] = vote3_slow<DT, TOL>(xe, tol);
          else o[e] = vote_general<DT, TOL, K>(xe, tol);
        }
      }
    }
    gen = 0;
  }
  return gen;
}

// Vote vectors [v0, v1) of a task with the calling workgroup (vector path:
// vector = 16 bytes; scalar path: vector = one element).  Lane `tid` handles
// v0 + tid + u*nthreads for u < U in each step, all loads of a step issued
// before any vote.
template <int DT, int TOL, int K, bool VEC, int U, bool INL = false, class A>
__device__ __forceinline__ void vote_range(const TaskD &t, uint64_t v0, uint64_t v1, A &acc, bool nt) {
  using W = typename VT<DT>::W;
  constexpr int V = VEC ? Vec<W>::V : 1;
  const uint32_t nth = blockDim.x;
  const uint32_t tid = threadIdx.x;
  const bool wc = t.cons != nullptr, wm = t.mask != nullptr;
  for (uint64_t base = v0; base < v1; base += (uint64_t)nth * U) {
    W x[U][K][V];
    const bool full = base + (uint64_t)U * nth <= v1;  // workgroup-uniform
    if (full) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint64_t vi = base + (uint64_t)u * nth + tid;
#pragma unroll
        for (int r = 0; r < K; ++r) {
          if constexpr (VEC) Vec<W>::unpack(ld16(t.rep[r], vi), x[u][r]);
          else x[u][r][0] = __builtin_nontemporal_load(reinterpret_cast<const W *>(t.rep[r]) + vi);
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint64_t vi = base + (uint64_t)u * nth + tid;
        const bool valid = vi < v1;
#pragma unroll
        for (int r = 0; r < K; ++r) {
          if constexpr (VEC) {
            u32x4 v = {0u, 0u, 0u, 0u};
            if (valid) v = ld16(t.rep[r], vi);
            Vec<W>::unpack(v, x[u][r]);
          } else {
            x[u][r][0] = valid ? __builtin_nontemporal_load(reinterpret_cast<const W *>(t.rep[r]) + vi)
                               : (W)0;
          }
        }
      }
    }
    // fast pass: every element is voted and stored; elements whose replicas
    // hold two or more differing bit patterns are flagged in `need`
    uint32_t need = 0;
    const __amdgpu_buffer_rsrc_t rc = stream_rsrc(reinterpret_cast<uintptr_t>(t.cons) + base * 16u);
    const __amdgpu_buffer_rsrc_t rm = stream_rsrc(reinterpret_cast<uintptr_t>(t.mask) + base * V);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t vi = base + (uint64_t)u * nth + tid;
      const bool valid = vi < v1;
      W cv[V];
      uint32_t mbs = 0;
      if constexpr (K == 3 || INL) {
        ElemOut<W> o[V];
        const uint32_t gen = vote_vec<DT, TOL, K, V, INL>(x[u], t.tol, valid, o);
        need |= gen << (u * V);
#pragma unroll
        for (int e = 0; e < V; ++e) {
          cv[e] = o[e].cons;
          mbs |= o[e].mb << (8 * e);
          acc.add(valid && !((gen >> e) & 1u), o[e].ne, o[e].mb);
        }
      } else {
        // element by element, each counted right after its vote (this order
        // keeps the scalar registers of the ballot counts of large k unspilled)
#pragma unroll
        for (int e = 0; e < V; ++e) {
          W xe[K];
#pragma unroll
          for (int r = 0; r < K; ++r) xe[r] = x[u][r][e];
          bool general = false;
          ElemOut<W> o;
          if constexpr (K == 2) o = vote_general<DT, TOL, 2>(xe, t.tol);
          else o = vote_fast<DT, TOL, K>(xe, t.tol, general);
          general = general && valid;
          need |= (uint32_t)general << (u * V + e);
          cv[e] = o.cons;
          mbs |= o.mb << (8 * e);
          acc.add(valid && !general, o.ne, o.mb);
        }
      }
      if (valid) {
        if constexpr (VEC) {
          const uint32_t so = (uint32_t)u * nth + tid;  // vector index within the step
          if (wc) {
            if (nt) __builtin_amdgcn_raw_buffer_store_b128(Vec<W>::pack(cv), rc, so * 16u, 0, kStreamStorePolicy);
            else reinterpret_cast<u32x4 *>(t.cons)[vi] = Vec<W>::pack(cv);
          }
          if (wm) {
            if constexpr (V == 4) {
              if (nt) __builtin_amdgcn_raw_buffer_store_b32(mbs, rm, so * 4u, 0, kStreamStorePolicy);
              else reinterpret_cast<uint32_t *>(t.mask)[vi] = mbs;
            } else {
              if (nt) __builtin_amdgcn_raw_buffer_store_b16((uint16_t)mbs, rm, so * 2u, 0, kStreamStorePolicy);
              else reinterpret_cast<uint16_t *>(t.mask)[vi] = (uint16_t)mbs;
            }
          }
        } else {
          if (wc) st_nt(reinterpret_cast<W *>(t.cons) + vi, cv[0], nt);
          if (wm) t.mask[vi] = (uint8_t)mbs;
        }
      }
    }
    // fix-up pass (k >= 4 without INL): the loaded vectors are dead here, so
    // the general vote does not add to the register footprint of the fast
    // pass.  The element is reloaded, voted and stored again after this lane's
    // earlier stores have completed.
    if constexpr (K >= 4 && !INL) {
      if (__ballot(need != 0u) != 0ull) {
        __threadfence_block();
#pragma unroll 1
        for (int q = 0; q < U * V; ++q) {
          const bool mine = (need >> q) & 1u;
          ElemOut<W> o{};
          if (mine) {
            const uint64_t i = (base + (uint64_t)(q / V) * nth + tid) * V + (uint64_t)(q % V);
            W xe[K];
#pragma unroll
            for (int r = 0; r < K; ++r) xe[r] = reinterpret_cast<const W *>(t.rep[r])[i];
            o = vote_slow<DT, TOL, K>(xe, t.tol, t.rep, i);
            if (wc) reinterpret_cast<W *>(t.cons)[i] = o.cons;
            if (wm) t.mask[i] = (uint8_t)o.mb;
          }
          acc.add(mine, o.ne, o.mb);
        }
      }
    }
  }
}

// One full step of the vector path: vectors [base, base + U*nthreads) all
// exist, so no lane is masked.  The outputs go out as streaming buffer stores
// against resources based at the step; a NULL output gets a resource of size
// zero, whose stores the hardware discards, so the step has no branch on the
// optional outputs and the loads, votes and stores form one straight block.
template <int DT, int TOL, int K, int U, bool INL = false, class A>
__device__ __forceinline__ void vote_step_full(const TaskD &t, uint64_t base, A &acc) {
  using W = typename VT<DT>::W;
  constexpr int V = Vec<W>::V;
  const uint32_t nth = blockDim.x;
  const uint32_t tid = threadIdx.x;
  W x[U][K][V];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint64_t vi = base + (uint64_t)u * nth + tid;
#pragma unroll
    for (int r = 0; r < K; ++r) Vec<W>::unpack(ld16(t.rep[r], vi), x[u][r]);
  }
  const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(
      reinterpret_cast<void *>(reinterpret_cast<uintptr_t>(t.cons) + base * 16u), (short)0,
      t.cons ? 0x7fffffff : 0, 0x00020000);
  const __amdgpu_buffer_rsrc_t rm = __builtin_amdgcn_make_buffer_rsrc(
      reinterpret_cast<void *>(reinterpret_cast<uintptr_t>(t.mask) + base * V), (short)0,
      t.mask ? 0x7fffffff : 0, 0x00020000);
  uint32_t need = 0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    W cv[V];
    uint32_t mbs = 0;
    if constexpr (K == 3 || INL) {
      ElemOut<W> o[V];
      const uint32_t gen = vote_vec<DT, TOL, K, V, INL>(x[u], t.tol, true, o);
      need |= gen << (u * V);
#pragma unroll
      for (int e = 0; e < V; ++e) {
        cv[e] = o[e].cons;
        mbs |= o[e].mb << (8 * e);
        acc.add(!((gen >> e) & 1u), o[e].ne, o[e].mb);
      }
    } else {
      // element by element, as in vote_range
#pragma unroll
      for (int e = 0; e < V; ++e) {
        W xe[K];
#pragma unroll
        for (int r = 0; r < K; ++r) xe[r] = x[u][r][e];
        bool general = false;
        ElemOut<W> o;
        if constexpr (K == 2) o = vote_general<DT, TOL, 2>(xe, t.tol);
        else o = vote_fast<DT, TOL, K>(xe, t.tol, general);
        need |= (uint32_t)general << (u * V + e);
        cv[e] = o.cons;
        mbs |= o.mb << (8 * e);
        acc.add(!general, o.ne, o.mb);
      }
    }
    const uint32_t so = (uint32_t)u * nth + tid;
    __builtin_amdgcn_raw_buffer_store_b128(Vec<W>::pack(cv), rc, so * 16u, 0, kStreamStorePolicy);
    if constexpr (V == 4) __builtin_amdgcn_raw_buffer_store_b32(mbs, rm, so * 4u, 0, kStreamStorePolicy);
    else __builtin_amdgcn_raw_buffer_store_b16((uint16_t)mbs, rm, so * 2u, 0, kStreamStorePolicy);
  }
  // fix-up pass (k >= 4 without INL), as in vote_range
  if constexpr (K >= 4 && !INL) {
    if (__ballot(need != 0u) != 0ull) {
      __threadfence_block();
#pragma unroll 1
      for (int q = 0; q < U * V; ++q) {
        const bool mine = (need >> q) & 1u;
        ElemOut<W> o{};
        if (mine) {
          const uint64_t i = (base + (uint64_t)(q / V) * nth + tid) * V + (uint64_t)(q % V);
          W xe[K];
#pragma unroll
          for (int r = 0; r < K; ++r) xe[r] = reinterpret_cast<const W *>(t.rep[r])[i];
          o = vote_slow<DT, TOL, K>(xe, t.tol, t.rep, i);
          if (t.cons) reinterpret_cast<W *>(t.cons)[i] = o.cons;
          if (t.mask) t.mask[i] = (uint8_t)o.mb;
        }
        acc.add(mine, o.ne, o.mb);
      }
    }
  }
}

// Elements [nvec*V, n) of a vector-path task (fewer than V), one per lane.
template <int DT, int TOL, int K, class A>
__device__ __forceinline__ void vote_tail(const TaskD &t, A &acc) {
  using W = typename VT<DT>::W;
  constexpr int V = Vec<W>::V;
  const uint64_t i = t.nvec * V + threadIdx.x;
  const bool valid = threadIdx.x < V && i < t.n;
  W xe[K];
#pragma unroll
  for (int r = 0; r < K; ++r) xe[r] = valid ? reinterpret_cast<const W *>(t.rep[r])[i] : (W)0;
  const ElemOut<W> o = vote_elem<DT, TOL, K>(xe, t.tol, t.rep, valid ? i : 0);
  acc.add(valid, o.ne, o.mb);
  if (valid) {
    if (t.cons) reinterpret_cast<W *>(t.cons)[i] = o.cons;
    if (t.mask) t.mask[i] = (uint8_t)o.mb;
  }
}

// Sum the wave accumulators of a workgroup; the result for counter q is
// returned in thread q (q < NC) of the workgroup.  `sh` holds >= 16*32 u64.
template <int K, class A>
__device__ __forceinline__ uint64_t block_total(A &acc, uint64_t *sh) {
  constexpr int NC = A::NC;
  if constexpr (A::kLane) acc.fold();
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint32_t nw = blockDim.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NC; ++q) sh[wave * kNumCounters + q] = acc.c[q];
  }
  __syncthreads();
  uint64_t s = 0;
  if (threadIdx.x < (uint32_t)NC)
    for (uint32_t w = 0; w < nw; ++w) s += sh[w * kNumCounters + threadIdx.x];
  __syncthreads();
  return s;
}

// Verdict and stats from the task totals tot[q], q < NC (LDS), by one thread.
__device__ __forceinline__ int pair_index(int K, int r, int j) {  // r < j
  return r * (2 * K - r - 1) / 2 + (j - r - 1);
}

template <int K>
__device__ __forceinline__ void write_stats(ftv_stats *st, const uint64_t *tot, uint64_t n) {
  constexpr int NP = NPair<K>::value;
  bool all_zero = true;
  for (int i = 0; i < NP; ++i) all_zero = all_zero && tot[i] == 0;
  int best = 0, bestT = -1, argmin = 0;
  for (int r = 0; r < K; ++r) {
    int T = 1;  // itself
    for (int j = 0; j < K; ++j)
      if (j != r) T += tot[pair_index(K, r < j ? r : j, r < j ? j : r)] == 0;
    if (T > bestT) {
      bestT = T;
      best = r;
    }
    if (tot[NP + r] < tot[NP + argmin]) argmin = r;
  }
  const uint64_t nomaj = tot[NP + K];
  int verdict, winner;
  if (all_zero) {
    verdict = FTV_UNANIMOUS;
    winner = 0;
  } else if (2 * bestT > K) {
    verdict = FTV_TASK_MAJORITY;
    winner = best;
  } else if (nomaj == 0) {
    verdict = FTV_ELEMENT_MAJORITY;
    winner = argmin;
  } else {
    verdict = FTV_UNRESOLVED;
    winner = argmin;
  }
  for (int r = 0; r < FTV_MAX_K; ++r)
    for (int j = 0; j < FTV_MAX_K; ++j) {
      uint64_t v = 0;
      if (r < K && j < K && r != j) v = tot[pair_index(K, r < j ? r : j, r < j ? j : r)];
      st->pair[r][j] = v;
    }
  for (int r = 0; r < FTV_MAX_K; ++r) st->disagree[r] = r < K ? tot[NP + r] : 0;
  st->no_majority = nomaj;
  st->n = n;
  st->verdict = verdict;
  st->winner = winner;
}

// Vectors per lane and loop step of the streaming vote: two for k <= 3 (six
// 16-byte loads in flight per lane), one for larger k.
template <int K>
struct Unroll {
  static constexpr int value = K <= 3 ? 2 : 1;
};

// Stats record of one task from its accumulator row, by one workgroup of at
// least kNumCounters threads; the row is cleared when `clear` is set.
__device__ __forceinline__ void finalize_task(const TaskD &t, uint64_t *row, bool clear,
                                              uint64_t *s_tot) {
  if (threadIdx.x < (uint32_t)kNumCounters) {
    s_tot[threadIdx.x] = __hip_atomic_load(&row[threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (clear) row[threadIdx.x] = 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    switch (t.k) {
      case 2: write_stats<2>(t.stats, s_tot, t.n); break;
      case 3: write_stats<3>(t.stats, s_tot, t.n); break;
      case 4: write_stats<4>(t.stats, s_tot, t.n); break;
      case 5: write_stats<5>(t.stats, s_tot, t.n); break;
      case 6: write_stats<6>(t.stats, s_tot, t.n); break;
      case 7: write_stats<7>(t.stats, s_tot, t.n); break;
    }
  }
  __syncthreads();
}

}  // namespace dev
}  // namespace ftv
