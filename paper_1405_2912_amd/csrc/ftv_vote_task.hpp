// ftv_vote_task.hpp -- the per-task vote kernel and its launcher, included by
// one translation unit per value type (ftv_vote_f32.hip, ...).
//
// A grid-stride loop over tiles of 16-byte vectors; each workgroup reduces its
// wave accumulators and adds the non-zero totals to the launch's device
// accumulators (most workgroups see no disagreement and add nothing).  The
// kernel runs one workgroup per CU, so registers are plentiful: counts go to
// per-lane counters and, up to k = 5, the general vote of an element with
// several differing values runs in place from the loaded registers.  A
// one-workgroup finalize kernel on the same stream then decides the verdict,
// writes the stats record and clears the accumulators: the kernel boundary
// orders the counts before the verdict, so the vote kernel needs neither a
// completion ticket nor device-scope fences.
//
// The value types live in separate translation units so that each code object
// stays small: on MI355X the same kernel measured about 7% slower when it was
// loaded from one code object holding every vote kernel (about 1 MB of code)
// than from a small one.
#pragma once

#include "ftv_internal.hpp"
#include "ftv_vote_dev.hpp"

namespace ftv {
namespace {

using namespace dev;

// Launch shape: one workgroup per CU, looping over tiles of `threads` x U
// vectors (grid-stride).  The threads per workgroup and the vectors per lane
// and step depend on the replica count and the element size; the values are
// those a sweep on MI355X found fastest for the vote of replicas that differ
// in few elements (k = 2..7, 4- and 8-byte elements, 1 GiB and 512 MiB per
// replica): for k = 3 fp32, 256 threads with four vectors in flight per lane
// and replica streamed at 0.76 ms against 0.79 ms for 512 threads with two.
// Full tiles go through the branch-free step of vote_step_full; where the
// sweep found the general step as fast (k = 3 with 8-byte elements) every
// tile uses vote_range.  Re-swept once counts moved to per-lane counters and
// general votes into the registers: k = 4 (256 threads, U = 2: fp32 0.946
// against 0.952 ms, fp64 8192^2 0.433 against 0.458 ms) and k = 6 (256
// threads, U = 4: fp32 1.408 against 1.441 ms, fp64 0.668 against 0.741 ms)
// changed; the other entries held.  Bit-wise (EXACT) votes of 8-byte
// elements keep 512 threads and the general step (k = 3 int32 once measured
// 0.74 ms that way against 0.80 ms); for 4-byte elements the re-sweep found
// 256 threads better up to k = 4 (int32 k = 3, U = 2: 0.762 against 0.787 ms;
// k = 2, U = 4: 0.593 against 0.601 ms).  More workgroups per CU measured
// slower throughout: longer contiguous steps and fewer concurrent streams keep
// DRAM page locality, and a grid larger than what is resident leaves a tail.
//
// xcd: the full tiles of one grid-stride round are handed out so that the
// workgroups of one XCD (the hardware deals workgroups out to the 8 XCDs
// round robin) take adjacent tiles, each XCD streaming one contiguous eighth
// of the round instead of every eighth tile.  Measured against the plain
// order on the 1 GiB / 512 MiB replicas: fp32 k = 3 0.727 against 0.740 ms,
// k = 2 0.576-0.581 against 0.582; int32 bit-wise k = 2 0.585 against
// 0.591-0.595; fp64 k = 7 0.738 against 0.752 ms, k = 4 0.422 against
// 0.424-0.428 ms; but fp32 k = 5 1.20-1.22 against 1.13 ms and k = 4 0.954
// against 0.942 ms, and no change elsewhere, so only those shapes use it.
struct VoteShape {
  int threads;
  int unroll;
  bool lean;
  bool xcd = false;
};
constexpr VoteShape vote_shape(int es, int tol, int k) {
  if (tol == FTV_TOL_EXACT && es == 4) {
    switch (k) {
      case 2: return {256, 4, true, true};
      case 3: return {256, 2, true};
      case 4: return {256, 2, true};
      default: return {512, 1, false};
    }
  }
  if (tol == FTV_TOL_EXACT) return {512, k <= 3 ? 2 : 1, false};
  if (es == 4) {
    switch (k) {
      case 2: return {256, 4, true, true};
      case 3: return {256, 4, true, true};
      case 4: return {256, 2, true};
      case 5: return {256, 2, true};
      case 6: return {256, 4, true};
      default: return {256, 1, true};
    }
  }
  switch (k) {
    case 2: return {256, 4, true};
    case 3: return {512, 2, false};
    case 4: return {256, 2, true, true};
    case 5: return {512, 2, true};
    case 6: return {256, 4, true};
    default: return {256, 1, true, true};
  }
}
constexpr int kVoteWgPerCu = 1;

template <int DT, int TOL, int K, bool VEC>
struct TaskShape {
  static constexpr VoteShape s =
      VEC ? vote_shape(sizeof(typename VT<DT>::W), TOL, K) : VoteShape{512, Unroll<K>::value, false};
  static constexpr int threads = s.threads;
  static constexpr int U = s.unroll;
  static constexpr bool lean = s.lean;
  static constexpr bool xcd = s.xcd;
};

// Counts in per-lane counters at every k; the general vote in place up to
// k = 5.  From k = 6 on the tolerance tests of an in-place general vote (15
// or 21 lane masks) overflow the scalar registers, which the compiler then
// spills through lanes of a vector register: for the fp32 16384^2 task the
// kernel measured 1.86 ms at k = 7 that way against 1.62-1.67 ms with the
// element-by-element loop and the fix-up pass, and 1.48 ms against 1.45 ms at
// k = 6, so k = 6 and 7 keep that loop.  There the per-lane counters also
// free the 58 scalar registers of 64-bit ballot counts (k = 7: 90 spilled
// scalars with ballot counts, none with per-lane ones; 1.66 -> 1.62 ms).
template <int K>
struct TaskAcc {
  static constexpr bool inl = K <= 5;
  using type = LaneAcc<K>;
};

template <int DT, int TOL, int K, bool VEC>
__global__ __launch_bounds__((TaskShape<DT, TOL, K, VEC>::threads)) void k_vote_task(TaskD t, VoteWs ws) {
  __shared__ uint64_t sh[16 * kNumCounters];
  using S = TaskShape<DT, TOL, K, VEC>;
  constexpr int U = S::U;
  constexpr bool INL = TaskAcc<K>::inl;
  using A = typename TaskAcc<K>::type;
  constexpr int NC = A::NC;
  A acc;
  acc.zero();
  const uint64_t tile = (uint64_t)blockDim.x * U;
  if constexpr (S::lean) {
    // full tiles grid-stride, then the partial tile (if any) by its owner
    const uint64_t nfull = t.nvec / tile;
    const uint32_t g = gridDim.x;
    const uint32_t first = (S::xcd && g % 8u == 0u) ? (blockIdx.x % 8u) * (g / 8u) + blockIdx.x / 8u : blockIdx.x;
    for (uint64_t i = first; i < nfull; i += g) vote_step_full<DT, TOL, K, U, INL>(t, i * tile, acc);
    if (nfull * tile < t.nvec && blockIdx.x == nfull % gridDim.x)
      vote_range<DT, TOL, K, VEC, U, INL>(t, nfull * tile, t.nvec, acc, true);
  } else {
    for (uint64_t b = (uint64_t)blockIdx.x * tile; b < t.nvec; b += (uint64_t)gridDim.x * tile) {
      const uint64_t e = b + tile < t.nvec ? b + tile : t.nvec;
      vote_range<DT, TOL, K, VEC, U, INL>(t, b, e, acc, true);
    }
  }
  if constexpr (VEC) {
    if (blockIdx.x == gridDim.x - 1) vote_tail<DT, TOL, K>(t, acc);
  }
  const uint64_t tot = block_total<K>(acc, sh);
  if (threadIdx.x < (uint32_t)NC && tot != 0)
    __hip_atomic_fetch_add(&ws.acc[threadIdx.x], tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(64) void k_vote_finalize(TaskD t, VoteWs ws) {
  __shared__ uint64_t s_tot[kNumCounters];
  finalize_task(t, ws.acc, true, s_tot);
}

// ---- per-task dispatch -----------------------------------------------------
// The grid never exceeds what is resident at once (one workgroup per CU):
// the grid-stride loop is only balanced when every workgroup runs from the
// start, a larger grid leaves a second, mostly empty wave of workgroups.
template <int DT, int TOL, int K, bool VEC>
hipError_t launch_one(const TaskD &t, const VoteWs &ws, int num_cus, hipStream_t s, bool finalize) {
  using S = TaskShape<DT, TOL, K, VEC>;
  const uint64_t tile = (uint64_t)S::threads * S::U;
  const uint64_t tiles = (t.nvec + tile - 1) / tile;
  uint64_t cap = (uint64_t)num_cus * kVoteWgPerCu;
  if (cap > (uint64_t)kMaxGrid) cap = kMaxGrid;
  const uint32_t grid = (uint32_t)(tiles < 1 ? 1 : (tiles < cap ? tiles : cap));
  hipLaunchKernelGGL((k_vote_task<DT, TOL, K, VEC>), dim3(grid), dim3(S::threads), 0, s, t, ws);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess || !finalize) return e;
  hipLaunchKernelGGL(k_vote_finalize, dim3(1), dim3(64), 0, s, t, ws);
  return hipGetLastError();
}

template <int DT, int TOL, bool VEC>
hipError_t launch_k(const TaskD &t, const VoteWs &ws, int num_cus, hipStream_t s, bool finalize) {
  switch (t.k) {
    case 2: return launch_one<DT, TOL, 2, VEC>(t, ws, num_cus, s, finalize);
    case 3: return launch_one<DT, TOL, 3, VEC>(t, ws, num_cus, s, finalize);
    case 4: return launch_one<DT, TOL, 4, VEC>(t, ws, num_cus, s, finalize);
    case 5: return launch_one<DT, TOL, 5, VEC>(t, ws, num_cus, s, finalize);
    case 6: return launch_one<DT, TOL, 6, VEC>(t, ws, num_cus, s, finalize);
    case 7: return launch_one<DT, TOL, 7, VEC>(t, ws, num_cus, s, finalize);
  }
  return hipErrorInvalidValue;
}

template <int DT, int TOL>
hipError_t launch_vec(const TaskD &t, const VoteWs &ws, int num_cus, hipStream_t s, bool finalize) {
  return t.vec ? launch_k<DT, TOL, true>(t, ws, num_cus, s, finalize)
               : launch_k<DT, TOL, false>(t, ws, num_cus, s, finalize);
}

}  // namespace
}  // namespace ftv
