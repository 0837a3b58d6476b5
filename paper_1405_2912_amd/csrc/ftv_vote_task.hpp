// ftv_vote_task.hpp -- the per-task vote kernel and its launcher, included by
// one translation unit per value type (ftv_vote_f32.hip, ...).
//
// A grid-stride loop over tiles of 16-byte vectors; each workgroup reduces its
// wave accumulators and adds the non-zero totals to the launch's device
// accumulators (most workgroups see no disagreement and add nothing).  A
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

// Launch shape: one workgroup of 512 threads per CU.  On MI355X, with the
// replicas' own (random) data, this streamed the k = 3 fp32 vote at 0.795 ms
// against 0.826 ms for two 256-thread workgroups per CU (the same waves per
// CU): a step of a workgroup then covers 16 KiB of every replica instead of
// 8 KiB, and fewer concurrent streams keep more DRAM page locality.  More
// waves per CU, or more vectors in flight per lane, measured slower.
constexpr int kVoteThreads = 512;
constexpr int kVoteWgPerCu = 1;

template <int DT, int TOL, int K, bool VEC>
__global__ __launch_bounds__(kVoteThreads) void k_vote_task(TaskD t, VoteWs ws) {
  __shared__ uint64_t sh[16 * kNumCounters];
  constexpr int U = Unroll<K>::value;
  constexpr int NC = Acc<K>::NC;
  Acc<K> acc;
  acc.zero();
  const uint64_t tile = (uint64_t)blockDim.x * U;
  for (uint64_t b = (uint64_t)blockIdx.x * tile; b < t.nvec; b += (uint64_t)gridDim.x * tile) {
    const uint64_t e = b + tile < t.nvec ? b + tile : t.nvec;
    vote_range<DT, TOL, K, VEC, U>(t, b, e, acc, true);
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
hipError_t launch_one(const TaskD &t, const VoteWs &ws, int num_cus, hipStream_t s) {
  constexpr int U = Unroll<K>::value;
  const uint64_t tile = (uint64_t)kVoteThreads * U;
  const uint64_t tiles = (t.nvec + tile - 1) / tile;
  uint64_t cap = (uint64_t)num_cus * kVoteWgPerCu;
  if (cap > (uint64_t)kMaxGrid) cap = kMaxGrid;
  const uint32_t grid = (uint32_t)(tiles < 1 ? 1 : (tiles < cap ? tiles : cap));
  hipLaunchKernelGGL((k_vote_task<DT, TOL, K, VEC>), dim3(grid), dim3(kVoteThreads), 0, s, t, ws);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_vote_finalize, dim3(1), dim3(64), 0, s, t, ws);
  return hipGetLastError();
}

template <int DT, int TOL, bool VEC>
hipError_t launch_k(const TaskD &t, const VoteWs &ws, int num_cus, hipStream_t s) {
  switch (t.k) {
    case 2: return launch_one<DT, TOL, 2, VEC>(t, ws, num_cus, s);
    case 3: return launch_one<DT, TOL, 3, VEC>(t, ws, num_cus, s);
    case 4: return launch_one<DT, TOL, 4, VEC>(t, ws, num_cus, s);
    case 5: return launch_one<DT, TOL, 5, VEC>(t, ws, num_cus, s);
    case 6: return launch_one<DT, TOL, 6, VEC>(t, ws, num_cus, s);
    case 7: return launch_one<DT, TOL, 7, VEC>(t, ws, num_cus, s);
  }
  return hipErrorInvalidValue;
}

template <int DT, int TOL>
hipError_t launch_vec(const TaskD &t, const VoteWs &ws, int num_cus, hipStream_t s) {
  return t.vec ? launch_k<DT, TOL, true>(t, ws, num_cus, s)
               : launch_k<DT, TOL, false>(t, ws, num_cus, s);
}

}  // namespace
}  // namespace ftv
