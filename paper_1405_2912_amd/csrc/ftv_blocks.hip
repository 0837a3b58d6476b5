// ftv_blocks.hip -- the block vote for gfx950: pass 2 and the stats.
//
// Block vote, two passes.  Pass 1 (ftv_hash.hip) fingerprints every block of
// every replica, replica after replica, and streams replica 0 into the
// consensus.  Pass 2 votes the k fingerprints of each block by exact
// equality, writes the block map and its counts, re-copies the blocks whose
// strict-majority fingerprint is not replica 0's from the lowest-indexed
// replica holding it (in the common case replica 0 agrees and the restore
// cost one write pass and no extra read), and runs the element vote over
// every block without a majority; a one-workgroup finalize kernel writes the
// stats.  No kernel waits on another's workgroups: kernel boundaries on the
// stream order them.

#include "ftv_blocks_dev.hpp"
#include "ftv_internal.hpp"
#include "ftv_vote_dev.hpp"

namespace ftv {
namespace {

using namespace dev;
using namespace blockdev;

// Workspace accumulators: [0] disagree blocks, [1] fallback blocks,
// [2] unresolved elements, [3..3+K) replica blocks; zero between calls.
constexpr int kBlkAcc = 3 + FTV_MAX_K;

// Pass 2: the vote of the fingerprints, in chunks of `chunk` blocks (at most
// the workgroup size, one block per thread): the block map and its counts, the
// re-copy of every whole block whose majority fingerprint is not replica 0's
// (from the lowest replica holding it), and the element vote over every block
// without a fingerprint majority; the workgroup runs the copies and the
// element votes block by block.  Per workgroup the non-zero counts go to the
// accumulators.
// The workgroup is wide (1024 threads, several vectors per lane for small k)
// so that a 64 KiB block takes one or two passes: a lone no-majority block is
// a latency chain of passes, not a bandwidth problem.
constexpr uint32_t kScanThreads = 1024;

template <int K>
struct ScanUnroll {
  static constexpr int value = K <= 2 ? 4 : (K <= 4 ? 2 : 1);
};

template <int DT, int TOL, int K>
__global__ __launch_bounds__(kScanThreads) void k_blocks_scan(BlockVoteD b, uint32_t chunk) {
  using W = typename VT<DT>::W;
  constexpr int NC = Acc<K>::NC;
  __shared__ uint64_t sh[16 * kNumCounters];
  __shared__ uint32_t s_cnt[kBlkAcc];
  __shared__ uint32_t s_nfb;
  __shared__ uint32_t s_ncp;
  __shared__ uint64_t s_list[kScanThreads];
  __shared__ uint64_t s_copy[kScanThreads];  // block | source replica << 56
  // the block's task record lives in LDS: a local record indexed at run time
  // (the rare general vote does) would be placed in scratch memory
  __shared__ TaskD t;
  const uint64_t per = b.block_bytes / sizeof(W);
  const uint64_t n = b.nbytes / sizeof(W);
  const uint64_t nwhole = b.nbytes / b.block_bytes;
  if (threadIdx.x < (uint32_t)kBlkAcc) s_cnt[threadIdx.x] = 0;
  uint32_t c_dis = 0, c_fb = 0, c_rep[K];
#pragma unroll
  for (int r = 0; r < K; ++r) c_rep[r] = 0;
  Acc<K> acc;
  acc.zero();
  for (uint64_t base = (uint64_t)blockIdx.x * chunk; base < b.nblocks; base += (uint64_t)gridDim.x * chunk) {
    const uint64_t blk = base + threadIdx.x;
    uint32_t bm = 0;
    int src = 0;
    if (threadIdx.x < chunk && blk < b.nblocks) {
      uint64_t f[K];
#pragma unroll
      for (int r = 0; r < K; ++r) f[r] = b.fps[(uint64_t)r * b.nblocks + blk];
      bm = vote_fps<K>(f, &src);
      b.blockmap[blk] = (uint8_t)bm;
    }
    c_dis += (bm & 0x7fu) != 0;
    c_fb += bm >> 7;
#pragma unroll
    for (int r = 0; r < K; ++r) c_rep[r] += (bm >> r) & 1u;
    // replica 0 outvoted in a whole block (the partial block restores itself)
    const bool recopy = !(bm & 0x80u) && (bm & 1u) && blk < nwhole;
    if (!__syncthreads_or((int)((bm & 0x80u) || recopy))) continue;
    if (threadIdx.x == 0) s_nfb = s_ncp = 0;
    __syncthreads();
    if (bm & 0x80u) s_list[atomicAdd(&s_nfb, 1u)] = blk;
    if (recopy) s_copy[atomicAdd(&s_ncp, 1u)] = blk | ((uint64_t)src << 56);
    __syncthreads();
    const uint32_t ncp = s_ncp;
    for (uint32_t i = 0; i < ncp; ++i) {
      const uint64_t cb = s_copy[i] & ((1ull << 56) - 1);
      const int from = (int)(s_copy[i] >> 56);
      const u32x4 *sp = reinterpret_cast<const u32x4 *>(
          reinterpret_cast<const uint8_t *>(rep_ptr<K>(b, from)) + cb * b.block_bytes);
      const uintptr_t dp = reinterpret_cast<uintptr_t>(b.cons) + cb * b.block_bytes;
      for (uint32_t v = threadIdx.x; v < (uint32_t)(b.block_bytes / 16); v += kScanThreads)
        stream_store16(dp, v * 16u, ld16(sp, v));
    }
    const uint32_t nfb = s_nfb;
    for (uint32_t i = 0; i < nfb; ++i) {
      const uint64_t e0 = s_list[i] * per;
      const uint64_t ne = (e0 + per < n ? e0 + per : n) - e0;
      __syncthreads();
      if (threadIdx.x == 0) {
        for (int r = 0; r < FTV_MAX_K; ++r)
          t.rep[r] = r < K ? (const void *)(reinterpret_cast<const W *>(b.rep[r]) + e0) : nullptr;
        t.cons = reinterpret_cast<W *>(b.cons) + e0;
        t.mask = b.mask ? b.mask + e0 : nullptr;
        t.stats = nullptr;
        t.n = ne;
        t.nvec = ne / Vec<W>::V;
        t.tol = b.tol;
        t.k = K;
      }
      __syncthreads();
      vote_range<DT, TOL, K, true, ScanUnroll<K>::value>(t, 0, t.nvec, acc, false);
      vote_tail<DT, TOL, K>(t, acc);
    }
  }
  const uint64_t tot = block_total<K>(acc, sh);  // thread NC-1: elements without a majority
  if (c_dis) atomicAdd(&s_cnt[0], c_dis);
  if (c_fb) atomicAdd(&s_cnt[1], c_fb);
#pragma unroll
  for (int r = 0; r < K; ++r)
    if (c_rep[r]) atomicAdd(&s_cnt[3 + r], c_rep[r]);
  __syncthreads();
  if (threadIdx.x < (uint32_t)(3 + K)) {
    const uint32_t q = threadIdx.x;
    const uint64_t v = q == 2 ? 0 : (uint64_t)s_cnt[q];
    if (v) __hip_atomic_fetch_add(&b.acc[q], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (threadIdx.x == (uint32_t)(NC - 1) && tot)
    __hip_atomic_fetch_add(&b.acc[2], tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Verdict and stats record from the accumulators, which are cleared.
template <int K>
__global__ __launch_bounds__(64) void k_blocks_finalize(BlockVoteD b) {
  if (threadIdx.x != 0) return;
  uint64_t a[kBlkAcc];
  for (int i = 0; i < kBlkAcc; ++i) {
    a[i] = __hip_atomic_load(&b.acc[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    b.acc[i] = 0;
  }
  ftv_block_stats *st = b.bstats;
  st->blocks = b.nblocks;
  st->disagree_blocks = a[0];
  st->fallback_blocks = a[1];
  st->unresolved_elems = a[2];
  int clean = -1, argmin = 0;
  for (int r = 0; r < FTV_MAX_K; ++r) {
    st->replica_blocks[r] = r < K ? a[3 + r] : 0;
    if (r < K && clean < 0 && a[3 + r] == 0) clean = r;
    if (r < K && a[3 + r] < a[3 + argmin]) argmin = r;
  }
  if (a[0] == 0) {
    st->verdict = FTV_UNANIMOUS;
    st->winner = 0;
  } else if (a[1] == 0 && clean >= 0) {
    st->verdict = FTV_TASK_MAJORITY;
    st->winner = clean;
  } else if (a[2] == 0) {
    st->verdict = FTV_ELEMENT_MAJORITY;
    st->winner = argmin;
  } else {
    st->verdict = FTV_UNRESOLVED;
    st->winner = argmin;
  }
}

__global__ void k_blocks_empty(ftv_block_stats *st) {
  if (threadIdx.x == 0) {
    st->blocks = st->disagree_blocks = st->fallback_blocks = st->unresolved_elems = 0;
    for (int r = 0; r < FTV_MAX_K; ++r) st->replica_blocks[r] = 0;
    st->verdict = FTV_UNANIMOUS;
    st->winner = 0;
  }
}

// Scan + finalize.  The chunk (blocks per workgroup step) is the largest power
// of two up to the workgroup size that still gives every CU two workgroups, so
// that a map full of no-majority blocks still spreads their element votes over
// the chip.
template <int DT, int TOL, int K>
hipError_t launch_scan(const BlockVoteD &b, int num_cus, hipStream_t s) {
  uint64_t chunk = kScanThreads;
  while (chunk > 1 && b.nblocks / chunk < (uint64_t)num_cus * 2) chunk >>= 1;
  uint64_t grid = (b.nblocks + chunk - 1) / chunk;
  if (grid > (uint64_t)num_cus * 2) grid = (uint64_t)num_cus * 2;
  hipLaunchKernelGGL((k_blocks_scan<DT, TOL, K>), dim3((uint32_t)grid), dim3(kScanThreads), 0, s, b,
                     (uint32_t)chunk);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_blocks_finalize<K>), dim3(1), dim3(64), 0, s, b);
  return hipGetLastError();
}

template <int K>
hipError_t launch_blocks_k(const BlockVoteD &b, int num_cus, hipStream_t s) {
  const hipError_t e = launch_blocks_hash(b, s);
  if (e != hipSuccess) return e;
  switch (b.dtype * 3 + b.tolkind) {
    case FTV_F32 * 3 + FTV_TOL_EXACT: return launch_scan<FTV_F32, FTV_TOL_EXACT, K>(b, num_cus, s);
    case FTV_F32 * 3 + FTV_TOL_ULP: return launch_scan<FTV_F32, FTV_TOL_ULP, K>(b, num_cus, s);
    case FTV_F32 * 3 + FTV_TOL_REL: return launch_scan<FTV_F32, FTV_TOL_REL, K>(b, num_cus, s);
    case FTV_F64 * 3 + FTV_TOL_EXACT: return launch_scan<FTV_F64, FTV_TOL_EXACT, K>(b, num_cus, s);
    case FTV_F64 * 3 + FTV_TOL_ULP: return launch_scan<FTV_F64, FTV_TOL_ULP, K>(b, num_cus, s);
    case FTV_F64 * 3 + FTV_TOL_REL: return launch_scan<FTV_F64, FTV_TOL_REL, K>(b, num_cus, s);
    case FTV_I32 * 3 + FTV_TOL_EXACT: return launch_scan<FTV_I32, FTV_TOL_EXACT, K>(b, num_cus, s);
    case FTV_I64 * 3 + FTV_TOL_EXACT: return launch_scan<FTV_I64, FTV_TOL_EXACT, K>(b, num_cus, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_vote_blocks(const BlockVoteD &b, int num_cus, hipStream_t s) {
  if (b.nblocks == 0) {
    hipLaunchKernelGGL(k_blocks_empty, dim3(1), dim3(64), 0, s, b.bstats);
    return hipGetLastError();
  }
  switch (b.k) {
    case 2: return launch_blocks_k<2>(b, num_cus, s);
    case 3: return launch_blocks_k<3>(b, num_cus, s);
    case 4: return launch_blocks_k<4>(b, num_cus, s);
    case 5: return launch_blocks_k<5>(b, num_cus, s);
    case 6: return launch_blocks_k<6>(b, num_cus, s);
    case 7: return launch_blocks_k<7>(b, num_cus, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace ftv
