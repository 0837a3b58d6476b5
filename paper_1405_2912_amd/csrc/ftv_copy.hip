// ftv_copy.hip -- device-side helpers of the sibling manager for gfx950: the
// copy that makes a backup sibling in device memory, and the per-block vote
// of sibling fingerprints.
//
// Copy: a grid-stride stream of 16-byte non-temporal loads and stores, four
// vectors in flight per lane, two workgroups per CU (the rate-optimal stream
// count measured for the vote kernels); a ragged tail below 16 bytes is
// copied byte by byte by the last workgroup.  Both pointers are 16-byte
// aligned (device allocations).
//
// Fingerprint vote: one thread per block compares the m fingerprints of the
// block; a sibling differing from a strict majority gets its flag set, a block
// without one counts as unresolved.
#include "ftv_internal.hpp"

namespace ftv {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kCopyUnroll = 4;

// Stores go out non-temporal at agent scope (nt sc1), written through the
// XCD's L2, against a buffer resource based at the step's first vector.
__device__ __forceinline__ void copy_store16(uintptr_t base, uint32_t off, u32x4 v) {
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void *>(base), (short)0, 0x7fffffff, 0x00020000);
  __builtin_amdgcn_raw_buffer_store_b128(v, rs, off, 0, 2 | 16);
}

__global__ __launch_bounds__(256) void k_copy(u32x4 *dst, const u32x4 *src, uint64_t nvec,
                                              uint8_t *dst_tail, const uint8_t *src_tail, uint32_t ntail) {
  const uint64_t step = (uint64_t)blockDim.x * kCopyUnroll;
  uint64_t base = (uint64_t)blockIdx.x * step;
  for (; base + step <= nvec; base += (uint64_t)gridDim.x * step) {
    u32x4 v[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u)
      v[u] = __builtin_nontemporal_load(src + base + (uint64_t)u * blockDim.x + threadIdx.x);
    const uintptr_t db = reinterpret_cast<uintptr_t>(dst + base);
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) copy_store16(db, (u * blockDim.x + threadIdx.x) * 16u, v[u]);
  }
  if (base < nvec) {  // this workgroup's partial step
    for (uint64_t i = base + threadIdx.x; i < nvec; i += blockDim.x) dst[i] = src[i];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x < ntail) dst_tail[threadIdx.x] = src_tail[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_fp_vote(const uint64_t *fps, uint32_t m, uint64_t nblocks,
                                                 uint32_t *bad, uint64_t *unresolved) {
  uint64_t my_unresolved = 0;
  for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nblocks;
       b += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t best = 0, best_support = 0;
    bool differ = false;
    for (uint32_t j = 0; j < m; ++j) {
      const uint64_t f = fps[(uint64_t)j * nblocks + b];
      differ = differ || f != fps[b];
      uint32_t support = 0;
      for (uint32_t q = 0; q < m; ++q) support += fps[(uint64_t)q * nblocks + b] == f;
      if (support > best_support) {
        best_support = support;
        best = j;
      }
    }
    if (2 * best_support > m) {
      const uint64_t f = fps[(uint64_t)best * nblocks + b];
      for (uint32_t j = 0; j < m; ++j)
        if (fps[(uint64_t)j * nblocks + b] != f) __hip_atomic_store(&bad[j], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if (differ) {
      ++my_unresolved;
    }
  }
  if (my_unresolved)
    __hip_atomic_fetch_add(unresolved, my_unresolved, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_zero_words(uint32_t *w, uint32_t n) {
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) w[i] = 0;
}

}  // namespace

hipError_t launch_copy(void *dst, const void *src, uint64_t bytes, int num_cus, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  const uint64_t nvec = bytes / 16;
  const uint32_t ntail = (uint32_t)(bytes % 16);
  const uint64_t per = 256ull * kCopyUnroll;
  uint64_t grid = (nvec + per - 1) / per;
  if (grid > (uint64_t)num_cus * 2) grid = (uint64_t)num_cus * 2;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_copy, dim3((uint32_t)grid), dim3(256), 0, s, reinterpret_cast<u32x4 *>(dst),
                     reinterpret_cast<const u32x4 *>(src), nvec, reinterpret_cast<uint8_t *>(dst) + nvec * 16,
                     reinterpret_cast<const uint8_t *>(src) + nvec * 16, ntail);
  return hipGetLastError();
}

hipError_t launch_fp_vote(const uint64_t *fps, uint32_t m, uint64_t nblocks, uint32_t *bad_and_unresolved,
                          int num_cus, hipStream_t s) {
  // layout of the result words: bad[m] (u32), then the unresolved count (u64,
  // 8-byte aligned)
  const uint32_t words = (m + 1) / 2 * 2 + 2;
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, bad_and_unresolved, words);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  uint64_t grid = (nblocks + 255) / 256;
  if (grid > (uint64_t)num_cus * 4) grid = (uint64_t)num_cus * 4;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_fp_vote, dim3((uint32_t)grid), dim3(256), 0, s, fps, m, nblocks, bad_and_unresolved,
                     reinterpret_cast<uint64_t *>(bad_and_unresolved + (m + 1) / 2 * 2));
  return hipGetLastError();
}

}  // namespace ftv
