// ftv_blocks_dev.hpp -- device helpers shared by the block hashing kernels
// (ftv_hash.hip) and the block vote (ftv_blocks.hip).
#pragma once

#include "ftv_internal.hpp"

namespace ftv {
namespace blockdev {

// b.rep[r] for a runtime r, as a select chain: indexing the by-value kernel
// argument with a runtime index would copy it to scratch memory.
template <int K>
__device__ __forceinline__ const void *rep_ptr(const BlockVoteD &b, int r) {
  const void *p = b.rep[0];
#pragma unroll
  for (int j = 1; j < K; ++j) p = (j == r) ? b.rep[j] : p;
  return p;
}
// Vote of the K block fingerprints (uniform across the workgroup): the block
// map byte (bit r: replica r differs from the source, bit 7: no majority) and
// the source replica.
template <int K>
__device__ __forceinline__ uint32_t vote_fps(const uint64_t (&f)[K], int *src_out) {
  int M = 0, src = 0;
#pragma unroll
  for (int r = 0; r < K; ++r) {
    int s = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) s += f[r] == f[j];
    if (s > M) {
      M = s;
      src = r;
    }
  }
  uint32_t bm = 0;
#pragma unroll
  for (int r = 0; r < K; ++r) bm |= (uint32_t)(f[r] != f[src]) << r;
  if (2 * M <= K) bm |= 0x80u;
  *src_out = src;
  return bm;
}

}  // namespace blockdev
}  // namespace ftv
