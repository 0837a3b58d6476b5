// ftv_blocks.hip -- block fingerprints and the fused block vote for gfx950.
//
// Fingerprint of a block (power-of-two size BB in [4 KiB, 64 KiB]): the block
// is read as little-endian 64-bit words, zero-padded past the end of the
// buffer; a leaf is 64-bit FNV-1a over 8 consecutive words (64 B) and leaves
// are combined pairwise, level by level, a node being FNV-1a over the two words
// (left, right).  One workgroup hashes one block with one leaf per thread:
// the first six levels of the tree are combined across the lanes of a wave,
// the remaining ones (up to four, for 16 waves) through LDS.
//
// Block vote: the same workgroup hashes the block in all k replicas, votes
// the k fingerprints by exact equality and restores the consensus from the
// lowest-indexed replica holding a strict-majority fingerprint.  Replica 0's
// data is streamed into the consensus while it is hashed, so in the common
// case (replica 0 agrees with the majority) the restore costs one write pass
// and no extra read.  Blocks without a majority fall back to the element vote
// over their elements in a second, small kernel.
#include "ftv_internal.hpp"
#include "ftv_vote_dev.hpp"

namespace ftv {
namespace {

using namespace dev;

constexpr uint64_t kFnvBasis = 0xcbf29ce484222325ull;

// (h ^ w) * 0x100000001b3 mod 2^64, with the prime split as 2^40 + 0x1b3.
__device__ __forceinline__ uint64_t fnv_step(uint64_t h, uint64_t w) {
  const uint64_t x = h ^ w;
  const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
  const uint64_t p = (uint64_t)lo * 0x1b3u;
  const uint32_t phi = (uint32_t)(p >> 32) + hi * 0x1b3u + (lo << 8);
  return ((uint64_t)phi << 32) | (uint32_t)p;
}

__device__ __forceinline__ uint64_t fnv_node(uint64_t l, uint64_t r) {
  return fnv_step(fnv_step(kFnvBasis, l), r);
}

// 64-byte leaf at byte offset `off` of a buffer of `nbytes` (zero beyond).
__device__ __forceinline__ void load_leaf(const void *base, uint64_t off, uint64_t nbytes,
                                          u32x4 (&v)[4]) {
  const uint8_t *b = reinterpret_cast<const uint8_t *>(base);
  if (off + 64 <= nbytes) {
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = ld16(b + off, (uint64_t)c);
    return;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const uint64_t o = off + 16ull * c;
    if (o + 16 <= nbytes) {
      v[c] = ld16(b + o, 0);
    } else {
      // partial chunk at the end of the buffer: bytes one by one, zero beyond
      uint32_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const uint32_t byte = (o + q < nbytes) ? (uint32_t)b[o + q] : 0u;
        const uint32_t sh = byte << (8 * (q & 3));
        if (q < 4) w0 |= sh;
        else if (q < 8) w1 |= sh;
        else if (q < 12) w2 |= sh;
        else w3 |= sh;
      }
      v[c].x = w0;
      v[c].y = w1;
      v[c].z = w2;
      v[c].w = w3;
    }
  }
}

__device__ __forceinline__ uint64_t leaf_hash(const u32x4 (&v)[4]) {
  uint64_t h = kFnvBasis;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    h = fnv_step(h, (uint64_t)v[c].x | ((uint64_t)v[c].y << 32));
    h = fnv_step(h, (uint64_t)v[c].z | ((uint64_t)v[c].w << 32));
  }
  return h;
}

// Root of the lane's LPT consecutive leaves (the lowest levels of the tree,
// combined in registers).  v holds the lane's 4*LPT 16-byte chunks in order.
template <int LPT>
__device__ __forceinline__ uint64_t lane_subtree(const u32x4 (&v)[4 * LPT]) {
  uint64_t h[LPT];
#pragma unroll
  for (int j = 0; j < LPT; ++j) {
    h[j] = kFnvBasis;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      h[j] = fnv_step(h[j], (uint64_t)v[4 * j + c].x | ((uint64_t)v[4 * j + c].y << 32));
      h[j] = fnv_step(h[j], (uint64_t)v[4 * j + c].z | ((uint64_t)v[4 * j + c].w << 32));
    }
  }
#pragma unroll
  for (int w = LPT; w > 1; w >>= 1)
#pragma unroll
    for (int j = 0; j < w / 2; ++j) h[j] = fnv_node(h[2 * j], h[2 * j + 1]);
  return h[0];
}

// Combine `levels` further levels across lanes (consecutive subtrees in
// consecutive lanes): afterwards lane 0 of each group of 2^levels lanes holds
// the group's root.
__device__ __forceinline__ uint64_t lane_tree(uint64_t h, int levels) {
  for (int lvl = 0; lvl < levels; ++lvl) {
    const uint64_t other = __shfl_xor(h, 1 << lvl, 64);
    h = fnv_node(h, other);  // meaningful on lanes whose bit `lvl` is clear
  }
  return h;
}

// Reduce `nw` wave roots in LDS (pairwise, in order) to the block root.
__device__ __forceinline__ uint64_t lds_tree(uint64_t *sh, uint32_t nw) {
  for (uint32_t len = nw; len > 1; len >>= 1)
    for (uint32_t j = 0; j < len / 2; ++j) sh[j] = fnv_node(sh[2 * j], sh[2 * j + 1]);
  return sh[0];
}

// The lane's LPT leaves at byte offset `off`: whole (no bounds tests) or with
// zero padding past the end of the buffer.
template <int LPT>
__device__ __forceinline__ void load_leaves(const void *base, uint64_t off, uint64_t nbytes, bool whole,
                                            u32x4 (&v)[4 * LPT]) {
  const uint8_t *p = reinterpret_cast<const uint8_t *>(base) + off;
  if (whole) {
#pragma unroll
    for (int c = 0; c < 4 * LPT; ++c) v[c] = ld16(p, (uint64_t)c);
  } else {
#pragma unroll
    for (int j = 0; j < LPT; ++j) {
      u32x4 w[4];
      load_leaf(base, off + 64ull * j, nbytes, w);
#pragma unroll
      for (int c = 0; c < 4; ++c) v[4 * j + c] = w[c];
    }
  }
}

__device__ __forceinline__ int ilog2(uint32_t x) { return 31 - __clz(x); }

// One workgroup per block, LPT leaves per lane; levels: LPT in registers,
// up to six across the lanes of a wave, the rest through LDS.
template <int LPT, bool WHOLE>
__global__ __launch_bounds__(LPT == 4 ? 256 : (LPT == 2 ? 64 : 1024)) void k_fingerprint(
    const void *buf, uint64_t nbytes, uint64_t block_bytes, uint64_t *fp_out, uint64_t blk0) {
  __shared__ uint64_t sh[16];
  const uint64_t blk = blk0 + blockIdx.x;
  const uint64_t off = blk * block_bytes + (uint64_t)threadIdx.x * (64ull * LPT);
  u32x4 v[4 * LPT];
  load_leaves<LPT>(buf, off, nbytes, WHOLE, v);
  const uint32_t nth = blockDim.x;
  const int wl = nth >= 64 ? 6 : ilog2(nth);
  const uint64_t h = lane_tree(lane_subtree<LPT>(v), wl);
  if ((threadIdx.x & 63u) == 0) sh[threadIdx.x >> 6] = h;
  __syncthreads();
  if (threadIdx.x == 0) fp_out[blk] = lds_tree(sh, (nth + 63) >> 6);
}

// ---- block vote ------------------------------------------------------------
// Workspace accumulators: [0] disagree blocks, [1] fallback blocks,
// [2] unresolved elements, [3..3+K) replica blocks.
constexpr int kBlkAcc = 3 + FTV_MAX_K;

// Store the lane's piece (LPT x 64 bytes at byte offset `off`) of the
// consensus -- bytes past the end are not written -- and, optionally, zero the
// mask bytes of its elements.
template <int LPT>
__device__ __forceinline__ void put_piece(const BlockVoteD &b, uint64_t off, const u32x4 (&v)[4 * LPT],
                                          bool whole, bool mask_too) {
  uint8_t *cb = reinterpret_cast<uint8_t *>(b.cons) + off;
  const uint64_t es = b.dtype == FTV_F32 || b.dtype == FTV_I32 ? 4 : 8;
  if (whole) {
#pragma unroll
    for (int c = 0; c < 4 * LPT; ++c) st16(cb, (uint64_t)c, v[c], true);
    if (mask_too && b.mask) {
      uint32_t *mw = reinterpret_cast<uint32_t *>(b.mask + off / es);
      for (uint64_t q = 0; q < (64ull * LPT / es) / 4; ++q) st_nt(mw + q, 0u, true);
    }
    return;
  }
  // the buffer ends inside this piece (its size is a multiple of 4 bytes)
  uint32_t *dst = reinterpret_cast<uint32_t *>(cb);
#pragma unroll
  for (int c = 0; c < 4 * LPT; ++c) {
    if (off + 16ull * c + 0 < b.nbytes) dst[4 * c + 0] = v[c].x;
    if (off + 16ull * c + 4 < b.nbytes) dst[4 * c + 1] = v[c].y;
    if (off + 16ull * c + 8 < b.nbytes) dst[4 * c + 2] = v[c].z;
    if (off + 16ull * c + 12 < b.nbytes) dst[4 * c + 3] = v[c].w;
  }
  if (mask_too && b.mask) {
    const uint64_t e0 = off / es;
    const uint64_t end = off + 64ull * LPT < b.nbytes ? off + 64ull * LPT : b.nbytes;
    for (uint64_t e = e0; e < end / es; ++e) b.mask[e] = 0;
  }
}

// b.rep[r] for a runtime r, as a select chain: indexing the by-value kernel
// argument with a runtime index would copy it to scratch memory.
template <int K>
__device__ __forceinline__ const void *rep_ptr(const BlockVoteD &b, int r) {
  const void *p = b.rep[0];
#pragma unroll
  for (int j = 1; j < K; ++j) p = (j == r) ? b.rep[j] : p;
  return p;
}

// Pass 1: fingerprints of the block in all k replicas, their vote, the block
// map, and the restore.  Replica 0's piece is written to the consensus while
// it is hashed (one replica's leaves per lane are live at a time); only a
// block whose majority fingerprint differs from replica 0's is copied again,
// from the source replica.  Blocks without a majority are left to pass 2,
// which rewrites their consensus and mask.
// Hash the lane's piece of every replica (one replica at a time, not
// unrolled, so that only one replica's leaves are live) and stream replica
// 0's piece into the consensus.  WHOLE: the block lies inside the buffer.
template <int K, int LPT, bool WHOLE>
__device__ __forceinline__ void hash_replicas(const BlockVoteD &b, uint64_t off, int wl,
                                              uint64_t (*sh)[16]) {
  const bool mine = off < b.nbytes;
#pragma unroll 1
  for (int r = 0; r < K; ++r) {
    u32x4 v[4 * LPT];
    load_leaves<LPT>(rep_ptr<K>(b, r), off, b.nbytes, WHOLE, v);
    if (r == 0 && mine) put_piece<LPT>(b, off, v, WHOLE, true);
    const uint64_t h = lane_tree(lane_subtree<LPT>(v), wl);
    if ((threadIdx.x & 63u) == 0) sh[r][threadIdx.x >> 6] = h;
  }
}

// WHOLE: every block of the launch lies inside the buffer (all but a partial
// last block, which gets a launch of its own with WHOLE = false, LPT = 1).
template <int K, int LPT, bool WHOLE>
__global__ __launch_bounds__(LPT == 4 ? 256 : (LPT == 2 ? 64 : 1024)) void k_vote_blocks(BlockVoteD b,
                                                                                       uint64_t blk0) {
  __shared__ uint64_t sh[K][16];
  const uint64_t blk = blk0 + blockIdx.x;
  const uint64_t off = blk * b.block_bytes + (uint64_t)threadIdx.x * (64ull * LPT);
  const uint32_t nth = blockDim.x;
  const uint32_t nw = (nth + 63) >> 6;
  const int wl = nth >= 64 ? 6 : ilog2(nth);
  constexpr bool whole = WHOLE;
  const bool mine = off < b.nbytes;
  hash_replicas<K, LPT, WHOLE>(b, off, wl, sh);
  __syncthreads();
  if (threadIdx.x < (uint32_t)K) {
    const uint32_t r = threadIdx.x;
    const uint64_t f = lds_tree(sh[r], nw);
    sh[r][0] = f;
    if (b.fps) b.fps[(uint64_t)r * b.nblocks + blk] = f;
  }
  __syncthreads();
  uint64_t fp_r[K];
#pragma unroll
  for (int r = 0; r < K; ++r) fp_r[r] = sh[r][0];
  // vote of the fingerprints (uniform across the workgroup)
  int M = 0, src = 0;
#pragma unroll
  for (int r = 0; r < K; ++r) {
    int s = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) s += fp_r[r] == fp_r[j];
    if (s > M) {
      M = s;
      src = r;
    }
  }
  uint32_t bm = 0;
#pragma unroll
  for (int r = 0; r < K; ++r) bm |= (uint32_t)(fp_r[r] != fp_r[src]) << r;
  const bool majority = 2 * M > K;
  if (!majority) bm |= 0x80u;
  if (majority && (bm & 1u) && mine) {  // replica 0 is not the majority: recopy
    u32x4 v[4 * LPT];
    load_leaves<LPT>(rep_ptr<K>(b, src), off, b.nbytes, whole, v);
    put_piece<LPT>(b, off, v, whole, false);
  }
  if (threadIdx.x == 0) {
    b.blockmap[blk] = (uint8_t)bm;
    if (bm & 0x7fu) atomicAdd((unsigned long long *)&b.acc[0], 1ull);
    if (!majority) atomicAdd((unsigned long long *)&b.acc[1], 1ull);
    for (int r = 0; r < K; ++r)
      if ((bm >> r) & 1u) atomicAdd((unsigned long long *)&b.acc[3 + r], 1ull);
  }
}

// Pass 2: element vote of every block without a fingerprint majority (a
// grid-stride scan of the block map), then the last workgroup writes the
// stats and clears the workspace.
template <int DT, int TOL, int K>
__global__ __launch_bounds__(256) void k_blocks_fallback(BlockVoteD b) {
  using W = typename VT<DT>::W;
  __shared__ uint64_t sh[16 * kNumCounters];
  __shared__ uint32_t s_last;
  constexpr int NC = Acc<K>::NC;
  const uint64_t per = b.block_bytes / sizeof(W);
  const uint64_t n = b.nbytes / sizeof(W);
  Acc<K> acc;
  acc.zero();
  // the block's task record lives in LDS: a local record indexed at run time
  // (the rare general vote does) would be placed in scratch memory
  __shared__ TaskD t;
  for (uint64_t blk = blockIdx.x; blk < b.nblocks; blk += gridDim.x) {
    if (!(b.blockmap[blk] & 0x80u)) continue;
    const uint64_t e0 = blk * per;
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
    vote_range<DT, TOL, K, true, 1>(t, 0, t.nvec, acc, false);
    vote_tail<DT, TOL, K>(t, acc);
  }
  const uint64_t tot = block_total<K>(acc, sh);
  if (threadIdx.x == (uint32_t)(NC - 1) && tot)
    atomicAdd((unsigned long long *)&b.acc[2], (unsigned long long)tot);
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t prev = __hip_atomic_fetch_add(b.ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    s_last = prev + 1 == gridDim.x;
  }
  __syncthreads();
  if (!s_last || threadIdx.x != 0) return;
  __threadfence();
  uint64_t a[kBlkAcc];
  for (int i = 0; i < kBlkAcc; ++i)
    a[i] = __hip_atomic_load(&b.acc[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
  for (int i = 0; i < kBlkAcc; ++i)
    __hip_atomic_store(&b.acc[i], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(b.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_blocks_empty(ftv_block_stats *st) {
  if (threadIdx.x == 0) {
    st->blocks = st->disagree_blocks = st->fallback_blocks = st->unresolved_elems = 0;
    for (int r = 0; r < FTV_MAX_K; ++r) st->replica_blocks[r] = 0;
    st->verdict = FTV_UNANIMOUS;
    st->winner = 0;
  }
}

template <int DT, int TOL, int K>
hipError_t launch_fallback(const BlockVoteD &b, int num_cus, hipStream_t s) {
  uint64_t grid = (uint64_t)num_cus * 4;
  if (grid > b.nblocks) grid = b.nblocks;
  hipLaunchKernelGGL((k_blocks_fallback<DT, TOL, K>), dim3((uint32_t)grid), dim3(256), 0, s, b);
  return hipGetLastError();
}

// Leaves per lane: 4 when the block has at least 256 leaves, so that each
// lane combines two tree levels in registers; smaller blocks keep one wave.
inline int leaves_per_lane(uint64_t block_bytes) {
  const uint64_t leaves = block_bytes / 64;
  return leaves >= 256 ? 4 : (leaves >= 128 ? 2 : 1);
}

template <int K, int LPT>
hipError_t launch_blocks_kl(const BlockVoteD &b, hipStream_t s) {
  const uint64_t nwhole = b.nbytes / b.block_bytes;
  if (nwhole) {
    const dim3 grid((uint32_t)nwhole), block((uint32_t)(b.block_bytes / 64 / LPT));
    hipLaunchKernelGGL((k_vote_blocks<K, LPT, true>), grid, block, 0, s, b, (uint64_t)0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (nwhole < b.nblocks) {  // the partial last block
    hipLaunchKernelGGL((k_vote_blocks<K, 1, false>), dim3(1), dim3((uint32_t)(b.block_bytes / 64)), 0, s,
                       b, nwhole);
    return hipGetLastError();
  }
  return hipSuccess;
}

template <int K>
hipError_t launch_blocks_k(const BlockVoteD &b, int num_cus, hipStream_t s) {
  const int lpt = leaves_per_lane(b.block_bytes);
  hipError_t e = lpt == 4 ? launch_blocks_kl<K, 4>(b, s)
                          : (lpt == 2 ? launch_blocks_kl<K, 2>(b, s) : launch_blocks_kl<K, 1>(b, s));
  if (e != hipSuccess) return e;
  switch (b.dtype * 3 + b.tolkind) {
    case FTV_F32 * 3 + FTV_TOL_EXACT: return launch_fallback<FTV_F32, FTV_TOL_EXACT, K>(b, num_cus, s);
    case FTV_F32 * 3 + FTV_TOL_ULP: return launch_fallback<FTV_F32, FTV_TOL_ULP, K>(b, num_cus, s);
    case FTV_F32 * 3 + FTV_TOL_REL: return launch_fallback<FTV_F32, FTV_TOL_REL, K>(b, num_cus, s);
    case FTV_F64 * 3 + FTV_TOL_EXACT: return launch_fallback<FTV_F64, FTV_TOL_EXACT, K>(b, num_cus, s);
    case FTV_F64 * 3 + FTV_TOL_ULP: return launch_fallback<FTV_F64, FTV_TOL_ULP, K>(b, num_cus, s);
    case FTV_F64 * 3 + FTV_TOL_REL: return launch_fallback<FTV_F64, FTV_TOL_REL, K>(b, num_cus, s);
    case FTV_I32 * 3 + FTV_TOL_EXACT: return launch_fallback<FTV_I32, FTV_TOL_EXACT, K>(b, num_cus, s);
    case FTV_I64 * 3 + FTV_TOL_EXACT: return launch_fallback<FTV_I64, FTV_TOL_EXACT, K>(b, num_cus, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_fingerprint(const void *buf, uint64_t nbytes, uint64_t block_bytes,
                              uint64_t *fp_out, hipStream_t s) {
  const uint64_t nblocks = (nbytes + block_bytes - 1) / block_bytes;
  if (nblocks == 0) return hipSuccess;
  const int lpt = leaves_per_lane(block_bytes);
  const uint64_t nwhole = nbytes / block_bytes;
  if (nwhole) {
    const dim3 grid((uint32_t)nwhole), block((uint32_t)(block_bytes / 64 / lpt));
    const uint64_t z = 0;
    if (lpt == 4) hipLaunchKernelGGL((k_fingerprint<4, true>), grid, block, 0, s, buf, nbytes, block_bytes, fp_out, z);
    else if (lpt == 2) hipLaunchKernelGGL((k_fingerprint<2, true>), grid, block, 0, s, buf, nbytes, block_bytes, fp_out, z);
    else hipLaunchKernelGGL((k_fingerprint<1, true>), grid, block, 0, s, buf, nbytes, block_bytes, fp_out, z);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (nwhole < nblocks)  // the partial last block
    hipLaunchKernelGGL((k_fingerprint<1, false>), dim3(1), dim3((uint32_t)(block_bytes / 64)), 0, s, buf, nbytes,
                       block_bytes, fp_out, nwhole);
  return hipGetLastError();
}

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
