// ftv_blocks.hip -- block fingerprints and the fused block vote for gfx950.
//
// Fingerprint of a block (power-of-two size BB in [4 KiB, 64 KiB]): the block
// is read as little-endian 64-bit words, zero-padded past the end of the
// buffer; a leaf is 64-bit FNV-1a over 8 consecutive words (64 B) and leaves
// are combined pairwise, level by level, a node being FNV-1a over the two words
// (left, right).
//
// Whole blocks: one workgroup of T = min(256, BB/64) threads per block walks
// it in sub-chunks of 64*T bytes (one leaf per thread).  The sub-chunk is
// read with fully coalesced 16-byte loads (chunk c*T + t to thread t, so each
// load instruction of a wave covers 1 KiB of consecutive bytes), transposed
// through LDS (double-buffered, XOR-swizzled so that neither the writes nor
// the leaf-major reads conflict on banks) so that thread t then holds leaf t.
// The first six tree levels are combined across the lanes of a wave, the next
// (up to two) over the wave roots in LDS, the last (up to two) over the
// sub-chunk roots.  The loads of the next sub-chunk are in flight while the
// current one is hashed.  Reading each lane's own 64-byte leaf directly from
// HBM instead (lanes 64 bytes apart in every load) measured 1.6x slower.
//
// Block vote, two passes.  Pass 1 fingerprints every block of every replica,
// replica after replica, so the chip streams one replica at a time (on
// MI355X five replicas read at the same offsets together streamed about 15%
// slower than one after another); replica 0's data is streamed into the
// consensus while it is hashed.  Pass 2 votes the k fingerprints of each
// block by exact equality, writes the block map and its counts, re-copies
// the blocks whose strict-majority fingerprint is not replica 0's from the
// lowest-indexed replica holding it (in the common case replica 0 agrees and
// the restore cost one write pass and no extra read), and runs the element
// vote over every block without a majority; a one-workgroup finalize kernel
// writes the stats.  No kernel waits on another's workgroups: kernel
// boundaries on the stream order them.
//
// A partial last block (the buffer ends inside it) is handled by one
// workgroup of BB/64 threads reading its leaves directly, with zero padding.
#include <string.h>

#include "ftv_internal.hpp"
#include "ftv_vote_dev.hpp"

namespace ftv {
namespace {

using namespace dev;

constexpr uint64_t kFnvBasis = 0xcbf29ce484222325ull;

// (h ^ w) * 0x100000001b3 mod 2^64.  With x = hi:lo and the prime split as
// 2^40 + 0x1b3: x * P = lo * 0x1b3 + ((hi * 0x1b3 + (lo << 8)) mod 2^32) * 2^32
// (mod 2^64) -- one 32x32->64 multiply-add and one 32-bit multiply.
__device__ __forceinline__ uint64_t fnv_step(uint64_t h, uint64_t w) {
  const uint64_t x = h ^ w;
  const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
  const uint32_t upper = hi * 0x1b3u + (lo << 8);
  return (uint64_t)lo * 0x1b3u + ((uint64_t)upper << 32);
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

// Reduce `nw` roots in LDS (pairwise, in order) to one.
__device__ __forceinline__ uint64_t lds_tree(uint64_t *sh, uint32_t nw) {
  for (uint32_t len = nw; len > 1; len >>= 1)
    for (uint32_t j = 0; j < len / 2; ++j) sh[j] = fnv_node(sh[2 * j], sh[2 * j + 1]);
  return sh[0];
}

__device__ __forceinline__ int ilog2(uint32_t x) { return 31 - __clz(x); }

// b.rep[r] for a runtime r, as a select chain: indexing the by-value kernel
// argument with a runtime index would copy it to scratch memory.
template <int K>
__device__ __forceinline__ const void *rep_ptr(const BlockVoteD &b, int r) {
  const void *p = b.rep[0];
#pragma unroll
  for (int j = 1; j < K; ++j) p = (j == r) ? b.rep[j] : p;
  return p;
}

// ---- whole blocks: coalesced loads transposed through LDS -----------------
// Threads per whole-block workgroup: 256 (a 16 KiB sub-chunk per step, its
// LDS tile double-buffered in 32 KiB).  The read-only fingerprint pass of a
// 2 GiB buffer takes 0.33 ms with 256 threads against 0.40 ms with 512.
constexpr uint32_t kFingerprintT = 256;

// LDS slot of 16-byte chunk g of a sub-chunk.  Thread t writes chunks c*T + t
// and reads chunks 4t .. 4t+3; XOR-ing bits 0-1 with bits 4-5 makes every
// group of 16 lanes hit 16 distinct 16-byte bank groups in both patterns.
__device__ __forceinline__ uint32_t lds_slot(uint32_t g) { return g ^ ((g >> 4) & 3u); }

// Geometry of a whole-block walk: step s = (buffer s >> lg_nsub, sub-chunk
// s & (nsub - 1)); a sub-chunk is 64*T bytes.
struct Walk {
  uint64_t boff;      // byte offset of the block
  uint32_t nth;       // T
  uint32_t sub_bytes; // 64 * T
  uint32_t lg_nsub;
  uint32_t nsub;
};

template <int K>
__device__ __forceinline__ void load_step(const BlockVoteD &b, const Walk &w, uint32_t s, u32x4 (&v)[4]) {
  const uint32_t r = s >> w.lg_nsub, sub = s & (w.nsub - 1);
  const uint8_t *p = reinterpret_cast<const uint8_t *>(rep_ptr<K>(b, (int)r)) + w.boff +
                     (uint64_t)sub * w.sub_bytes + 16ull * threadIdx.x;
#pragma unroll
  for (int c = 0; c < 4; ++c) v[c] = ld16(p, (uint64_t)c * w.nth);
}

// Hash step s held in v: buffer 0's chunks also go to the consensus (mask
// bytes of their elements zeroed) when CONS.  Leaves sroot[r][sub].
template <bool CONS>
__device__ __forceinline__ void hash_step(const BlockVoteD &b, const Walk &w, uint32_t s, const u32x4 (&v)[4],
                                          u32x4 *lbuf, uint64_t *sw, uint64_t (*sroot)[4]) {
  const uint32_t t = threadIdx.x;
  const uint32_t r = s >> w.lg_nsub, sub = s & (w.nsub - 1);
  const uint64_t soff = w.boff + (uint64_t)sub * w.sub_bytes;
  if (CONS && r == 0) {
    const uintptr_t cb = reinterpret_cast<uintptr_t>(b.cons) + soff;
#pragma unroll
    for (int c = 0; c < 4; ++c) stream_store16(cb, (c * w.nth + t) * 16u, v[c]);
    if (b.mask) {
      // 64 bytes of the sub-chunk per thread = 8 (8-byte) or 16 (4-byte) elements
      const uint32_t es = b.dtype == FTV_F32 || b.dtype == FTV_I32 ? 4u : 8u;
      const uint32_t per = 64u / es;
      // one store per thread, so that each store instruction covers whole lines
      const uintptr_t mb = reinterpret_cast<uintptr_t>(b.mask) + soff / es;
      if (per == 16) stream_store16(mb, t * 16u, u32x4{0u, 0u, 0u, 0u});
      else stream_store8(mb, t * 8u, 0ull);
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) lbuf[lds_slot((uint32_t)c * w.nth + t)] = v[c];
  __syncthreads();
  u32x4 leaf[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) leaf[q] = lbuf[lds_slot(4u * t + q)];
  const uint64_t h = lane_tree(leaf_hash(leaf), 6);
  if ((t & 63u) == 0) sw[t >> 6] = h;
  __syncthreads();
  if (t == 0) sroot[r][sub] = lds_tree(sw, w.nth >> 6);
}

// Sub-chunk roots of block `blk` in the first K buffers of b (K = 1:
// fingerprints of b.rep[0]), the next step's loads in flight while one is
// hashed.  Ends with a barrier: sroot is then complete.
template <int K, bool CONS, uint32_t T>
__device__ __forceinline__ void walk_block(const BlockVoteD &b, const Walk &w, u32x4 (*lbuf)[4 * T],
                                           uint64_t *sw, uint64_t (*sroot)[4]) {
  const uint32_t nstep = (uint32_t)K << w.lg_nsub;
  u32x4 va[4], vb[4];
  load_step<K>(b, w, 0, va);
  for (uint32_t s = 0; s < nstep; s += 2) {
    if (s + 1 < nstep) load_step<K>(b, w, s + 1, vb);
    hash_step<CONS>(b, w, s, va, lbuf[0], sw, sroot);
    if (s + 1 >= nstep) break;
    if (s + 2 < nstep) load_step<K>(b, w, s + 2, va);
    hash_step<CONS>(b, w, s + 1, vb, lbuf[1], sw, sroot);
  }
  __syncthreads();
}

__device__ __forceinline__ Walk make_walk(uint64_t blk, uint64_t block_bytes) {
  Walk w;
  w.nth = blockDim.x;
  w.sub_bytes = 64u * w.nth;
  w.nsub = (uint32_t)(block_bytes / w.sub_bytes);
  w.lg_nsub = (uint32_t)ilog2(w.nsub);
  w.boff = blk * block_bytes;
  return w;
}

// Block blockIdx.x of buffer blockIdx.y (one of b.k buffers).
__global__ __launch_bounds__(kFingerprintT) void k_fingerprint(BlockVoteD b) {
  __shared__ u32x4 lbuf[2][4 * kFingerprintT];
  __shared__ uint64_t sw[kFingerprintT / 64];
  __shared__ uint64_t sroot[1][4];
  BlockVoteD one = b;
  one.rep[0] = rep_ptr<FTV_MAX_K>(b, (int)blockIdx.y);
  const Walk w = make_walk(blockIdx.x, b.block_bytes);
  walk_block<1, false, kFingerprintT>(one, w, lbuf, sw, sroot);
  if (threadIdx.x == 0) b.fps[(uint64_t)blockIdx.y * b.nblocks + blockIdx.x] = lds_tree(sroot[0], w.nsub);
}

// ---- block vote ------------------------------------------------------------
// Workspace accumulators: [0] disagree blocks, [1] fallback blocks,
// [2] unresolved elements, [3..3+K) replica blocks; zero between calls.
constexpr int kBlkAcc = 3 + FTV_MAX_K;

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

// Pass 1 over whole blocks: the fingerprints of every whole block of the k
// replicas, one workgroup per (block, replica), dispatched replica after
// replica (blockIdx.y outer), so that the chip streams one replica at a time;
// the workgroups of replica 0 also stream its data into the consensus and
// zero the mask bytes of its elements.  The vote of the fingerprints, the
// block map and the re-copy of blocks where replica 0 is outvoted are pass 2's.
__global__ __launch_bounds__(kFingerprintT) void k_hash_replicas(BlockVoteD b) {
  __shared__ u32x4 lbuf[2][4 * kFingerprintT];
  __shared__ uint64_t sw[kFingerprintT / 64];
  __shared__ uint64_t sroot[1][4];
  BlockVoteD one = b;
  one.rep[0] = rep_ptr<FTV_MAX_K>(b, (int)blockIdx.y);
  const Walk w = make_walk(blockIdx.x, b.block_bytes);
  if (blockIdx.y == 0) walk_block<1, true, kFingerprintT>(one, w, lbuf, sw, sroot);
  else walk_block<1, false, kFingerprintT>(one, w, lbuf, sw, sroot);
  if (threadIdx.x == 0) b.fps[(uint64_t)blockIdx.y * b.nblocks + blockIdx.x] = lds_tree(sroot[0], w.nsub);
}

// ---- the partial last block: one leaf per thread, read directly ------------
// (the buffer ends inside the block; bytes past the end hash as zero and are
// never written)
__device__ __forceinline__ uint64_t partial_block_root(const void *buf, uint64_t off, uint64_t nbytes,
                                                       uint64_t *sh, u32x4 (&v)[4]) {
  load_leaf(buf, off, nbytes, v);
  const uint32_t nth = blockDim.x;
  const uint64_t h = lane_tree(leaf_hash(v), 6);
  if ((threadIdx.x & 63u) == 0) sh[threadIdx.x >> 6] = h;
  __syncthreads();
  uint64_t root = 0;
  if (threadIdx.x == 0) root = lds_tree(sh, nth >> 6);
  __syncthreads();
  return root;
}

__global__ __launch_bounds__(1024) void k_fingerprint_partial(const void *buf, uint64_t nbytes,
                                                              uint64_t block_bytes, uint64_t *fp_out,
                                                              uint64_t blk) {
  __shared__ uint64_t sh[16];
  u32x4 v[4];
  const uint64_t root = partial_block_root(buf, blk * block_bytes + 64ull * threadIdx.x, nbytes, sh, v);
  if (threadIdx.x == 0) fp_out[blk] = root;
}

// Consensus piece of a lane of the partial block: its 64 bytes up to the end
// of the buffer (a multiple of 4 bytes), and optionally the mask bytes of its
// elements zeroed.
__device__ __forceinline__ void put_partial(const BlockVoteD &b, uint64_t off, const u32x4 (&v)[4], bool mask_too) {
  uint32_t *dst = reinterpret_cast<uint32_t *>(reinterpret_cast<uint8_t *>(b.cons) + off);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (off + 16ull * c + 0 < b.nbytes) dst[4 * c + 0] = v[c].x;
    if (off + 16ull * c + 4 < b.nbytes) dst[4 * c + 1] = v[c].y;
    if (off + 16ull * c + 8 < b.nbytes) dst[4 * c + 2] = v[c].z;
    if (off + 16ull * c + 12 < b.nbytes) dst[4 * c + 3] = v[c].w;
  }
  if (mask_too && b.mask) {
    const uint64_t es = b.dtype == FTV_F32 || b.dtype == FTV_I32 ? 4 : 8;
    const uint64_t end = off + 64 < b.nbytes ? off + 64 : b.nbytes;
    for (uint64_t e = off / es; e < end / es; ++e) b.mask[e] = 0;
  }
}

template <int K>
__global__ __launch_bounds__(1024) void k_vote_block_partial(BlockVoteD b, uint64_t blk) {
  __shared__ uint64_t sh[16];
  __shared__ uint64_t s_fp[K];
  const uint64_t off = blk * b.block_bytes + 64ull * threadIdx.x;
  const bool mine = off < b.nbytes;
#pragma unroll 1
  for (int r = 0; r < K; ++r) {
    u32x4 v[4];
    const uint64_t root = partial_block_root(rep_ptr<K>(b, r), off, b.nbytes, sh, v);
    if (r == 0 && mine) put_partial(b, off, v, true);
    if (threadIdx.x == 0) {
      s_fp[r] = root;
      if (b.fps) b.fps[(uint64_t)r * b.nblocks + blk] = root;
    }
  }
  __syncthreads();
  uint64_t f[K];
#pragma unroll
  for (int r = 0; r < K; ++r) f[r] = s_fp[r];
  int src = 0;
  const uint32_t bm = vote_fps<K>(f, &src);
  if (!(bm & 0x80u) && (bm & 1u) && mine) {
    u32x4 v[4];
    load_leaf(rep_ptr<K>(b, src), off, b.nbytes, v);
    put_partial(b, off, v, false);
  }
  if (threadIdx.x == 0) b.blockmap[blk] = (uint8_t)bm;
}

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

// Threads of a whole-block workgroup: one leaf per thread per sub-chunk.
inline uint32_t block_threads(uint64_t block_bytes, uint32_t max_t) {
  const uint64_t leaves = block_bytes / 64;
  return (uint32_t)(leaves < max_t ? leaves : max_t);
}

template <int K>
hipError_t launch_blocks_hash(const BlockVoteD &b, hipStream_t s) {
  const uint64_t nwhole = b.nbytes / b.block_bytes;
  if (nwhole) {
    hipLaunchKernelGGL(k_hash_replicas, dim3((uint32_t)nwhole, (uint32_t)K),
                       dim3(block_threads(b.block_bytes, kFingerprintT)), 0, s, b);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (nwhole < b.nblocks) {  // the partial last block
    hipLaunchKernelGGL((k_vote_block_partial<K>), dim3(1), dim3((uint32_t)(b.block_bytes / 64)), 0, s, b,
                       nwhole);
    return hipGetLastError();
  }
  return hipSuccess;
}

template <int K>
hipError_t launch_blocks_k(const BlockVoteD &b, int num_cus, hipStream_t s) {
  const hipError_t e = launch_blocks_hash<K>(b, s);
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

hipError_t launch_fingerprints(const void *const *bufs, uint32_t m, uint64_t nbytes, uint64_t block_bytes,
                               uint64_t *fp_out, hipStream_t s) {
  const uint64_t nblocks = (nbytes + block_bytes - 1) / block_bytes;
  if (nblocks == 0 || m == 0) return hipSuccess;
  if (m > FTV_MAX_K) return hipErrorInvalidValue;
  const uint64_t nwhole = nbytes / block_bytes;
  if (nwhole) {
    BlockVoteD b;
    memset(&b, 0, sizeof(b));
    for (uint32_t j = 0; j < m; ++j) b.rep[j] = bufs[j];
    b.k = m;
    b.nbytes = nbytes;
    b.block_bytes = block_bytes;
    b.nblocks = nblocks;
    b.fps = fp_out;
    hipLaunchKernelGGL(k_fingerprint, dim3((uint32_t)nwhole, m), dim3(block_threads(block_bytes, kFingerprintT)), 0,
                       s, b);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  for (uint32_t j = 0; j < m && nwhole < nblocks; ++j) {  // the partial last blocks
    hipLaunchKernelGGL(k_fingerprint_partial, dim3(1), dim3((uint32_t)(block_bytes / 64)), 0, s, bufs[j], nbytes,
                       block_bytes, fp_out + (uint64_t)j * nblocks, nwhole);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_fingerprint(const void *buf, uint64_t nbytes, uint64_t block_bytes,
                              uint64_t *fp_out, hipStream_t s) {
  return launch_fingerprints(&buf, 1, nbytes, block_bytes, fp_out, s);
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
