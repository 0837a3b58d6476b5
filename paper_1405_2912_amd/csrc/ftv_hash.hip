// ftv_hash.hip -- block fingerprints and pass 1 of the block vote for gfx950.
//
// Fingerprint of a block (power-of-two size BB in [4 KiB, 64 KiB]): the block
// is read as little-endian 64-bit words, zero-padded past the end of the
// buffer; a leaf is 64-bit FNV-1a over 8 consecutive words (64 B) and leaves
// are combined pairwise, level by level, a node being FNV-1a over the two words
// (left, right).
//
// Whole blocks: one workgroup per block walks it in sub-chunks of 64*L*T
// bytes, T threads holding L consecutive leaves each (L = 2 and T = 128 for
// blocks of 16 KiB and more).  The sub-chunk is read with fully coalesced
// 16-byte loads (chunk c*T + t to thread t, so each load instruction of a
// wave covers 1 KiB of consecutive bytes), transposed through LDS
// (double-buffered, XOR-swizzled so that neither the writes nor the
// leaf-major reads conflict on banks) so that thread t then holds leaves
// L*t .. L*t+L-1.  The leaves of a thread are combined in registers, the next
// six tree levels across the lanes of a wave, the next ones over the wave
// roots in LDS and the last over the sub-chunk roots.  Two leaves per lane
// halve the lane-tree work per byte (with one leaf per lane the six lane
// levels cost more multiplies than the leaf itself).  The loads of the next
// sub-chunk are in flight while the current one is hashed.  Reading each
// lane's own 64-byte leaf directly from HBM instead (lanes 64 bytes apart in
// every load) measured 1.6x slower.
//
// Pass 1 of the block vote fingerprints every block of every replica,
// replica after replica, so the chip streams one replica at a time (on
// MI355X five replicas read at the same offsets together streamed about 15%
// slower than one after another); replica 0's data is streamed into the
// consensus while it is hashed.  Pass 2 (ftv_blocks.hip) votes the
// fingerprints.
//
// A partial last block (the buffer ends inside it) is handled by one
// workgroup of BB/64 threads reading its leaves directly, with zero padding.
//
// These kernels live in a code object of their own, apart from the 48
// block-vote scan kernels (about 1 MB of code): a large code object measured
// slower for the vote kernels, and here the split gained about 1%.
#include <string.h>

#include "ftv_blocks_dev.hpp"
#include "ftv_internal.hpp"
#include "ftv_vote_dev.hpp"

namespace ftv {
namespace {

using namespace dev;
using namespace blockdev;

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

// ---- whole blocks: coalesced loads transposed through LDS -----------------
// Threads per whole-block workgroup at most.
constexpr uint32_t kBlockT = 128;

// Geometry of a whole block of BB bytes (a power of two in [4 KiB, 64 KiB]),
// fixed at compile time so that every load and store offset of a step folds
// into the instruction: L leaves per lane and T threads -- two leaves and 128
// threads (16 KiB sub-chunks) from 16 KiB on, one wave for smaller blocks --
// and NSUB sub-chunks of SUB bytes.  On MI355X the read-only pass over 2 GiB
// of 64 KiB blocks takes 0.297-0.300 ms in this shape (a plain read of the
// same bytes: 0.297-0.299 ms), 0.298-0.306 ms with one leaf per lane in 256
// threads, and the same with four leaves per lane in one-wave workgroups
// (twice the registers); with its geometry read at run time from the block
// size and the workgroup size it measured 4-6% slower.
template <uint32_t BB>
struct Geo {
  static constexpr int L = BB < 8192 ? 1 : 2;
  static constexpr uint32_t T = BB < 8192 ? BB / 64 : (BB / 128 < kBlockT ? BB / 128 : kBlockT);
  static constexpr uint32_t SUB = 64u * L * T;  // bytes per sub-chunk
  static constexpr uint32_t NSUB = BB / SUB;
  static constexpr uint32_t CHUNKS = SUB / 16;  // 16-byte chunks per sub-chunk
  static constexpr uint32_t NBUF = NSUB > 1 ? 2 : 1;
  static_assert(T % 64 == 0 && NSUB >= 1 && NSUB <= 4 && NSUB * SUB == BB, "block geometry");
};

// LDS slot of 16-byte chunk g of a sub-chunk.  Thread t writes chunks c*T + t
// and reads chunks 4Lt .. 4Lt+4L-1; XOR-ing bits 0..log2(4L)-1 with the bits
// above bit 3 makes every group of 16 lanes hit 16 distinct 16-byte bank
// groups in both patterns.  The slot stays within the chunk's group of 16.
template <int L>
__device__ __forceinline__ uint32_t lds_slot(uint32_t g) { return g ^ ((g >> 4) & (4u * L - 1u)); }

// Sub-chunk `sub` of the block at byte offset boff: thread t takes chunks
// c*T + t.
template <class G>
__device__ __forceinline__ void load_sub(const void *buf, uint64_t boff, uint32_t sub, u32x4 (&v)[4 * G::L]) {
  const uint8_t *p = reinterpret_cast<const uint8_t *>(buf) + boff + sub * G::SUB + 16u * threadIdx.x;
#pragma unroll
  for (int c = 0; c < 4 * G::L; ++c) v[c] = ld16(p, (uint64_t)c * G::T);
}

// Root of a thread's L consecutive leaves (chunks 4Lt .. 4Lt+4L-1 of the
// LDS tile), the leaves hashed side by side.
template <int L>
__device__ __forceinline__ uint64_t thread_root(const u32x4 *lbuf, uint32_t t) {
  uint64_t h[L];
#pragma unroll
  for (int l = 0; l < L; ++l) h[l] = kFnvBasis;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    u32x4 x[L];
#pragma unroll
    for (int l = 0; l < L; ++l) x[l] = lbuf[lds_slot<L>(4u * L * t + 4u * l + q)];
#pragma unroll
    for (int l = 0; l < L; ++l) {
      h[l] = fnv_step(h[l], (uint64_t)x[l].x | ((uint64_t)x[l].y << 32));
      h[l] = fnv_step(h[l], (uint64_t)x[l].z | ((uint64_t)x[l].w << 32));
    }
  }
#pragma unroll
  for (int w = 1; w < L; w *= 2)
#pragma unroll
    for (int l = 0; l < L; l += 2 * w) h[l] = fnv_node(h[l], h[l + w]);
  return h[0];
}

// Hash sub-chunk `sub` held in v into sroot[sub]; with CONS its chunks also
// go to the consensus and the mask bytes of its elements are zeroed.
template <class G, bool CONS>
__device__ __forceinline__ void hash_sub(const BlockVoteD &b, uint64_t boff, uint32_t sub,
                                         const u32x4 (&v)[4 * G::L], u32x4 *lbuf, uint64_t *sw, uint64_t *sroot) {
  constexpr int L = G::L;
  const uint32_t t = threadIdx.x;
  const uint64_t soff = boff + sub * G::SUB;
  if (CONS) {
    const uintptr_t cb = reinterpret_cast<uintptr_t>(b.cons) + soff;
#pragma unroll
    for (int c = 0; c < 4 * L; ++c) stream_store16(cb, (c * G::T + t) * 16u, v[c]);
    if (b.mask) {
      // 64*L bytes of the sub-chunk per thread = 16L (4-byte) or 8L (8-byte)
      // elements; whole 16-byte stores where they fit, so that each store
      // instruction covers whole lines
      const bool four = b.dtype == FTV_F32 || b.dtype == FTV_I32;
      const uintptr_t mb = reinterpret_cast<uintptr_t>(b.mask) + (four ? soff / 4 : soff / 8);
      if (four) {
#pragma unroll
        for (int j = 0; j < L; ++j) stream_store16(mb, (j * G::T + t) * 16u, u32x4{0u, 0u, 0u, 0u});
      } else if (L == 2) {
        stream_store16(mb, t * 16u, u32x4{0u, 0u, 0u, 0u});
      } else {
        stream_store8(mb, t * 8u, 0ull);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 4 * L; ++c) lbuf[lds_slot<L>((uint32_t)c * G::T + t)] = v[c];
  __syncthreads();
  const uint64_t h = lane_tree(thread_root<L>(lbuf, t), 6);
  if ((t & 63u) == 0) sw[t >> 6] = h;
  __syncthreads();
  if (t == 0) sroot[sub] = lds_tree(sw, G::T / 64);
}

// Fingerprint of block `blk` of buf, the next sub-chunk's loads in flight
// while one is hashed (CONS: also streamed into the consensus).
template <uint32_t BB, bool CONS>
__device__ __forceinline__ uint64_t hash_block(const BlockVoteD &b, const void *buf, uint64_t blk,
                                               u32x4 (*lbuf)[Geo<BB>::CHUNKS], uint64_t *sw, uint64_t *sroot) {
  using G = Geo<BB>;
  const uint64_t boff = blk * BB;
  u32x4 va[4 * G::L], vb[4 * G::L];
  load_sub<G>(buf, boff, 0, va);
#pragma unroll
  for (uint32_t s = 0; s < G::NSUB; s += 2) {
    if (s + 1 < G::NSUB) load_sub<G>(buf, boff, s + 1, vb);
    hash_sub<G, CONS>(b, boff, s, va, lbuf[0], sw, sroot);
    if (s + 1 < G::NSUB) {
      if (s + 2 < G::NSUB) load_sub<G>(buf, boff, s + 2, va);
      hash_sub<G, CONS>(b, boff, s + 1, vb, lbuf[G::NBUF - 1], sw, sroot);
    }
  }
  __syncthreads();
  uint64_t root = 0;  // thread 0's is the fingerprint
  if (threadIdx.x == 0) root = lds_tree(sroot, G::NSUB);
  return root;
}

// The block a workgroup hashes.  The hardware deals workgroups out to the 8
// XCDs round robin; within each run of 8 x kXcdRun workgroups the index is
// permuted so that the workgroups of one XCD take kXcdRun adjacent blocks
// (the grid's last, partial run keeps the plain order).  On the 2 GiB
// fingerprint in 64 KiB blocks this measured 0.295-0.296 ms against
// 0.302 ms in the plain order, and the k = 5 fp64 16384^2 block vote
// 1.98-1.99 ms against 2.10-2.11 ms (runs of 4: 2.00-2.01, of 16: 1.99-2.00).
constexpr uint32_t kXcdRun = 64;
__device__ __forceinline__ uint32_t xcd_block(uint32_t bx, uint32_t nx) {
  constexpr uint32_t C = 8u * kXcdRun;
  const uint32_t base = bx / C * C;
  if (base + C > nx) return bx;
  return base + (bx % 8u) * kXcdRun + (bx % C) / 8u;
}

// Block xcd_block(blockIdx.x) of buffer blockIdx.y (one of b.k buffers).
template <uint32_t BB>
__global__ __launch_bounds__(Geo<BB>::T) void k_fingerprint(BlockVoteD b) {
  using G = Geo<BB>;
  __shared__ u32x4 lbuf[G::NBUF][G::CHUNKS];
  __shared__ uint64_t sw[G::T / 64];
  __shared__ uint64_t sroot[G::NSUB];
  const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
  const uint64_t root = hash_block<BB, false>(b, rep_ptr<FTV_MAX_K>(b, (int)blockIdx.y), blk, lbuf, sw, sroot);
  if (threadIdx.x == 0) b.fps[(uint64_t)blockIdx.y * b.nblocks + blk] = root;
}

// Pass 1 over whole blocks: the fingerprints of every whole block of the k
// replicas, one workgroup per (block, replica; blocks in the XCD order of
// xcd_block), dispatched replica after
// replica (blockIdx.y outer), so that the chip streams one replica at a time;
// the workgroups of replica 0 also stream its data into the consensus and
// zero the mask bytes of its elements.  The vote of the fingerprints, the
// block map and the re-copy of blocks where replica 0 is outvoted are pass 2's.
template <uint32_t BB>
__global__ __launch_bounds__(Geo<BB>::T) void k_hash_replicas(BlockVoteD b) {
  using G = Geo<BB>;
  __shared__ u32x4 lbuf[G::NBUF][G::CHUNKS];
  __shared__ uint64_t sw[G::T / 64];
  __shared__ uint64_t sroot[G::NSUB];
  const void *buf = rep_ptr<FTV_MAX_K>(b, (int)blockIdx.y);
  const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
  const uint64_t root = blockIdx.y == 0 ? hash_block<BB, true>(b, buf, blk, lbuf, sw, sroot)
                                        : hash_block<BB, false>(b, buf, blk, lbuf, sw, sroot);
  if (threadIdx.x == 0) b.fps[(uint64_t)blockIdx.y * b.nblocks + blk] = root;
}

// Whole blocks of the first m buffers of b: pass 1 of the block vote (VOTE)
// or plain fingerprints, the geometry chosen by the block size.
template <uint32_t BB>
hipError_t launch_whole_bb(const BlockVoteD &b, uint64_t nwhole, uint32_t m, bool vote, hipStream_t s) {
  const dim3 grid((uint32_t)nwhole, m), block(Geo<BB>::T);
  if (vote) hipLaunchKernelGGL(k_hash_replicas<BB>, grid, block, 0, s, b);
  else hipLaunchKernelGGL(k_fingerprint<BB>, grid, block, 0, s, b);
  return hipGetLastError();
}

hipError_t launch_whole(const BlockVoteD &b, uint64_t nwhole, uint32_t m, bool vote, hipStream_t s) {
  switch (b.block_bytes) {
    case 4096: return launch_whole_bb<4096>(b, nwhole, m, vote, s);
    case 8192: return launch_whole_bb<8192>(b, nwhole, m, vote, s);
    case 16384: return launch_whole_bb<16384>(b, nwhole, m, vote, s);
    case 32768: return launch_whole_bb<32768>(b, nwhole, m, vote, s);
    case 65536: return launch_whole_bb<65536>(b, nwhole, m, vote, s);
  }
  return hipErrorInvalidValue;
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

}  // namespace

hipError_t launch_blocks_hash(const BlockVoteD &b, hipStream_t s) {
  const uint64_t nwhole = b.nbytes / b.block_bytes;
  if (nwhole) {
    const hipError_t e = launch_whole(b, nwhole, b.k, true, s);
    if (e != hipSuccess) return e;
  }
  if (nwhole < b.nblocks) {  // the partial last block
    const dim3 g(1), t((uint32_t)(b.block_bytes / 64));
    switch (b.k) {
      case 2: hipLaunchKernelGGL(k_vote_block_partial<2>, g, t, 0, s, b, nwhole); break;
      case 3: hipLaunchKernelGGL(k_vote_block_partial<3>, g, t, 0, s, b, nwhole); break;
      case 4: hipLaunchKernelGGL(k_vote_block_partial<4>, g, t, 0, s, b, nwhole); break;
      case 5: hipLaunchKernelGGL(k_vote_block_partial<5>, g, t, 0, s, b, nwhole); break;
      case 6: hipLaunchKernelGGL(k_vote_block_partial<6>, g, t, 0, s, b, nwhole); break;
      case 7: hipLaunchKernelGGL(k_vote_block_partial<7>, g, t, 0, s, b, nwhole); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  return hipSuccess;
}

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
    const hipError_t e = launch_whole(b, nwhole, m, false, s);
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

}  // namespace ftv
