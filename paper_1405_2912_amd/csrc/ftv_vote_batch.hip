// ftv_vote_batch.hip -- the batched (persistent) vote kernel for gfx950, the
// serving iteration kernels, and the per-task dispatch by value type.
//
// Batched launch: one persistent grid pulls tiles from an atomic queue over a
// table of (task, vector range) entries; a tile may belong to any task, so the
// body dispatches on the task's (value type, tolerance, k) code, a
// workgroup-uniform branch.  Per tile the workgroup adds its non-zero counts
// to the task's accumulators; a finalize kernel writes every task's stats.
#include <algorithm>

#include "ftv_internal.hpp"
#include "ftv_vote_dev.hpp"

namespace ftv {
namespace {

using namespace dev;

// ---- batched persistent launch -------------------------------------------
template <int DT, int TOL, int K>
__device__ __forceinline__ void run_tile(const TaskD &t, const TileD &tile, const BatchLaunch &b,
                                         uint64_t *sh) {
  constexpr int U = Unroll<K>::value;
  constexpr int NC = Acc<K>::NC;
  Acc<K> acc;
  acc.zero();
  vote_range<DT, TOL, K, true, U>(t, tile.v0, tile.v1, acc, b.nt_stores != 0);
  if (tile.last) vote_tail<DT, TOL, K>(t, acc);
  const uint64_t tot = block_total<K>(acc, sh);
  uint64_t *tacc = b.acc + (uint64_t)tile.task * kNumCounters;
  if (threadIdx.x < (uint32_t)NC && tot != 0)
    __hip_atomic_fetch_add(&tacc[threadIdx.x], tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

#define FTV_CASE(DT, TOL, K)                                   \
  case spec_code(DT, TOL, K):                                  \
    run_tile<DT, TOL, K>(t, tile, b, sh);                      \
    break;
#define FTV_CASES_K(DT, TOL) \
  FTV_CASE(DT, TOL, 2)       \
  FTV_CASE(DT, TOL, 3)       \
  FTV_CASE(DT, TOL, 4)       \
  FTV_CASE(DT, TOL, 5)       \
  FTV_CASE(DT, TOL, 6)       \
  FTV_CASE(DT, TOL, 7)

__global__ __launch_bounds__(512) void k_vote_batch(BatchLaunch b) {
  __shared__ uint64_t sh[16 * kNumCounters];
  __shared__ uint32_t s_tile;
  __shared__ TileD s_tl;
  const uint64_t ntiles = b.ntiles_dev[0];
  const uint64_t ntasks = b.ntiles_dev[1];
  uint64_t hint = 0;  // thread 0: task of the previous tile (tile numbers only grow)
  bool first = true;  // a workgroup's first tile is its own index; the queue hands out the rest
  // when the grid covers every tile, each tile is some workgroup's first and
  // the queue has nothing to hand out: no atomic round trip before exiting
  const bool queue = gridDim.x < ntiles;
  for (;;) {
    if (threadIdx.x == 0) {
      const uint32_t q = first ? blockIdx.x
                         : !queue ? (uint32_t)ntiles
                                  : gridDim.x + __hip_atomic_fetch_add(b.queue_head, 1u, __ATOMIC_RELAXED,
                                                                       __HIP_MEMORY_SCOPE_AGENT);
      first = false;
      s_tile = q;
      if (q < ntiles) {
        if (b.prefix) {
          // the task whose tile range holds q: the last t with prefix[t] <= q.
          // It is at or after `hint`; gallop from there (usually one probe:
          // the same or the next task), then bisect, keeping
          // prefix[lo] <= q < prefix[hi] (prefix[ntasks] = ntiles > q).
          uint64_t lo = hint, hi = hint + 1, step = 1;
          while (hi < ntasks && b.prefix[hi] <= q) {
            lo = hi;
            step <<= 1;
            hi = lo + step;
          }
          if (hi > ntasks) hi = ntasks;
          while (hi - lo > 1) {
            const uint64_t mid = (lo + hi) >> 1;
            if (b.prefix[mid] <= q) lo = mid;
            else hi = mid;
          }
          hint = lo;
          const uint64_t j = q - b.prefix[lo];
          const uint64_t nvec = b.tasks[lo].nvec;
          TileD tl;
          tl.task = (uint32_t)lo;
          tl.v0 = j * b.tile_vecs < nvec ? j * b.tile_vecs : nvec;
          tl.v1 = tl.v0 + b.tile_vecs < nvec ? tl.v0 + b.tile_vecs : nvec;
          tl.last = (q + 1 == b.prefix[lo + 1]) ? 1u : 0u;
          s_tl = tl;
        } else {
          s_tl = b.tiles[q];
        }
      }
    }
    __syncthreads();
    const uint32_t ti = s_tile;
    if (ti >= ntiles) break;
    const TileD tile = s_tl;
    const TaskD &t = b.tasks[tile.task];  // read in place: a copy would go to scratch
    switch (t.spec) {
      FTV_CASES_K(FTV_F32, FTV_TOL_EXACT)
      FTV_CASES_K(FTV_F32, FTV_TOL_ULP)
      FTV_CASES_K(FTV_F32, FTV_TOL_REL)
      FTV_CASES_K(FTV_F64, FTV_TOL_EXACT)
      FTV_CASES_K(FTV_F64, FTV_TOL_ULP)
      FTV_CASES_K(FTV_F64, FTV_TOL_REL)
      FTV_CASES_K(FTV_I32, FTV_TOL_EXACT)
      FTV_CASES_K(FTV_I64, FTV_TOL_EXACT)
      default:
        break;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_batch_zero(BatchLaunch b) {
  const uint64_t ntasks = b.ntiles_dev[1];
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = gid; i < ntasks * kNumCounters; i += stride) b.acc[i] = 0;
  if (gid == 0) *b.queue_head = 0;
}

// Stats of every task of the batch, one workgroup per task (grid-stride).
__global__ __launch_bounds__(64) void k_batch_finalize(BatchLaunch b) {
  __shared__ uint64_t s_tot[kNumCounters];
  const uint64_t ntasks = b.ntiles_dev[1];
  for (uint64_t i = blockIdx.x; i < ntasks; i += gridDim.x)
    finalize_task(b.tasks[i], b.acc + i * kNumCounters, false, s_tot);
}

// Serving iterations: bring the iteration's table from pinned host memory into
// device memory (the kernels after this one read it there), re-arm the tile
// queue, and for the slots whose requests join in this iteration install
// their task records and clear their accumulators -- both read straight from
// the host table (slots[0..nnew), newt[0..nnew)).  No separate copy precedes
// the kernel.
// The host rewrites the table between iterations: it is read with
// system-scope loads, coherent with the host's writes whatever the caches hold.
// Each such load is a round trip over the host link, so every thread issues
// all of its loads -- a table word, the slot of an accumulator word, the slot
// and the word of a task record -- before any store, and the grid gives each
// thread about one index: the kernel then lasts about one round trip.
// Several dependent round trips per thread measured 8.7 us per iteration.
__device__ __forceinline__ uint64_t ld_host64(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint32_t ld_host32(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ __launch_bounds__(256) void k_slots_init(uint32_t *queue_head, uint64_t *acc, const uint64_t *table_h,
                                                    uint64_t *table_d, uint64_t table_words, const uint32_t *slots,
                                                    const TaskD *newt, uint64_t nnew, TaskD *tasks) {
  static_assert(sizeof(TaskD) % 8 == 0, "task records are copied in 8-byte words");
  constexpr uint64_t W = sizeof(TaskD) / 8;
  const uint64_t nacc = nnew * kNumCounters, ntw = nnew * W;
  const uint64_t nmax = table_words > nacc ? (table_words > ntw ? table_words : ntw) : (nacc > ntw ? nacc : ntw);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t *newt_w = reinterpret_cast<const uint64_t *>(newt);
  uint64_t *tasks_w = reinterpret_cast<uint64_t *>(tasks);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nmax; i += stride) {
    const bool has_t = i < table_words, has_a = i < nacc, has_n = i < ntw;
    uint64_t tw = 0, nw = 0;
    uint32_t aslot = 0, nslot = 0;
    if (has_t) tw = ld_host64(table_h + i);
    if (has_a) aslot = ld_host32(slots + i / kNumCounters);
    if (has_n) {
      nslot = ld_host32(slots + i / W);
      nw = ld_host64(newt_w + i);
    }
    if (has_t) table_d[i] = tw;
    if (has_a) acc[(uint64_t)aslot * kNumCounters + i % kNumCounters] = 0;
    if (has_n) tasks_w[(uint64_t)nslot * W + i % W] = nw;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *queue_head = 0;
}

// Serving iterations: stats of the slots whose requests finish in this one.
__global__ __launch_bounds__(64) void k_slots_finalize(const TaskD *tasks, const uint64_t *acc,
                                                       const uint32_t *fin, uint32_t nfin) {
  __shared__ uint64_t s_tot[kNumCounters];
  for (uint32_t i = blockIdx.x; i < nfin; i += gridDim.x) {
    const uint32_t slot = fin[i];
    finalize_task(tasks[slot], const_cast<uint64_t *>(acc) + (uint64_t)slot * kNumCounters, false,
                  s_tot);
  }
}

// Stats record of one task assembled from several vote launches.
__global__ __launch_bounds__(64) void k_task_finalize(TaskD t, VoteWs ws) {
  __shared__ uint64_t s_tot[kNumCounters];
  finalize_task(t, ws.acc, true, s_tot);
}

}  // namespace

hipError_t launch_vote_task(const TaskD &t, const VoteWs &ws, int num_cus, hipStream_t s, bool finalize) {
  switch ((int)(t.spec / 24)) {
    case FTV_F32: return launch_vote_task_f32(t, ws, num_cus, s, finalize);
    case FTV_F64: return launch_vote_task_f64(t, ws, num_cus, s, finalize);
    case FTV_I32: return launch_vote_task_i32(t, ws, num_cus, s, finalize);
    case FTV_I64: return launch_vote_task_i64(t, ws, num_cus, s, finalize);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_vote_finalize(const TaskD &t, const VoteWs &ws, hipStream_t s) {
  hipLaunchKernelGGL(k_task_finalize, dim3(1), dim3(64), 0, s, t, ws);
  return hipGetLastError();
}

hipError_t launch_batch_zero(const BatchLaunch &b, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_zero, dim3(64), dim3(256), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_slots_init(uint32_t *queue_head, uint64_t *acc, const void *table_h, void *table_d,
                             uint64_t table_bytes, const uint32_t *slots_h, const TaskD *newt_h, uint64_t nnew,
                             TaskD *tasks, hipStream_t s) {
  const uint64_t words = (table_bytes + 7) / 8;
  const uint64_t most = std::max<uint64_t>({words, nnew * kNumCounters, nnew * (sizeof(TaskD) / 8)});
  uint64_t grid = (most + 255) / 256;   // one index per thread
  grid = grid < 1 ? 1 : (grid > 1024 ? 1024 : grid);
  hipLaunchKernelGGL(k_slots_init, dim3((uint32_t)grid), dim3(256), 0, s, queue_head, acc,
                     static_cast<const uint64_t *>(table_h), static_cast<uint64_t *>(table_d), words, slots_h,
                     newt_h, nnew, tasks);
  return hipGetLastError();
}

hipError_t launch_slots_finalize(const TaskD *tasks, const uint64_t *acc, const uint32_t *fin,
                                 uint32_t nfin, hipStream_t s) {
  if (nfin == 0) return hipSuccess;
  const uint32_t grid = nfin < 1024 ? nfin : 1024;
  hipLaunchKernelGGL(k_slots_finalize, dim3(grid), dim3(64), 0, s, tasks, acc, fin, nfin);
  return hipGetLastError();
}

hipError_t launch_batch_vote(const BatchLaunch &b, hipStream_t s) {
  hipLaunchKernelGGL(k_vote_batch, dim3(b.grid), dim3(b.block), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_batch_finalize(const BatchLaunch &b, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_finalize, dim3(1024), dim3(64), 0, s, b);
  return hipGetLastError();
}

}  // namespace ftv
