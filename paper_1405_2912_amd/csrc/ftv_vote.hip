// ftv_vote.hip -- per-task and batched (persistent) vote kernels for gfx950.
//
// Per-task launch: a grid-stride loop over tiles of 16-byte vectors; each
// workgroup reduces its wave accumulators and adds the non-zero totals to the
// launch's device accumulators (most workgroups see no disagreement and add
// nothing).  A one-workgroup finalize kernel on the same stream then decides
// the verdict, writes the stats record and clears the accumulators: the
// kernel boundary orders the counts before the verdict, so the vote kernel
// needs neither a completion ticket nor device-scope fences.
//
// Batched launch: one persistent grid pulls tiles from an atomic queue over a
// table of (task, vector range) entries; a tile may belong to any task, so the
// body dispatches on the task's (value type, tolerance, k) code, a
// workgroup-uniform branch.  Per tile the workgroup adds its non-zero counts
// to the task's accumulators; a finalize kernel writes every task's stats.
#include "ftv_internal.hpp"
#include "ftv_vote_dev.hpp"

namespace ftv {
namespace {

using namespace dev;

constexpr int kVoteWgPerCu = 2;

template <int K>
struct Unroll {
  static constexpr int value = K <= 3 ? 2 : 1;
};

template <int DT, int TOL, int K, bool VEC>
__global__ __launch_bounds__(256) void k_vote_task(TaskD t, VoteWs ws) {
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

__global__ __launch_bounds__(64) void k_vote_finalize(TaskD t, VoteWs ws) {
  __shared__ uint64_t s_tot[kNumCounters];
  finalize_task(t, ws.acc, true, s_tot);
}

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
  for (;;) {
    if (threadIdx.x == 0) {
      const uint32_t q = __hip_atomic_fetch_add(b.queue_head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_tile = q;
      if (q < ntiles) {
        if (b.prefix) {
          // the task whose tile range holds q: last t with prefix[t] <= q
          uint64_t lo = 0, hi = ntasks;
          while (hi - lo > 1) {
            const uint64_t mid = (lo + hi) >> 1;
            if (b.prefix[mid] <= q) lo = mid;
            else hi = mid;
          }
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

// Serving iterations: re-arm the tile queue and clear the accumulators of the
// slots whose requests join in this iteration (slots[0..hdr[2]) ).
__global__ __launch_bounds__(256) void k_slots_init(uint32_t *queue_head, uint64_t *acc,
                                                    const uint32_t *slots, const uint64_t *hdr) {
  const uint64_t nnew = hdr[2];
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = gid; i < nnew * kNumCounters; i += stride)
    acc[(uint64_t)slots[i / kNumCounters] * kNumCounters + i % kNumCounters] = 0;
  if (gid == 0) *queue_head = 0;
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

// ---- per-task dispatch -----------------------------------------------------
// Workgroups of this instance that fit on one CU at once.  The grid-stride
// loop is only balanced when every workgroup of the grid is resident: a grid
// larger than the machine leaves a second, mostly empty wave of workgroups.
template <int DT, int TOL, int K, bool VEC>
int resident_per_cu() {
  static const int nb = [] {
    int v = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_vote_task<DT, TOL, K, VEC>, 256, 0) !=
            hipSuccess ||
        v < 1) {
      (void)hipGetLastError();
      v = 4;
    }
    return v;
  }();
  return nb;
}

template <int DT, int TOL, int K, bool VEC>
hipError_t launch_one(const TaskD &t, const VoteWs &ws, int num_cus, hipStream_t s) {
  constexpr int U = Unroll<K>::value;
  const uint64_t tile = 256ull * U;
  uint64_t tiles = (t.nvec + tile - 1) / tile;
  // two workgroups per CU stream the replicas at the highest rate measured on
  // MI355X (more concurrent streams lose DRAM page locality); never more than
  // fit at once
  const int per_cu = resident_per_cu<DT, TOL, K, VEC>() < kVoteWgPerCu ? resident_per_cu<DT, TOL, K, VEC>()
                                                                       : kVoteWgPerCu;
  uint64_t cap = (uint64_t)num_cus * per_cu;
  if (cap > (uint64_t)kMaxGrid) cap = kMaxGrid;
  const uint32_t grid = (uint32_t)(tiles < 1 ? 1 : (tiles < cap ? tiles : cap));
  hipLaunchKernelGGL((k_vote_task<DT, TOL, K, VEC>), dim3(grid), dim3(256), 0, s, t, ws);
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

hipError_t launch_vote_task(const TaskD &t, const VoteWs &ws, int num_cus, hipStream_t s) {
  const int dtype = (int)(t.spec / 24), tol = (int)((t.spec / 8) % 3);
  switch (dtype) {
    case FTV_F32:
      if (tol == FTV_TOL_EXACT) return launch_vec<FTV_F32, FTV_TOL_EXACT>(t, ws, num_cus, s);
      if (tol == FTV_TOL_ULP) return launch_vec<FTV_F32, FTV_TOL_ULP>(t, ws, num_cus, s);
      return launch_vec<FTV_F32, FTV_TOL_REL>(t, ws, num_cus, s);
    case FTV_F64:
      if (tol == FTV_TOL_EXACT) return launch_vec<FTV_F64, FTV_TOL_EXACT>(t, ws, num_cus, s);
      if (tol == FTV_TOL_ULP) return launch_vec<FTV_F64, FTV_TOL_ULP>(t, ws, num_cus, s);
      return launch_vec<FTV_F64, FTV_TOL_REL>(t, ws, num_cus, s);
    case FTV_I32: return launch_vec<FTV_I32, FTV_TOL_EXACT>(t, ws, num_cus, s);
    case FTV_I64: return launch_vec<FTV_I64, FTV_TOL_EXACT>(t, ws, num_cus, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_batch_zero(const BatchLaunch &b, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_zero, dim3(64), dim3(256), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_slots_init(uint32_t *queue_head, uint64_t *acc, const uint32_t *slots,
                             const uint64_t *hdr, hipStream_t s) {
  hipLaunchKernelGGL(k_slots_init, dim3(32), dim3(256), 0, s, queue_head, acc, slots, hdr);
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
