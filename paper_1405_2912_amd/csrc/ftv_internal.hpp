// ftv_internal.hpp -- host/device shared declarations of the gfx950 voter.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ftv.h"

namespace ftv {

// Tolerance as the kernels see it.  max_ulp is clamped to the key range of the
// value type on the host so the device compares in the type's own width.
struct TolD {
  uint64_t max_ulp;
  double delta;
  double abs_floor;
};

// Specialisation code of a task: value type, tolerance kind and replica count.
// spec = (dtype * 3 + tolkind) * 8 + k.  Integer types only use EXACT.
__host__ __device__ constexpr uint32_t spec_code(int dtype, int tolkind, int k) {
  return (uint32_t)((dtype * 3 + tolkind) * 8 + k);
}

// A task as the device sees it (per-task launch and batched launch).
struct TaskD {
  const void *rep[FTV_MAX_K];
  void *cons;
  uint8_t *mask;
  ftv_stats *stats;
  uint64_t n;      // elements
  uint64_t nvec;   // 16-byte vectors (vector path) or elements (scalar path)
  TolD tol;
  uint32_t k;
  uint32_t spec;
  uint32_t ntiles; // batched launch: tiles of this task (host bookkeeping)
  uint32_t vec;    // 1 = 16-byte vector path, 0 = scalar path
};

// One tile of the batched launch: vectors [v0, v1) of task `task`.
struct TileD {
  uint32_t task;
  uint32_t last;   // 1 if this tile also owns the scalar tail of the task
  uint64_t v0;
  uint64_t v1;
};

constexpr int kMaxGrid = 8192;     // per-task launch: workgroups (partials rows)
constexpr int kNumCounters = 32;   // >= 21 pairs + 7 disagree + 1 no-majority

// Device accumulators of the per-task launch, left zeroed by the launch's
// finalize kernel.
struct VoteWs {
  uint64_t *acc;     // [kNumCounters]
};

int elem_size(int dtype);

// ---- launchers (ftv_vote_*.hip) -----------------------------------------
// The vote kernel followed by a one-workgroup finalize kernel on the same
// stream (stats record from the accumulators, accumulators cleared).  With
// finalize = false only the vote kernel: its counts stay in the accumulators,
// to be added to by further launches (pieces of one task) and finalized by
// launch_vote_finalize.
hipError_t launch_vote_task(const TaskD &t, const VoteWs &ws, int num_cus, hipStream_t s, bool finalize = true);
// The same per value type (one translation unit each).
hipError_t launch_vote_task_f32(const TaskD &t, const VoteWs &ws, int num_cus, hipStream_t s, bool finalize);
hipError_t launch_vote_task_f64(const TaskD &t, const VoteWs &ws, int num_cus, hipStream_t s, bool finalize);
hipError_t launch_vote_task_i32(const TaskD &t, const VoteWs &ws, int num_cus, hipStream_t s, bool finalize);
hipError_t launch_vote_task_i64(const TaskD &t, const VoteWs &ws, int num_cus, hipStream_t s, bool finalize);
// Stats record of task t (t.n, t.k, t.stats) from the accumulators, which it
// clears (ftv_vote_batch.hip).
hipError_t launch_vote_finalize(const TaskD &t, const VoteWs &ws, hipStream_t s);

// A persistent launch over a queue of tiles.  Two ways to name the tiles:
//  * prefix mode (batched calls): prefix[t] = first tile of task t (ntasks+1
//    entries); tile j of task t covers vectors [j*tile_vecs, (j+1)*tile_vecs);
//  * table mode (server iterations, prefix == nullptr): explicit TileD entries.
struct BatchLaunch {
  const TaskD *tasks;          // device
  const TileD *tiles;          // device, table mode
  const uint64_t *prefix;      // device, prefix mode
  const uint64_t *ntiles_dev;  // device: [0] = tiles, [1] = tasks
  uint64_t *acc;               // device [ntasks][kNumCounters]
  uint32_t *queue_head;        // device
  uint32_t block;
  uint32_t grid;
  uint32_t nt_stores;
  uint32_t tile_vecs;          // prefix mode
};
// A batched call is three kernels: zero (queue head, accumulators of
// ntiles_dev[1] tasks), the persistent vote, finalize (every task's stats).
hipError_t launch_batch_zero(const BatchLaunch &b, hipStream_t s);
hipError_t launch_batch_vote(const BatchLaunch &b, hipStream_t s);
hipError_t launch_batch_finalize(const BatchLaunch &b, hipStream_t s);
// Serving: copy the iteration table (table_bytes, 16-byte multiple) from pinned
// host memory (a device-visible address) to table_d, zero queue_head, and for
// slots_h[0..nnew) copy newt_h[i] to tasks[slots_h[i]] and zero their
// accumulators (slots_h and newt_h: device-visible addresses in the host table).
hipError_t launch_slots_init(uint32_t *queue_head, uint64_t *acc, const void *table_h, void *table_d,
                             uint64_t table_bytes, const uint32_t *slots_h, const TaskD *newt_h, uint64_t nnew,
                             TaskD *tasks, hipStream_t s);
// Serving: stats records of the nfin slots listed in fin (host count).
hipError_t launch_slots_finalize(const TaskD *tasks, const uint64_t *acc, const uint32_t *fin,
                                 uint32_t nfin, hipStream_t s);

// ---- fingerprints and block vote (ftv_blocks.hip) ----------------------
hipError_t launch_fingerprint(const void *buf, uint64_t nbytes, uint64_t block_bytes,
                              uint64_t *fp_out, hipStream_t s);
// The fingerprints of m <= FTV_MAX_K buffers of nbytes each in one launch;
// buffer j's go to fp_out[j * nblocks ...].
hipError_t launch_fingerprints(const void *const *bufs, uint32_t m, uint64_t nbytes, uint64_t block_bytes,
                               uint64_t *fp_out, hipStream_t s);

struct BlockVoteD {
  const void *rep[FTV_MAX_K];
  uint32_t k;
  int32_t dtype;
  int32_t tolkind;
  uint32_t pad;
  TolD tol;
  uint64_t nbytes;
  uint64_t block_bytes;
  uint64_t nblocks;
  uint64_t *fps;          // may be null
  uint8_t *blockmap;
  void *cons;
  uint8_t *mask;          // may be null
  ftv_block_stats *bstats;
  uint64_t *acc;          // device workspace [16], left zeroed by the finalize kernel
};
hipError_t launch_vote_blocks(const BlockVoteD &b, int num_cus, hipStream_t s);
// Pass 1 of the block vote: whole-block fingerprints of every replica (replica
// 0 also streamed into the consensus, its mask bytes zeroed) and the vote of
// the partial last block.
hipError_t launch_blocks_hash(const BlockVoteD &b, hipStream_t s);

// ---- sibling manager helpers (ftv_copy.hip) ------------------------------
// Device-to-device copy of `bytes` (both pointers 16-byte aligned).
hipError_t launch_copy(void *dst, const void *src, uint64_t bytes, int num_cus, hipStream_t s);
// Vote of m fingerprints per block (fps: m rows of nblocks): res[j] = 1 for a
// sibling that differs from a strict majority in some block (u32 x m), then
// the count of blocks without a strict majority (u64 at word (m+1)/2*2).
hipError_t launch_fp_vote(const uint64_t *fps, uint32_t m, uint64_t nblocks, uint32_t *res, int num_cus,
                          hipStream_t s);

}  // namespace ftv
