// ftv_vote_noalloc.hip -- ftv_vote_batch_noalloc: the batched vote of
// ftv_vote_batch for callers that cannot allocate (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).
//
// There is no context.  The device workspace of a batched launch -- table
// header and tile queue, the per-task tile prefix, the task records and the
// per-task count accumulators -- lives in `scratch`, a static device array of
// this file that every GPU the library runs on holds until the process ends.
// Its device address is looked up once per device (hipGetSymbolAddress with
// that device current) and only that address is handed to kernels and copies:
// in host code the array's name is a host-side stand-in, not a device address.
// The host side of a call builds the table in static host arrays (one mutex
// serialises that and the upload), so a call allocates neither device nor host
// memory.  The kernels are those of ftv_vote_batch with its default schedule;
// the zero kernel clears the queue and the accumulators, so every call starts
// from a clean workspace whatever the previous call left.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "ftv_common.hpp"

namespace ftv {
namespace {

constexpr uint64_t kNaMaxTasks = FTV_NOALLOC_MAX_TASKS;
constexpr size_t round256(size_t x) { return (x + 255) / 256 * 256; }
// [header 256 B: tiles, tasks, ..., queue head at byte 128][prefix u64 x (T+1)]
// [TaskD x T][accumulators u64 x kNumCounters x T]
constexpr size_t kHdrBytes = 256;
constexpr size_t kQueueOff = 128;
constexpr size_t kPrefixOff = kHdrBytes;
constexpr size_t kTasksOff = round256(kPrefixOff + 8 * (kNaMaxTasks + 1));
constexpr size_t kAccOff = round256(kTasksOff + sizeof(TaskD) * kNaMaxTasks);
constexpr size_t kScratchBytes = kAccOff + 8 * kNumCounters * kNaMaxTasks;
static_assert(kScratchBytes <= FTV_NOALLOC_SCRATCH_BYTES, "scratch layout exceeds the declared size");

// the schedule of ftv_vote_batch's default: 2 MiB tiles of 16-byte vectors,
// 512 threads, 4 workgroups per CU, largest task first, streaming stores
constexpr uint32_t kNaTileVecs = 131072;
constexpr uint32_t kNaBlock = 512;
constexpr uint32_t kNaGridMult = 4;

constexpr int kNaMaxDevices = 64;

}  // namespace
}  // namespace ftv

static __device__ __align__(256) unsigned char scratch[FTV_NOALLOC_SCRATCH_BYTES];

namespace ftv {
namespace {

std::mutex g_na_mu;
// per device: the address of `scratch` on that device, and its CU count
char *g_na_ptr[kNaMaxDevices];
int g_na_cus[kNaMaxDevices];
// host staging of a call's table (guarded by g_na_mu)
uint64_t g_na_head[(kHdrBytes + 8 * (kNaMaxTasks + 1)) / 8];
TaskD g_na_tasks[kNaMaxTasks];
TaskD g_na_sorted[kNaMaxTasks];
uint32_t g_na_ord[kNaMaxTasks];

// Device address of `scratch` on the current device (set-up on first use,
// with that device current).  Called with g_na_mu held.
int na_scratch(char **ptr, int *cus) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNaMaxDevices) return fail(FTV_E_INVALID, "device index beyond 63");
  if (!g_na_ptr[dev]) {
    void *p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    int n = 0;
    HIPCHK(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
    g_na_cus[dev] = n > 0 ? n : 256;
    g_na_ptr[dev] = static_cast<char *>(p);
  }
  *ptr = g_na_ptr[dev];
  *cus = g_na_cus[dev];
  return FTV_OK;
}

}  // namespace
}  // namespace ftv

using namespace ftv;

extern "C" int ftv_vote_batch_noalloc(const ftv_vote_desc *descs, uint64_t ntasks, void *stream) {
  if (ntasks && !descs) return fail(FTV_E_INVALID, "NULL descriptor array");
  if (ntasks > kNaMaxTasks)
    return fail(FTV_E_INVALID, "ftv_vote_batch_noalloc takes at most " + std::to_string(kNaMaxTasks) +
                                   " tasks per call (its static workspace holds no more)");
  if (ntasks == 0) return FTV_OK;
  std::lock_guard<std::mutex> lk(g_na_mu);
  uint64_t tiles = 0;
  for (uint64_t i = 0; i < ntasks; ++i) {
    TaskD &t = g_na_tasks[i];
    int rc = make_task(&descs[i], true, &t);
    if (rc) return fail(rc, "task " + std::to_string(i) + ": " + g_err);
    const uint64_t nt = std::max<uint64_t>(1, (t.nvec + kNaTileVecs - 1) / kNaTileVecs);
    if (nt > 0xffffffffull) return fail(FTV_E_INVALID, "task too large for one batch");
    t.ntiles = (uint32_t)nt;
    tiles += nt;
    g_na_ord[i] = (uint32_t)i;
  }
  if (tiles > 0xffffffffull) return fail(FTV_E_INVALID, "batch has too many tiles");
  char *p = nullptr;
  int cus = 0;
  int rc = na_scratch(&p, &cus);
  if (rc) return rc;
  // largest task first, ties by position (std::sort works in place)
  auto bytes_of = [](const TaskD &t) { return t.n * t.k * (uint64_t)elem_size((int)(t.spec / 24)); };
  std::sort(g_na_ord, g_na_ord + ntasks, [&](uint32_t a, uint32_t b) {
    const uint64_t ba = bytes_of(g_na_tasks[a]), bb = bytes_of(g_na_tasks[b]);
    return ba != bb ? ba > bb : a < b;
  });
  memset(g_na_head, 0, kHdrBytes);
  uint64_t *pre = g_na_head + kPrefixOff / 8;
  uint64_t acc_tiles = 0;
  for (uint64_t i = 0; i < ntasks; ++i) {
    g_na_sorted[i] = g_na_tasks[g_na_ord[i]];
    pre[i] = acc_tiles;
    acc_tiles += g_na_sorted[i].ntiles;
  }
  pre[ntasks] = acc_tiles;
  g_na_head[0] = acc_tiles;
  g_na_head[1] = ntasks;
  hipStream_t s = (hipStream_t)stream;
  // from pageable host memory: each copy has consumed its source when it
  // returns, so the next call may rewrite the staging
  HIPCHK(hipMemcpyAsync(p, g_na_head, kPrefixOff + 8 * (ntasks + 1), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(p + kTasksOff, g_na_sorted, sizeof(TaskD) * ntasks, hipMemcpyHostToDevice, s));
  BatchLaunch b;
  b.tasks = reinterpret_cast<const TaskD *>(p + kTasksOff);
  b.tiles = nullptr;
  b.prefix = reinterpret_cast<const uint64_t *>(p + kPrefixOff);
  b.ntiles_dev = reinterpret_cast<const uint64_t *>(p);
  b.acc = reinterpret_cast<uint64_t *>(p + kAccOff);
  b.queue_head = reinterpret_cast<uint32_t *>(p + kQueueOff);
  b.block = kNaBlock;
  b.grid = (uint32_t)std::min<uint64_t>((uint64_t)kNaGridMult * (uint64_t)cus, acc_tiles);
  b.nt_stores = 1;
  b.tile_vecs = kNaTileVecs;
  hipError_t e = launch_batch_zero(b, s);
  if (e != hipSuccess) return hip_fail(e, "zero kernel launch");
  e = launch_batch_vote(b, s);
  if (e != hipSuccess) return hip_fail(e, "batch kernel launch");
  e = launch_batch_finalize(b, s);
  if (e != hipSuccess) return hip_fail(e, "finalize kernel launch");
  return FTV_OK;
}
