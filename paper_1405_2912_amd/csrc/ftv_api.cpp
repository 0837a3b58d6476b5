// ftv_api.cpp -- C ABI entry points: context, validation, per-task vote,
// batched vote (table build, HIP graph replay) and its autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <ctime>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "ftv.h"
#include "ftv_common.hpp"
#include "ftv_internal.hpp"

namespace ftv {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  (void)hipGetLastError();  // clear the sticky launch error, if any
  return FTV_E_HIP;
}

int elem_size(int dtype) { return (dtype == FTV_F32 || dtype == FTV_I32) ? 4 : 8; }

static bool aligned(const void *p, uintptr_t a) { return ((uintptr_t)p % a) == 0; }

int check_tol(int dtype, const ftv_tol &t) {
  if (dtype < FTV_F32 || dtype > FTV_I64) return fail(FTV_E_DTYPE, "unknown dtype");
  if (t.reserved != 0) return fail(FTV_E_INVALID, "tol.reserved must be 0");
  if (t.kind < FTV_TOL_EXACT || t.kind > FTV_TOL_REL) return fail(FTV_E_INVALID, "unknown tolerance kind");
  const bool fl = dtype == FTV_F32 || dtype == FTV_F64;
  if (!fl && t.kind != FTV_TOL_EXACT)
    return fail(FTV_E_DTYPE, "integer types are compared bit-wise (FTV_TOL_EXACT only)");
  if (t.kind == FTV_TOL_REL && (!(t.delta >= 0.0) || !(t.abs_floor >= 0.0)))
    return fail(FTV_E_INVALID, "REL tolerance needs delta >= 0 and abs_floor >= 0");
  return FTV_OK;
}

TolD to_tol_d(int dtype, const ftv_tol &t) {
  TolD d;
  d.max_ulp = t.max_ulp;
  if (elem_size(dtype) == 4 && d.max_ulp > 0xffffffffull) d.max_ulp = 0xffffffffull;
  d.delta = t.delta;
  d.abs_floor = t.abs_floor;
  return d;
}

bool spans_meet(const Span &a, const Span &b) {
  if (!a.p || !b.p || !a.len || !b.len) return false;
  const uintptr_t x = reinterpret_cast<uintptr_t>(a.p), y = reinterpret_cast<uintptr_t>(b.p);
  return x < y + b.len && y < x + a.len;
}

// The outputs of one launch share no byte with its inputs or with each other:
// the kernels read replica elements again after some outputs of the same
// launch are stored (the fix-up pass of the general vote, the block restore),
// and outputs written by different lanes would race.  Input ranges may
// overlap (read only).
int check_disjoint(const Span *outs, int nouts, const Span *ins, int nins) {
  for (int o = 0; o < nouts; ++o) {
    for (int r = 0; r < nins; ++r)
      if (spans_meet(outs[o], ins[r])) return fail(FTV_E_INVALID, "an output overlaps a replica");
    for (int q = o + 1; q < nouts; ++q)
      if (spans_meet(outs[o], outs[q])) return fail(FTV_E_INVALID, "two outputs overlap");
  }
  return FTV_OK;
}

int check_vote_overlaps(const ftv_vote_desc *d) {
  if (d->n > (UINT64_MAX >> 4)) return fail(FTV_E_INVALID, "n too large");
  const uint64_t nb = d->n * (uint64_t)elem_size(d->dtype);
  const Span outs[3] = {{d->consensus, nb}, {d->mask, d->n}, {d->stats, sizeof(ftv_stats)}};
  Span ins[FTV_MAX_K];
  for (uint32_t r = 0; r < d->k; ++r) ins[r] = {d->replicas[r], nb};
  return check_disjoint(outs, 3, ins, (int)d->k);
}

// Validate a vote descriptor and fill the device task record.  strict = batch
// alignment rules (16-byte replicas/consensus, 4-byte mask).
int make_task(const ftv_vote_desc *d, bool strict, TaskD *out) {
  if (!d) return fail(FTV_E_INVALID, "NULL descriptor");
  if (d->k < 2 || d->k > FTV_MAX_K) return fail(FTV_E_K, "k must be in [2, 7]");
  int rc = check_tol(d->dtype, d->tol);
  if (rc) return rc;
  if (!d->stats) return fail(FTV_E_INVALID, "stats pointer is NULL");
  if (!aligned(d->stats, 8)) return fail(FTV_E_ALIGN, "stats must be 8-byte aligned");
  const int es = elem_size(d->dtype);
  bool vec = true;
  for (uint32_t r = 0; r < d->k; ++r) {
    if (!d->replicas[r] && d->n) return fail(FTV_E_INVALID, "replica pointer is NULL");
    if (!aligned(d->replicas[r], es)) return fail(FTV_E_ALIGN, "replica not element-aligned");
    vec = vec && aligned(d->replicas[r], 16);
  }
  if (d->consensus) {
    if (!aligned(d->consensus, es)) return fail(FTV_E_ALIGN, "consensus not element-aligned");
    vec = vec && aligned(d->consensus, 16);
  }
  if (d->mask) vec = vec && aligned(d->mask, 4);
  if (strict && !vec)
    return fail(FTV_E_ALIGN, "batched tasks need 16-byte aligned replicas/consensus, 4-byte mask");
  rc = check_vote_overlaps(d);
  if (rc) return rc;
  memset(out, 0, sizeof(*out));
  for (uint32_t r = 0; r < d->k; ++r) out->rep[r] = d->replicas[r];
  out->cons = d->consensus;
  out->mask = d->mask;
  out->stats = d->stats;
  out->n = d->n;
  out->vec = vec ? 1u : 0u;
  out->nvec = vec ? d->n / (uint64_t)(16 / es) : d->n;
  out->tol = to_tol_d(d->dtype, d->tol);
  out->k = d->k;
  out->spec = spec_code(d->dtype, d->tol.kind, (int)d->k);
  out->ntiles = 1;
  return FTV_OK;
}

}  // namespace ftv

using namespace ftv;

// ---------------------------------------------------------------------------
// Count accumulators are kept per stream: calls on one stream are ordered by
// it and share a slot; calls on different streams get different slots, so two
// streams voting with one context can never mix their counts.  A slot holds
// the per-task vote counters and the block-vote counters; the kernels leave
// both zeroed.
constexpr int kStreamSlots = 64;
constexpr int kBlkWords = 16;
constexpr int kSlotWords = kNumCounters + kBlkWords;
// launches whose kernel time a context records at most between two reads
constexpr uint32_t kMaxTimed = 1024;

struct ftv_ctx {
  int device = 0;
  int num_cus = 256;
  std::string name;
  // count accumulators, kStreamSlots x kSlotWords (zero between launches),
  // and the stream each slot belongs to
  uint64_t *slots = nullptr;
  hipStream_t slot_stream[kStreamSlots] = {};
  int nslots = 0;
  // batched launch
  ftv_batch_cfg cfg{};
  uint64_t cap_tasks = 0;
  char *d_tab = nullptr;   // [hdr 256 B][prefix u64 x (cap_tasks+1)][TaskD x cap_tasks]
  char *h_tab = nullptr;   // pinned staging of the same layout
  uint64_t *d_acc = nullptr;
  uint32_t *d_queue = nullptr;
  hipEvent_t staged{};
  bool staged_pending = false;
  hipStream_t cap_stream{};
  // the last batched launch: later batches on another stream wait for it, and
  // the tables are only freed once it has finished
  hipEvent_t batch_done{};
  hipStream_t batch_stream{};
  bool batch_pending = false;
  hipGraphExec_t gexec{};
  hipGraph_t graph{};
  bool gvalid = false;
  uint32_t g_grid = 0;
  ftv_batch_cfg g_cfg{};
  // ftv_run_redundant: replicas abandoned after a timeout, freed once their
  // work has finished (ftv_run.cpp)
  RunState *run = nullptr;
  // ftv_vote_mem: two device staging sets for host replicas, their copy
  // stream and the events that order copies and votes
  char *stage = nullptr;
  uint64_t stage_bytes = 0;
  hipStream_t copy_stream{};
  hipEvent_t mem_entry{}, mem_copied[2]{}, mem_consumed[2]{};
  bool mem_ready = false;
  // the last ftv_vote_mem call: a call on another stream waits for it before
  // it touches the staging sets
  hipEvent_t mem_done{};
  hipStream_t mem_stream{};
  bool mem_pending = false;
  // ftv_vote_blocks without caller fingerprints: the fingerprints of every
  // replica's blocks (pass 1 writes them, pass 2 votes them).  A call on
  // another stream than the last one waits for it; a grown buffer's
  // predecessor is freed with the context (the last call may still read it).
  uint64_t *blk_fps = nullptr;
  uint64_t blk_fps_cap = 0;  // words
  std::vector<void *> retired;
  hipEvent_t blk_done{};
  hipStream_t blk_stream{};
  bool blk_pending = false;
  // kernel timing (ftv_ctx_set_timing): a pair of events around the vote
  // kernel of each ftv_vote and the persistent kernel of each ftv_vote_batch
  bool timing = false;
  hipEvent_t tev[2 * kMaxTimed] = {};
  uint32_t ntev = 0;
};

namespace {

// the schedule the autotuner found fastest most often on MI355X for a mixed batch of
// thousands of uneven tasks: 2 MiB tiles, 512 threads, 4 workgroups per CU, largest
// task first, streaming stores
const ftv_batch_cfg kDefaultCfg = {131072u, 512u, 4u, 1u, 1u, 0u};

int cfg_check(const ftv_batch_cfg &c) {
  if (c.block != 256 && c.block != 512) return fail(FTV_E_INVALID, "block must be 256 or 512");
  if (c.tile_vecs < 256 || c.tile_vecs > (1u << 22)) return fail(FTV_E_INVALID, "tile_vecs out of range");
  if (c.grid_mult < 1 || c.grid_mult > 32) return fail(FTV_E_INVALID, "grid_mult out of range");
  if (c.order > 3 || c.nt_stores > 1 || c.reserved != 0) return fail(FTV_E_INVALID, "bad order/nt_stores");
  return FTV_OK;
}

size_t prefix_off() { return 256; }
size_t tasks_off(uint64_t cap) { return (256 + 8 * (cap + 1) + 255) / 256 * 256; }
size_t tab_bytes(uint64_t cap) { return tasks_off(cap) + sizeof(TaskD) * cap; }

void free_batch(ftv_ctx *c) {
  if (c->gvalid) {
    (void)hipGraphExecDestroy(c->gexec);
    (void)hipGraphDestroy(c->graph);
    c->gvalid = false;
  }
  if (c->d_tab) (void)hipFree(c->d_tab);
  if (c->h_tab) (void)hipHostFree(c->h_tab);
  if (c->d_acc) (void)hipFree(c->d_acc);
  c->d_tab = nullptr;
  c->h_tab = nullptr;
  c->d_acc = nullptr;
  c->cap_tasks = 0;
}

// The count slot of stream s (assigned on first use).
int stream_slot(ftv_ctx *c, hipStream_t s, uint64_t **acc) {
  for (int j = 0; j < c->nslots; ++j)
    if (c->slot_stream[j] == s) {
      *acc = c->slots + (uint64_t)j * kSlotWords;
      return FTV_OK;
    }
  if (c->nslots == kStreamSlots)
    return fail(FTV_E_BUSY, "a context keeps count accumulators for at most 64 streams");
  c->slot_stream[c->nslots] = s;
  *acc = c->slots + (uint64_t)c->nslots * kSlotWords;
  ++c->nslots;
  return FTV_OK;
}

int ensure_capacity(ftv_ctx *c, uint64_t tasks, hipStream_t s) {
  if (tasks <= c->cap_tasks) return FTV_OK;
  // the old buffers may still be read by the last batch, on whatever stream
  // it was launched (the caller's stream s is ordered after it already)
  (void)s;
  if (c->batch_pending) HIPCHK(hipEventSynchronize(c->batch_done));
  if (c->staged_pending) {
    HIPCHK(hipEventSynchronize(c->staged));
    c->staged_pending = false;
  }
  free_batch(c);
  const uint64_t nt = std::max<uint64_t>(tasks + tasks / 2, 1024);
  const size_t tb = tab_bytes(nt);
  if (hipMalloc(&c->d_tab, tb) != hipSuccess || hipHostMalloc(&c->h_tab, tb) != hipSuccess ||
      hipMalloc(&c->d_acc, sizeof(uint64_t) * kNumCounters * nt) != hipSuccess) {
    (void)hipGetLastError();
    free_batch(c);
    return fail(FTV_E_NOMEM, "cannot allocate the batch tables");
  }
  c->cap_tasks = nt;
  return FTV_OK;
}

BatchLaunch make_launch(ftv_ctx *c, uint32_t grid) {
  BatchLaunch b;
  b.tasks = reinterpret_cast<const TaskD *>(c->d_tab + tasks_off(c->cap_tasks));
  b.tiles = nullptr;
  b.prefix = reinterpret_cast<const uint64_t *>(c->d_tab + prefix_off());
  b.ntiles_dev = reinterpret_cast<const uint64_t *>(c->d_tab);
  b.acc = c->d_acc;
  b.queue_head = c->d_queue;
  b.block = c->cfg.block;
  b.grid = grid;
  b.nt_stores = c->cfg.nt_stores;
  b.tile_vecs = c->cfg.tile_vecs;
  return b;
}

// Capture zero + persistent + finalize kernels once per (capacity, grid, cfg); the
// kernels read the task and tile counts from the table header, so a new batch
// only needs a new table upload.
int ensure_graph(ftv_ctx *c, uint32_t grid) {
  if (c->gvalid && c->g_grid == grid && !memcmp(&c->g_cfg, &c->cfg, sizeof(c->cfg))) return FTV_OK;
  if (c->gvalid) {
    (void)hipGraphExecDestroy(c->gexec);
    (void)hipGraphDestroy(c->graph);
    c->gvalid = false;
  }
  const BatchLaunch b = make_launch(c, grid);
  HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t e1 = launch_batch_zero(b, c->cap_stream);
  hipError_t e2 = launch_batch_vote(b, c->cap_stream);
  hipError_t e2f = launch_batch_finalize(b, c->cap_stream);
  hipGraph_t g{};
  hipError_t e3 = hipStreamEndCapture(c->cap_stream, &g);
  if (e3 == hipSuccess && (e1 != hipSuccess || e2 != hipSuccess || e2f != hipSuccess)) (void)hipGraphDestroy(g);
  if (e1 != hipSuccess) return hip_fail(e1, "capture zero kernel");
  if (e2 != hipSuccess) return hip_fail(e2, "capture batch kernel");
  if (e2f != hipSuccess) return hip_fail(e2f, "capture finalize kernel");
  if (e3 != hipSuccess) return hip_fail(e3, "hipStreamEndCapture");
  hipError_t e4 = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
  if (e4 != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(e4, "hipGraphInstantiate");
  }
  c->graph = g;
  c->gvalid = true;
  c->g_grid = grid;
  c->g_cfg = c->cfg;
  return FTV_OK;
}

// Order the task records by the schedule and write them with the prefix sum
// of their tile counts into pinned staging, then upload (O(tasks) host work).
int build_tables(ftv_ctx *c, const ftv_vote_desc *descs, uint64_t ntasks, hipStream_t s,
                 uint64_t *ntiles_out) {
  std::vector<TaskD> tasks(ntasks);
  const uint64_t tv = c->cfg.tile_vecs;
  for (uint64_t i = 0; i < ntasks; ++i) {
    int rc = make_task(&descs[i], true, &tasks[i]);
    if (rc) return fail(rc, "task " + std::to_string(i) + ": " + g_err);
    const uint64_t nt = std::max<uint64_t>(1, (tasks[i].nvec + tv - 1) / tv);
    if (nt > 0xffffffffull) return fail(FTV_E_INVALID, "task too large for one batch");
    tasks[i].ntiles = (uint32_t)nt;
  }
  if (ntasks > 0xffffffffull) return fail(FTV_E_INVALID, "batch too large");
  int rc = ensure_capacity(c, ntasks, s);
  if (rc) return rc;
  if (c->staged_pending) {  // the previous upload must have left the staging
    HIPCHK(hipEventSynchronize(c->staged));
    c->staged_pending = false;
  }
  std::vector<uint32_t> ord(ntasks);
  for (uint64_t i = 0; i < ntasks; ++i) ord[i] = (uint32_t)i;
  auto bytes_of = [&](uint32_t i) { return tasks[i].n * tasks[i].k * (uint64_t)elem_size((int)(tasks[i].spec / 24)); };
  if (c->cfg.order == 1)
    std::stable_sort(ord.begin(), ord.end(), [&](uint32_t a, uint32_t b) { return bytes_of(a) > bytes_of(b); });
  else if (c->cfg.order == 2)
    std::stable_sort(ord.begin(), ord.end(), [&](uint32_t a, uint32_t b) { return bytes_of(a) < bytes_of(b); });
  else if (c->cfg.order == 3)
    std::stable_sort(ord.begin(), ord.end(), [&](uint32_t a, uint32_t b) {
      if (tasks[a].spec != tasks[b].spec) return tasks[a].spec < tasks[b].spec;
      return bytes_of(a) > bytes_of(b);
    });
  uint64_t *hdr = reinterpret_cast<uint64_t *>(c->h_tab);
  uint64_t *pre = reinterpret_cast<uint64_t *>(c->h_tab + prefix_off());
  TaskD *ht = reinterpret_cast<TaskD *>(c->h_tab + tasks_off(c->cap_tasks));
  uint64_t ntiles = 0;
  for (uint64_t i = 0; i < ntasks; ++i) {
    pre[i] = ntiles;
    ht[i] = tasks[ord[i]];
    ntiles += ht[i].ntiles;
  }
  pre[ntasks] = ntiles;
  if (ntiles > 0xffffffffull) return fail(FTV_E_INVALID, "batch has too many tiles");
  hdr[0] = ntiles;
  hdr[1] = ntasks;
  HIPCHK(hipMemcpyAsync(c->d_tab, c->h_tab, prefix_off() + 8 * (ntasks + 1), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(c->d_tab + tasks_off(c->cap_tasks), ht, sizeof(TaskD) * ntasks,
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipEventRecord(c->staged, s));
  c->staged_pending = true;
  *ntiles_out = ntiles;
  return FTV_OK;
}

int batch_run(ftv_ctx *c, const ftv_vote_desc *descs, uint64_t ntasks, hipStream_t s) {
  if (ntasks == 0) return FTV_OK;
  // the tables, queue head and accumulators are the context's: a batch on
  // another stream than the last one is ordered after it on the device
  if (c->batch_pending && c->batch_stream != s) HIPCHK(hipStreamWaitEvent(s, c->batch_done, 0));
  uint64_t ntiles = 0;
  int rc = build_tables(c, descs, ntasks, s, &ntiles);
  if (rc) return rc;
  uint64_t grid = (uint64_t)c->cfg.grid_mult * c->num_cus;
  grid = std::min<uint64_t>(grid, ntiles);
  // quantise the grid so that small batches share one captured graph
  uint32_t g = 1;
  while (g < grid) g <<= 1;
  g = (uint32_t)std::min<uint64_t>(g, (uint64_t)c->cfg.grid_mult * c->num_cus);
  if (c->timing && c->ntev < kMaxTimed) {
    // timed: the graph's three kernels launched directly, with events around
    // the persistent one (same launch parameters as the captured graph)
    const BatchLaunch b = make_launch(c, g);
    hipEvent_t *ev = c->tev + 2 * c->ntev;
    hipError_t e = launch_batch_zero(b, s);
    if (e != hipSuccess) return hip_fail(e, "zero kernel launch");
    HIPCHK(hipEventRecord(ev[0], s));
    e = launch_batch_vote(b, s);
    if (e != hipSuccess) return hip_fail(e, "batch kernel launch");
    HIPCHK(hipEventRecord(ev[1], s));
    e = launch_batch_finalize(b, s);
    if (e != hipSuccess) return hip_fail(e, "finalize kernel launch");
    ++c->ntev;
  } else {
    rc = ensure_graph(c, g);
    if (rc) return rc;
    HIPCHK(hipGraphLaunch(c->gexec, s));
  }
  HIPCHK(hipEventRecord(c->batch_done, s));
  c->batch_stream = s;
  c->batch_pending = true;
  return FTV_OK;
}

// ---- tune cache (flat JSON object: key -> [tile_vecs, block, grid_mult, order, nt]) ----
std::string tune_key(ftv_ctx *c, const ftv_vote_desc *d, uint64_t n) {
  uint64_t bytes = 0;
  for (uint64_t i = 0; i < n; ++i) bytes += d[i].n * d[i].k * elem_size(d[i].dtype);
  int lt = 0, lb = 0;
  while ((1ull << lt) < n) ++lt;
  while ((1ull << lb) < bytes) ++lb;
  std::ostringstream o;
  o << c->name << "|cu" << c->num_cus << "|t2^" << lt << "|b2^" << lb;
  return o.str();
}

bool cache_lookup(const std::string &path, const std::string &key, ftv_batch_cfg *out) {
  std::ifstream f(path);
  if (!f) return false;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string txt = ss.str();
  const std::string pat = "\"" + key + "\": [";
  size_t p = txt.find(pat);
  if (p == std::string::npos) return false;
  unsigned v[5];
  if (sscanf(txt.c_str() + p + pat.size(), "%u, %u, %u, %u, %u", &v[0], &v[1], &v[2], &v[3], &v[4]) != 5)
    return false;
  ftv_batch_cfg cfg = {v[0], v[1], v[2], v[3], v[4], 0};
  if (cfg_check(cfg) != FTV_OK) return false;
  *out = cfg;
  return true;
}

void cache_store(const std::string &path, const std::string &key, const ftv_batch_cfg &cfg) {
  std::vector<std::pair<std::string, std::string>> items;
  {
    std::ifstream f(path);
    std::string line;
    while (f && std::getline(f, line)) {
      size_t a = line.find('"'), b = line.find("\": [");
      if (a == std::string::npos || b == std::string::npos || b <= a) continue;
      std::string k = line.substr(a + 1, b - a - 1);
      size_t e = line.find(']', b);
      if (e == std::string::npos) continue;
      if (k != key) items.emplace_back(k, line.substr(b + 4, e - b - 4));
    }
  }
  std::ostringstream v;
  v << cfg.tile_vecs << ", " << cfg.block << ", " << cfg.grid_mult << ", " << cfg.order << ", " << cfg.nt_stores;
  items.emplace_back(key, v.str());
  std::ofstream f(path, std::ios::trunc);
  f << "{\n";
  for (size_t i = 0; i < items.size(); ++i)
    f << "  \"" << items[i].first << "\": [" << items[i].second << "]" << (i + 1 < items.size() ? "," : "") << "\n";
  f << "}\n";
}

// The pieces of an ftv_vote_mem call: copy, vote without finalizing.
// Device-visible address of a host replica the GPU can read in place:
// page-locked memory mapped into the device's address space (hipHostMalloc,
// PyTorch's pinned tensors) whose whole range [p, p + bytes) lies in one
// allocation.  nullptr for pageable memory or whatever the runtime does not
// report as such an allocation.
const void *mapped_host(const void *p, uint64_t bytes) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  if (a.type != hipMemoryTypeHost) return nullptr;
  void *base = nullptr;
  size_t size = 0;
  if (hipPointerGetAttribute(&base, HIP_POINTER_ATTRIBUTE_RANGE_START_ADDR, (hipDeviceptr_t)p) != hipSuccess ||
      hipPointerGetAttribute(&size, HIP_POINTER_ATTRIBUTE_RANGE_SIZE, (hipDeviceptr_t)p) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  const char *b = static_cast<const char *>(base), *q = static_cast<const char *>(p);
  if (!b || q < b || bytes > size || (uint64_t)(q - b) > size - bytes) return nullptr;
  hipPointerAttribute_t ab;
  if (hipPointerGetAttributes(&ab, base) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  if (ab.type != hipMemoryTypeHost || !ab.devicePointer || ab.hostPointer != base) return nullptr;
  return static_cast<const char *>(ab.devicePointer) + (q - b);
}

int mem_pieces(ftv_ctx *c, const ftv_vote_desc *desc, const int32_t *memory, const TaskD &t, const VoteWs &ws,
               bool vec, uint64_t es, uint64_t chunk, uint64_t set_bytes, uint32_t nhost, hipStream_t s) {
  const uint64_t n = desc->n;
  for (uint64_t off = 0, i = 0; off < n; off += chunk, ++i) {
    const int j = (int)(i & 1);
    const uint64_t len = std::min<uint64_t>(chunk, n - off);
    if (i >= 2) HIPCHK(hipStreamWaitEvent(c->copy_stream, c->mem_consumed[j], 0));
    char *set = c->stage + (uint64_t)j * set_bytes;
    TaskD tc = t;
    uint32_t h = 0;
    for (uint32_t r = 0; r < desc->k; ++r) {
      const char *src = reinterpret_cast<const char *>(desc->replicas[r]) + off * es;
      if (memory[r] == FTV_MEM_HOST) {
        char *dst = set + (uint64_t)h++ * (set_bytes / nhost);
        HIPCHK(hipMemcpyAsync(dst, src, len * es, hipMemcpyHostToDevice, c->copy_stream));
        tc.rep[r] = dst;
      } else {
        tc.rep[r] = src;
      }
    }
    HIPCHK(hipEventRecord(c->mem_copied[j], c->copy_stream));
    HIPCHK(hipStreamWaitEvent(s, c->mem_copied[j], 0));
    tc.cons = desc->consensus ? reinterpret_cast<char *>(desc->consensus) + off * es : nullptr;
    tc.mask = desc->mask ? desc->mask + off : nullptr;
    tc.n = len;
    tc.vec = vec ? 1u : 0u;
    tc.nvec = vec ? len / (16 / es) : len;
    hipError_t e = launch_vote_task(tc, ws, c->num_cus, s, false);
    if (e != hipSuccess) return hip_fail(e, "vote kernel launch");
    HIPCHK(hipEventRecord(c->mem_consumed[j], s));
  }
  return FTV_OK;
}

}  // namespace

// ===========================================================================
extern "C" {

const char *ftv_version(void) { return "ftv 0.1 gfx950"; }

const char *ftv_last_error(void) { return g_err.c_str(); }

int64_t ftv_now_ns(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (int64_t)ts.tv_sec * 1000000000ll + ts.tv_nsec;
}

int ftv_ctx_create(int device, ftv_ctx **out) {
  if (!out) return fail(FTV_E_INVALID, "NULL output handle");
  *out = nullptr;
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(FTV_E_INVALID, "no such device");
  HIPCHK(hipSetDevice(device));
  ftv_ctx *c = new (std::nothrow) ftv_ctx();
  if (!c) return fail(FTV_E_NOMEM, "out of host memory");
  c->device = device;
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "hipGetDeviceProperties");
  }
  c->num_cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  c->name = prop.gcnArchName;
  c->cfg = kDefaultCfg;
  const size_t slot_bytes = sizeof(uint64_t) * kSlotWords * kStreamSlots;
  bool ok = hipMalloc(&c->slots, slot_bytes) == hipSuccess && hipMemset(c->slots, 0, slot_bytes) == hipSuccess &&
            hipMalloc(&c->d_queue, 256) == hipSuccess &&
            hipEventCreateWithFlags(&c->staged, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&c->batch_done, hipEventDisableTiming) == hipSuccess &&
            hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) == hipSuccess &&
            hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    ftv_ctx_destroy(c);
    return fail(FTV_E_NOMEM, "cannot allocate the context workspace");
  }
  *out = c;
  return FTV_OK;
}

}  // extern "C"

namespace ftv {
RunState *&ctx_run_state(ftv_ctx *c) { return c->run; }
}  // namespace ftv

extern "C" {

int ftv_ctx_destroy(ftv_ctx *c) {
  if (!c) return FTV_OK;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  free_batch(c);
  run_state_destroy(c->run);
  for (uint32_t i = 0; i < 2 * kMaxTimed && c->tev[0]; ++i) (void)hipEventDestroy(c->tev[i]);
  if (c->slots) (void)hipFree(c->slots);
  if (c->d_queue) (void)hipFree(c->d_queue);
  if (c->staged) (void)hipEventDestroy(c->staged);
  if (c->batch_done) (void)hipEventDestroy(c->batch_done);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->mem_ready) {
    (void)hipEventDestroy(c->mem_entry);
    for (int j = 0; j < 2; ++j) {
      (void)hipEventDestroy(c->mem_copied[j]);
      (void)hipEventDestroy(c->mem_consumed[j]);
    }
    (void)hipEventDestroy(c->mem_done);
    (void)hipStreamDestroy(c->copy_stream);
  }
  if (c->stage) (void)hipFree(c->stage);
  if (c->blk_fps) (void)hipFree(c->blk_fps);
  for (void *p : c->retired) (void)hipFree(p);
  if (c->blk_done) (void)hipEventDestroy(c->blk_done);
  delete c;
  return FTV_OK;
}

int ftv_vote(ftv_ctx *c, const ftv_vote_desc *desc, void *stream) {
  if (!c) return fail(FTV_E_INVALID, "NULL context");
  TaskD t;
  int rc = make_task(desc, false, &t);
  if (rc) return rc;
  VoteWs ws{nullptr};
  rc = stream_slot(c, (hipStream_t)stream, &ws.acc);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (c->timing && c->ntev < kMaxTimed) {
    hipEvent_t *ev = c->tev + 2 * c->ntev;
    HIPCHK(hipEventRecord(ev[0], s));
    hipError_t e = launch_vote_task(t, ws, c->num_cus, s, false);
    if (e != hipSuccess) return hip_fail(e, "vote kernel launch");
    HIPCHK(hipEventRecord(ev[1], s));
    e = launch_vote_finalize(t, ws, s);
    if (e != hipSuccess) return hip_fail(e, "finalize kernel launch");
    ++c->ntev;
    return FTV_OK;
  }
  hipError_t e = launch_vote_task(t, ws, c->num_cus, s);
  if (e != hipSuccess) return hip_fail(e, "vote kernel launch");
  return FTV_OK;
}

int ftv_ctx_set_timing(ftv_ctx *c, int on) {
  if (!c || (on != 0 && on != 1)) return fail(FTV_E_INVALID, "NULL context or on not 0/1");
  if (on && !c->tev[0]) {
    for (uint32_t i = 0; i < 2 * kMaxTimed; ++i)
      if (hipEventCreate(&c->tev[i]) != hipSuccess) {
        (void)hipGetLastError();
        for (uint32_t j = 0; j < i; ++j) (void)hipEventDestroy(c->tev[j]);
        memset(c->tev, 0, sizeof(c->tev));
        return fail(FTV_E_HIP, "cannot create the timing events");
      }
  }
  c->timing = on != 0;
  c->ntev = 0;
  return FTV_OK;
}

int ftv_ctx_kernel_times(ftv_ctx *c, float *ms, uint32_t cap, uint32_t *count) {
  if (!c || !count || (cap && !ms)) return fail(FTV_E_INVALID, "NULL argument");
  const uint32_t n = std::min(c->ntev, cap);
  for (uint32_t i = 0; i < n; ++i) {
    HIPCHK(hipEventSynchronize(c->tev[2 * i + 1]));
    HIPCHK(hipEventElapsedTime(&ms[i], c->tev[2 * i], c->tev[2 * i + 1]));
  }
  *count = c->ntev;
  c->ntev = 0;
  return FTV_OK;
}


int ftv_vote_mem(ftv_ctx *c, const ftv_vote_desc *desc, const int32_t *memory, uint64_t chunk_bytes,
                 void *stream) {
  if (!c) return fail(FTV_E_INVALID, "NULL context");
  if (!desc || !memory) return fail(FTV_E_INVALID, "NULL argument");
  TaskD t;
  int rc = make_task(desc, false, &t);
  if (rc) return rc;
  for (uint32_t r = 0; r < desc->k; ++r)
    if (memory[r] != FTV_MEM_HOST && memory[r] != FTV_MEM_DEVICE)
      return fail(FTV_E_INVALID, "memory[r] must be FTV_MEM_HOST or FTV_MEM_DEVICE");
  if (desc->n == 0) return ftv_vote(c, desc, stream);
  // host replicas the device can read in place (pinned, mapped) are voted
  // there, over the link; only pageable ones go through the staging sets
  ftv_vote_desc dd = *desc;
  int32_t mem[FTV_MAX_K];
  uint32_t nhost = 0;
  const uint64_t rbytes = desc->n * (uint64_t)elem_size(desc->dtype);
  for (uint32_t r = 0; r < desc->k; ++r) {
    mem[r] = memory[r];
    if (memory[r] != FTV_MEM_HOST) continue;
    const void *m = mapped_host(desc->replicas[r], rbytes);
    if (m) {
      dd.replicas[r] = m;
      mem[r] = FTV_MEM_DEVICE;
    } else {
      ++nhost;
    }
  }
  if (nhost == 0) return ftv_vote(c, &dd, stream);
  desc = &dd;
  memory = mem;
  rc = make_task(desc, false, &t);
  if (rc) return rc;
  if (chunk_bytes < (1u << 20) || chunk_bytes > (1ull << 32))
    return fail(FTV_E_INVALID, "chunk_bytes must be in [1 MiB, 4 GiB]");
  // the staged pieces are aligned, so every piece takes the vector path when
  // the device replicas and the outputs allow it
  bool vec = (!desc->consensus || (uintptr_t)desc->consensus % 16 == 0) &&
             (!desc->mask || (uintptr_t)desc->mask % 4 == 0);
  for (uint32_t r = 0; r < desc->k; ++r)
    if (memory[r] == FTV_MEM_DEVICE) vec = vec && (uintptr_t)desc->replicas[r] % 16 == 0;
  const uint64_t es = (uint64_t)elem_size(desc->dtype);
  const uint64_t chunk = chunk_bytes / es / 4096 * 4096;  // elements per piece (whole vectors)
  const uint64_t set_bytes = (chunk * es + 255) / 256 * 256 * nhost;
  hipStream_t s = (hipStream_t)stream;
  if (!c->mem_ready) {
    bool ok = hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&c->mem_entry, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&c->mem_done, hipEventDisableTiming) == hipSuccess;
    for (int j = 0; j < 2; ++j)
      ok = ok && hipEventCreateWithFlags(&c->mem_copied[j], hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&c->mem_consumed[j], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      return fail(FTV_E_HIP, "cannot create the staging stream and events");
    }
    c->mem_ready = true;
  }
  VoteWs ws{nullptr};
  rc = stream_slot(c, s, &ws.acc);
  if (rc) return rc;
  // the staging sets are the context's: a call on another stream than the
  // last one is ordered after it on the device
  if (c->mem_pending && c->mem_stream != s) HIPCHK(hipStreamWaitEvent(s, c->mem_done, 0));
  if (c->stage_bytes < 2 * set_bytes) {
    HIPCHK(hipStreamSynchronize(s));  // the old staging may still be read
    HIPCHK(hipStreamSynchronize(c->copy_stream));
    if (c->stage) (void)hipFree(c->stage);
    c->stage = nullptr;
    c->stage_bytes = 0;
    if (hipMalloc(&c->stage, 2 * set_bytes) != hipSuccess) {
      (void)hipGetLastError();
      c->stage = nullptr;
      return fail(FTV_E_NOMEM, "cannot allocate the staging buffers");
    }
    c->stage_bytes = 2 * set_bytes;
  }
  // copies into a staging set wait for the votes that last read it: the
  // previous calls' (this entry event) and the piece two before
  HIPCHK(hipEventRecord(c->mem_entry, s));
  HIPCHK(hipStreamWaitEvent(c->copy_stream, c->mem_entry, 0));
  rc = mem_pieces(c, desc, memory, t, ws, vec, es, chunk, set_bytes, nhost, s);
  if (rc != FTV_OK) {
    // leave the accumulators zeroed for the next call
    (void)hipMemsetAsync(ws.acc, 0, sizeof(uint64_t) * kNumCounters, s);
    return rc;
  }
  hipError_t e = launch_vote_finalize(t, ws, s);
  if (e != hipSuccess) return hip_fail(e, "finalize kernel launch");
  HIPCHK(hipEventRecord(c->mem_done, s));
  c->mem_stream = s;
  c->mem_pending = true;
  return FTV_OK;
}


int ftv_vote_batch(ftv_ctx *c, const ftv_vote_desc *descs, uint64_t ntasks, void *stream) {
  if (!c) return fail(FTV_E_INVALID, "NULL context");
  if (ntasks && !descs) return fail(FTV_E_INVALID, "NULL descriptor array");
  return batch_run(c, descs, ntasks, (hipStream_t)stream);
}

int ftv_batch_get_config(ftv_ctx *c, ftv_batch_cfg *out) {
  if (!c || !out) return fail(FTV_E_INVALID, "NULL argument");
  *out = c->cfg;
  return FTV_OK;
}

int ftv_batch_set_config(ftv_ctx *c, const ftv_batch_cfg *cfg) {
  if (!c || !cfg) return fail(FTV_E_INVALID, "NULL argument");
  int rc = cfg_check(*cfg);
  if (rc) return rc;
  c->cfg = *cfg;
  return FTV_OK;
}

int ftv_tune_batch(ftv_ctx *c, const ftv_vote_desc *descs, uint64_t ntasks, void *stream,
                   uint32_t iters, ftv_batch_cfg *best) {
  if (!c) return fail(FTV_E_INVALID, "NULL context");
  if (ntasks && !descs) return fail(FTV_E_INVALID, "NULL descriptor array");
  hipStream_t s = (hipStream_t)stream;
  if (iters < 1) iters = 1;
  const char *path = getenv("FTV_TUNE_CACHE");
  const std::string key = tune_key(c, descs, ntasks);
  ftv_batch_cfg hit;
  if (path && *path && cache_lookup(path, key, &hit)) {
    c->cfg = hit;
    int rc = batch_run(c, descs, ntasks, s);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(s));
    if (best) *best = hit;
    return FTV_OK;
  }
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  // the mean of n back-to-back runs after a warm one, as an application
  // issues them: each call's host work (validating, ordering and uploading
  // the descriptors) overlaps the previous call's kernels, so the estimate is
  // the device time and not the host's
  auto time_cfg_n = [&](const ftv_batch_cfg &cfg, uint32_t n, double *ms) -> int {
    c->cfg = cfg;
    int rc = batch_run(c, descs, ntasks, s);  // warm: capture + first touch
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipEventRecord(e0, s));
    for (uint32_t i = 0; i < n; ++i) {
      rc = batch_run(c, descs, ntasks, s);
      if (rc) return rc;
    }
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float total = 0;
    HIPCHK(hipEventElapsedTime(&total, e0, e1));
    *ms = total / n;
    return FTV_OK;
  };
  auto time_cfg = [&](const ftv_batch_cfg &cfg, double *ms) { return time_cfg_n(cfg, iters, ms); };
  // coordinate descent from the current schedule, one parameter at a time,
  // two passes; then the winner is re-timed against the starting schedule
  const ftv_batch_cfg start = c->cfg;
  ftv_batch_cfg cur = start;
  double best_ms = 1e30;
  int rc = time_cfg(cur, &best_ms);
  const std::vector<uint32_t> tiles = {1024, 4096, 16384, 65536, 131072, 262144};
  const std::vector<uint32_t> blocks = {256, 512};
  const std::vector<uint32_t> grids = {1, 2, 3, 4, 8};
  const std::vector<uint32_t> orders = {0, 1, 2, 3};
  const std::vector<uint32_t> nts = {0, 1};
  for (int field = 0; field < 10 && rc == FTV_OK; ++field) {
    const int f5 = field % 5;
    const std::vector<uint32_t> &vals =
        f5 == 0 ? tiles : f5 == 1 ? blocks : f5 == 2 ? grids : f5 == 3 ? orders : nts;
    for (uint32_t v : vals) {
      ftv_batch_cfg cand = cur;
      uint32_t *f = f5 == 0 ? &cand.tile_vecs : f5 == 1 ? &cand.block
                  : f5 == 2 ? &cand.grid_mult : f5 == 3 ? &cand.order : &cand.nt_stores;
      if (*f == v) continue;
      *f = v;
      double ms = 0;
      rc = time_cfg(cand, &ms);
      if (rc) break;
      if (ms < best_ms) {
        best_ms = ms;
        cur = cand;
      }
    }
  }
  if (rc == FTV_OK && memcmp(&cur, &start, sizeof(cur)) != 0) {
    // interleaved, so that a drift of the machine's speed hits both alike
    double ms_cur = 0, ms_start = 0;
    for (int rep = 0; rep < 2 && rc == FTV_OK; ++rep) {
      double a = 0, b = 0;
      rc = time_cfg_n(cur, 2 * iters, &a);
      if (rc == FTV_OK) rc = time_cfg_n(start, 2 * iters, &b);
      ms_cur += a;
      ms_start += b;
    }
    if (rc == FTV_OK && ms_start <= ms_cur) cur = start;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  c->cfg = cur;
  rc = batch_run(c, descs, ntasks, s);  // leave the batch's outputs from the chosen schedule
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(s));
  if (path && *path) cache_store(path, key, cur);
  if (best) *best = cur;
  return FTV_OK;
}

}  // extern "C"

// ---- fingerprints and block vote --------------------------------------------
namespace {
bool pow2_in(uint64_t x, uint64_t lo, uint64_t hi) { return x >= lo && x <= hi && !(x & (x - 1)); }
}  // namespace

extern "C" {

int ftv_fingerprint(ftv_ctx *c, const void *buf, uint64_t nbytes, uint64_t block_bytes,
                    uint64_t *fp_out, void *stream) {
  if (!c) return fail(FTV_E_INVALID, "NULL context");
  if (!pow2_in(block_bytes, 4096, 65536))
    return fail(FTV_E_INVALID, "block_bytes must be a power of two in [4096, 65536]");
  if (nbytes == 0) return FTV_OK;
  if (!buf || !fp_out) return fail(FTV_E_INVALID, "NULL buffer");
  if ((uintptr_t)buf % 16) return fail(FTV_E_ALIGN, "buffer must be 16-byte aligned");
  if ((uintptr_t)fp_out % 8) return fail(FTV_E_ALIGN, "fp_out must be 8-byte aligned");
  if ((nbytes + block_bytes - 1) / block_bytes > 0x7fffffffull)
    return fail(FTV_E_INVALID, "too many blocks for one launch");
  hipError_t e = launch_fingerprint(buf, nbytes, block_bytes, fp_out, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "fingerprint kernel launch");
  return FTV_OK;
}

int ftv_vote_blocks(ftv_ctx *c, const void *const *replicas, uint32_t k, int32_t dtype,
                    uint64_t nbytes, uint64_t block_bytes, const ftv_tol *fallback_tol,
                    uint64_t *fps, uint8_t *blockmap, void *consensus, uint8_t *mask,
                    ftv_block_stats *bstats, void *stream) {
  if (!c) return fail(FTV_E_INVALID, "NULL context");
  if (!replicas || !fallback_tol || !bstats) return fail(FTV_E_INVALID, "NULL argument");
  if (k < 2 || k > FTV_MAX_K) return fail(FTV_E_K, "k must be in [2, 7]");
  int rc = check_tol(dtype, *fallback_tol);
  if (rc) return rc;
  if (!pow2_in(block_bytes, 4096, 65536))
    return fail(FTV_E_INVALID, "block_bytes must be a power of two in [4096, 65536]");
  const uint64_t es = (uint64_t)elem_size(dtype);
  if (nbytes % es) return fail(FTV_E_INVALID, "nbytes must be a multiple of the element size");
  if ((uintptr_t)bstats % 8) return fail(FTV_E_ALIGN, "bstats must be 8-byte aligned");
  const uint64_t nblocks = (nbytes + block_bytes - 1) / block_bytes;
  if (nblocks > 0x7fffffffull) return fail(FTV_E_INVALID, "too many blocks for one launch");
  if (nbytes) {
    if (!blockmap || !consensus) return fail(FTV_E_INVALID, "NULL blockmap or consensus");
    for (uint32_t r = 0; r < k; ++r) {
      if (!replicas[r]) return fail(FTV_E_INVALID, "replica pointer is NULL");
      if ((uintptr_t)replicas[r] % 16) return fail(FTV_E_ALIGN, "replicas must be 16-byte aligned");
    }
    if ((uintptr_t)consensus % 16) return fail(FTV_E_ALIGN, "consensus must be 16-byte aligned");
    if (mask && (uintptr_t)mask % 4) return fail(FTV_E_ALIGN, "mask must be 4-byte aligned");
    if (fps && (uintptr_t)fps % 8) return fail(FTV_E_ALIGN, "fps must be 8-byte aligned");
  }
  {
    // no output may touch a replica or another output: pass 1 streams
    // replica 0 into the consensus while pass 2 still reads every replica of
    // the blocks that need the element vote
    const Span outs[5] = {{consensus, nbytes}, {mask, nbytes / es}, {blockmap, nblocks},
                          {fps, fps ? (uint64_t)k * nblocks * 8 : 0}, {bstats, sizeof(ftv_block_stats)}};
    Span ins[FTV_MAX_K];
    for (uint32_t r = 0; r < k; ++r) ins[r] = {replicas[r], nbytes};
    rc = check_disjoint(outs, 5, ins, (int)k);
    if (rc) return rc;
  }
  BlockVoteD b;
  memset(&b, 0, sizeof(b));
  for (uint32_t r = 0; r < k; ++r) b.rep[r] = replicas[r];
  b.k = k;
  b.dtype = dtype;
  b.tolkind = fallback_tol->kind;
  b.tol = to_tol_d(dtype, *fallback_tol);
  b.nbytes = nbytes;
  b.block_bytes = block_bytes;
  b.nblocks = nblocks;
  b.fps = fps;
  b.blockmap = blockmap;
  b.cons = consensus;
  b.mask = mask;
  b.bstats = bstats;
  uint64_t *slot = nullptr;
  hipStream_t s = (hipStream_t)stream;
  rc = stream_slot(c, s, &slot);
  if (rc) return rc;
  b.acc = slot + kNumCounters;
  const bool own_fps = !fps && nblocks;
  if (own_fps) {
    if (!c->blk_done) HIPCHK(hipEventCreateWithFlags(&c->blk_done, hipEventDisableTiming));
    if (c->blk_pending && c->blk_stream != s) HIPCHK(hipStreamWaitEvent(s, c->blk_done, 0));
    const uint64_t words = (uint64_t)k * nblocks;
    if (words > c->blk_fps_cap) {
      uint64_t cap = 1ull << 16;
      while (cap < words) cap <<= 1;
      void *p = nullptr;
      if (hipMalloc(&p, cap * 8) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FTV_E_NOMEM, "cannot allocate the block fingerprints");
      }
      if (c->blk_fps) c->retired.push_back(c->blk_fps);
      c->blk_fps = (uint64_t *)p;
      c->blk_fps_cap = cap;
    }
    b.fps = c->blk_fps;
  }
  hipError_t e = launch_vote_blocks(b, c->num_cus, s);
  if (e != hipSuccess) return hip_fail(e, "block vote kernel launch");
  if (own_fps) {
    HIPCHK(hipEventRecord(c->blk_done, s));
    c->blk_stream = s;
    c->blk_pending = true;
  }
  return FTV_OK;
}

}  // extern "C"
