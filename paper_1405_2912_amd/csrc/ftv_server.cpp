// ftv_server.cpp -- the voter as a service with continuous batching.
//
// Requests (a vote of k replicas already in HBM, or a fingerprint of a buffer)
// arrive from any thread.  A server thread admits them in arrival order while
// the HBM budget, the output arena and the slot count allow, and runs
// iterations: one iteration is one launch of the persistent batched vote
// kernel over a tile table that holds the next chunk (<= chunk_bytes per
// replica) of EVERY admitted request, so a request that arrives while others
// are on the GPU joins the very next launch and its tiles share the machine
// with theirs.  Two iterations are kept in flight on the server's stream so
// the device never idles while the host builds the next table.  Per-request
// counts live in slot accumulators that persist across iterations; after the
// iteration that issues a request's last tile, a small finalize kernel writes
// its stats record straight into host-mapped memory, and the server thread
// observes completion through the iteration's event.  While iterations are in
// flight, and for a millisecond after its last work, the server thread spins
// (polling events and the queue) instead of sleeping, so completions and new
// requests are seen within microseconds; an idle server waits on a condition
// variable.  Latency is measured from the request's scheduled arrival time.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ftv.h"
#include "ftv_common.hpp"
#include "ftv_internal.hpp"

using namespace ftv;

namespace {

constexpr uint32_t kTileVecs = 4096;       // largest tile: 64 KiB per replica
constexpr uint32_t kMinTileVecs = 512;     // smallest tile: one step of a 256-thread workgroup
constexpr uint64_t kMaxIterTiles = 65536;  // tiles per iteration table
constexpr int kRing = 2;                   // iterations in flight
constexpr uint64_t kGranule = 256;
constexpr int64_t kSpinNs = 1000000;      // the server thread spins for 1 ms after its last work

// First-fit allocator over one device allocation (256-byte granules).
struct Arena {
  char *base = nullptr;
  uint64_t size = 0;
  std::map<uint64_t, uint64_t> free_;  // offset -> length
  int init(uint64_t bytes) {
    size = (bytes / kGranule) * kGranule;
    if (!size) return FTV_OK;
    if (hipMalloc(&base, size) != hipSuccess) {
      (void)hipGetLastError();
      base = nullptr;
      size = 0;
      return fail(FTV_E_NOMEM, "cannot allocate the server output arena");
    }
    free_[0] = size;
    return FTV_OK;
  }
  static uint64_t round(uint64_t b) { return ((b ? b : 1) + kGranule - 1) / kGranule * kGranule; }
  void *alloc(uint64_t bytes) {
    const uint64_t need = round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= need) {
        const uint64_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > need) free_[off + need] = len - need;
        return base + off;
      }
    }
    return nullptr;
  }
  void release(void *p, uint64_t bytes) {
    if (!p) return;
    uint64_t off = (uint64_t)((char *)p - base), len = round(bytes);
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + len == next->first) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += len;
        return;
      }
    }
    free_[off] = len;
  }
  void destroy() {
    if (base) (void)hipFree(base);
    base = nullptr;
    free_.clear();
  }
};

enum { Q_QUEUED = 0, Q_ACTIVE = 1, Q_DONE = 2 };

struct Req {
  uint64_t ticket = 0;
  ftv_request rq{};
  int state = Q_QUEUED;
  int64_t t_arrival = 0, t_submit = 0, t_admit = 0, t_done = 0;
  uint64_t in_bytes = 0, out_bytes = 0, replica_bytes = 0;
  int slot = -1;
  uint64_t nvec = 0;
  uint32_t tile_vecs = kTileVecs;
  uint32_t ntiles = 0, issued = 0;
  bool new_slot = false;
  void *cons = nullptr;
  uint8_t *mask = nullptr;
  uint64_t *fps = nullptr;
  uint64_t nfps = 0;
  bool own_cons = false, own_mask = false, own_fps = false;
  uint64_t cons_bytes = 0, mask_bytes = 0;
  int status = FTV_OK;
  bool admitted = false;  // its bytes count against the budget
  ftv_stats stats{};
};

struct Iter {
  hipEvent_t ev{};
  bool busy = false;
  // [hdr 256 B][new slots u32 x max_slots][finishing slots u32 x max_slots]
  // [task records of the new slots][tiles]
  char *h_buf = nullptr;
  char *h_buf_dev = nullptr;  // the device's address of h_buf (pinned, mapped)
  char *d_buf = nullptr;
  uint32_t *d_queue = nullptr;
  std::vector<uint64_t> finishing;
};

}  // namespace

struct ftv_server {
  ftv_server_cfg cfg{};
  int num_cus = 256;
  hipStream_t stream{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread th;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Req> reqs;
  std::vector<uint64_t> active;   // admitted votes with tiles still to issue
  std::vector<uint64_t> fp_wait;  // admitted fingerprints not yet launched
  std::vector<int> free_slots;
  uint64_t bytes_in_flight = 0, peak_bytes = 0;
  Arena arena;
  TaskD *d_tasks = nullptr, *h_tasks = nullptr;
  uint64_t *d_acc = nullptr;
  ftv_stats *h_stats = nullptr, *d_stats = nullptr;
  Iter ring[kRing];
  int ring_next = 0;
  // statistics
  uint64_t submitted = 0, completed = 0, rejected = 0, iterations = 0, peak_q = 0;
  uint64_t shared_iters = 0, max_reqs_iter = 0;
  double q_integral = 0;
  int64_t q_last_t = 0, t_first = 0, t_last_done = 0;
  int64_t t_active = 0;  // last time the server thread admitted, launched or completed work
  uint64_t replica_bytes_done = 0;
  std::vector<double> lat_us;
};

namespace {

// Bytes of an iteration table at most: header, two slot lists, the task
// records of up to max_slots new requests (the tiles start at the next
// 256-byte boundary after them) and kMaxIterTiles tiles.
size_t iter_bytes(const ftv_server *s) {
  return 256 + 2 * sizeof(uint32_t) * s->cfg.max_slots + (sizeof(TaskD) * s->cfg.max_slots + 255) / 256 * 256 +
         sizeof(TileD) * kMaxIterTiles;
}

// Tile size of a request: as small as one workgroup step, as large as 64 KiB
// per replica, and just large enough that the request alone fills the
// iteration's grid once (3 workgroups per CU).  A small request is then spread
// over many workgroups that each take one short tile -- its latency is a few
// load round trips instead of the sixteen steps of one 64 KiB tile -- while a
// large one keeps long tiles and few queue operations.
uint32_t request_tile_vecs(uint64_t nvec, int num_cus) {
  const uint64_t wgs = 3ull * (uint64_t)num_cus;
  uint64_t t = (nvec + wgs - 1) / wgs;
  t = (t + kMinTileVecs - 1) / kMinTileVecs * kMinTileVecs;
  return (uint32_t)std::min<uint64_t>(std::max<uint64_t>(t, kMinTileVecs), kTileVecs);
}

void note_queue(ftv_server *s, int64_t now) {
  if (s->q_last_t) s->q_integral += (double)s->queue.size() * (double)(now - s->q_last_t);
  s->q_last_t = now;
}

void free_outputs(ftv_server *s, Req &r) {
  if (r.own_cons) s->arena.release(r.cons, r.cons_bytes);
  if (r.own_mask) s->arena.release(r.mask, r.mask_bytes);
  if (r.own_fps) s->arena.release(r.fps, r.nfps * 8);
  r.own_cons = r.own_mask = r.own_fps = false;
}

// Admit queued requests in arrival order while slots, budget and arena allow.
void admit(ftv_server *s) {
  const int64_t now = ftv_now_ns();
  while (!s->queue.empty() && !s->free_slots.empty()) {
    Req &r = s->reqs[s->queue.front()];
    if (s->bytes_in_flight + r.in_bytes + r.out_bytes > s->cfg.hbm_budget_bytes) break;
    if (r.rq.kind == FTV_REQ_VOTE) {
      ftv_vote_desc d = r.rq.vote;
      const uint64_t es = (d.dtype == FTV_F32 || d.dtype == FTV_I32) ? 4 : 8;
      if (!d.consensus) {
        r.cons_bytes = d.n * es;
        r.cons = s->arena.alloc(r.cons_bytes);
        if (!r.cons) break;
        r.own_cons = true;
      } else {
        r.cons = d.consensus;
      }
      if (!d.mask) {
        r.mask_bytes = d.n;
        r.mask = (uint8_t *)s->arena.alloc(r.mask_bytes);
        if (!r.mask) {
          free_outputs(s, r);
          break;
        }
        r.own_mask = true;
      } else {
        r.mask = d.mask;
      }
      const int slot = s->free_slots.back();
      d.consensus = r.cons;
      d.mask = r.mask;
      d.stats = s->d_stats + slot;
      TaskD t;
      const int trc = make_task(&d, true, &t);
      if (trc != FTV_OK) {
        // validated at submission with the caller's outputs; only the
        // server's own placement could fail here: end the request with the
        // error instead of launching it
        free_outputs(s, r);
        r.state = Q_DONE;
        r.status = trc;
        r.t_done = now;
        note_queue(s, now);
        s->queue.pop_front();
        s->cv_done.notify_all();
        continue;
      }
      s->free_slots.pop_back();
      r.slot = slot;
      r.nvec = t.nvec;
      r.tile_vecs = request_tile_vecs(t.nvec, s->num_cus);
      r.ntiles = (uint32_t)std::max<uint64_t>(1, (t.nvec + r.tile_vecs - 1) / r.tile_vecs);
      t.ntiles = r.ntiles;
      s->h_tasks[slot] = t;
      r.new_slot = true;
      s->active.push_back(r.ticket);
    } else {
      r.nfps = (r.rq.fp_bytes + r.rq.block_bytes - 1) / r.rq.block_bytes;
      if (r.nfps) {
        r.fps = (uint64_t *)s->arena.alloc(r.nfps * 8);
        if (!r.fps) break;
        r.own_fps = true;
      }
      r.slot = -1;
      s->fp_wait.push_back(r.ticket);
    }
    r.state = Q_ACTIVE;
    r.t_admit = now;
    r.admitted = true;
    s->bytes_in_flight += r.in_bytes + r.out_bytes;
    s->peak_bytes = std::max(s->peak_bytes, s->bytes_in_flight);
    note_queue(s, now);
    s->queue.pop_front();
  }
}

bool has_work(const ftv_server *s) { return !s->active.empty() || !s->fp_wait.empty(); }

// Build one iteration table (the next chunk of every active vote) and launch.
int launch_iteration(ftv_server *s, Iter &it) {
  uint64_t *hdr = reinterpret_cast<uint64_t *>(it.h_buf);
  const size_t slots_bytes = sizeof(uint32_t) * s->cfg.max_slots;
  uint32_t *hs = reinterpret_cast<uint32_t *>(it.h_buf + 256);
  uint32_t *hf = reinterpret_cast<uint32_t *>(it.h_buf + 256 + slots_bytes);
  TaskD *hn = reinterpret_cast<TaskD *>(it.h_buf + 256 + 2 * slots_bytes);
  uint64_t nnew = 0, nfin = 0, ntiles = 0, nreq = s->fp_wait.size();
  for (uint64_t tk : s->active)
    if (s->reqs[tk].new_slot) ++nnew;
  // the tiles follow the new slots' task records
  const size_t tiles_off = 256 + 2 * slots_bytes + (sizeof(TaskD) * nnew + 255) / 256 * 256;
  TileD *ht = reinterpret_cast<TileD *>(it.h_buf + tiles_off);
  nnew = 0;
  std::vector<uint64_t> still;
  for (uint64_t tk : s->active) {
    Req &r = s->reqs[tk];
    if (r.new_slot) {
      // the work that produces the request's replicas comes first
      if (r.rq.ready) HIPCHK(hipStreamWaitEvent(s->stream, (hipEvent_t)r.rq.ready, 0));
      hn[nnew] = s->h_tasks[r.slot];
      hs[nnew++] = (uint32_t)r.slot;
      r.new_slot = false;
    }
    const uint64_t chunk_tiles = std::max<uint64_t>(1, s->cfg.chunk_bytes / (16ull * r.tile_vecs));
    const uint64_t take = std::min<uint64_t>({chunk_tiles, (uint64_t)(r.ntiles - r.issued),
                                              kMaxIterTiles - ntiles});
    for (uint64_t j = r.issued; j < r.issued + take; ++j) {
      TileD &d = ht[ntiles++];
      d.task = (uint32_t)r.slot;
      d.v0 = std::min<uint64_t>(j * r.tile_vecs, r.nvec);
      d.v1 = std::min<uint64_t>((j + 1) * r.tile_vecs, r.nvec);
      d.last = (j + 1 == r.ntiles) ? 1u : 0u;
    }
    r.issued += (uint32_t)take;
    nreq += take ? 1 : 0;
    if (r.issued == r.ntiles) {
      it.finishing.push_back(tk);
      hf[nfin++] = (uint32_t)r.slot;
    } else {
      still.push_back(tk);
    }
  }
  s->active.swap(still);
  hdr[0] = ntiles;
  hdr[1] = s->cfg.max_slots;
  hdr[2] = nnew;
  hdr[3] = nfin;
  // the slot-init kernel reads the table in place (pinned memory) and brings
  // it into device memory for the vote and finalize kernels: no copy command
  const size_t bytes = (tiles_off + sizeof(TileD) * ntiles + 7) / 8 * 8;
  const uint64_t *d_hdr = reinterpret_cast<const uint64_t *>(it.d_buf);
  const uint32_t *d_fin = reinterpret_cast<const uint32_t *>(it.d_buf + 256 + slots_bytes);
  const uint32_t *slots_h = reinterpret_cast<const uint32_t *>(it.h_buf_dev + 256);
  const TaskD *new_h = reinterpret_cast<const TaskD *>(it.h_buf_dev + 256 + 2 * slots_bytes);
  HIPCHK(launch_slots_init(it.d_queue, s->d_acc, it.h_buf_dev, it.d_buf, bytes, slots_h, new_h, nnew, s->d_tasks,
                           s->stream));
  if (ntiles) {
    BatchLaunch b;
    b.tasks = s->d_tasks;
    b.tiles = reinterpret_cast<const TileD *>(it.d_buf + tiles_off);
    b.prefix = nullptr;  // table mode: the iteration lists its tiles
    b.tile_vecs = kTileVecs;
    b.ntiles_dev = d_hdr;
    b.acc = s->d_acc;
    b.queue_head = it.d_queue;
    b.block = 256;
    b.grid = (uint32_t)std::min<uint64_t>((uint64_t)s->num_cus * 3, ntiles);
    b.nt_stores = 1;
    HIPCHK(launch_batch_vote(b, s->stream));
  }
  HIPCHK(launch_slots_finalize(s->d_tasks, s->d_acc, d_fin, (uint32_t)nfin, s->stream));
  for (uint64_t tk : s->fp_wait) {
    Req &r = s->reqs[tk];
    if (r.rq.ready) HIPCHK(hipStreamWaitEvent(s->stream, (hipEvent_t)r.rq.ready, 0));
    if (r.rq.fp_bytes)
      HIPCHK(launch_fingerprint(r.rq.fp_buf, r.rq.fp_bytes, r.rq.block_bytes, r.fps, s->stream));
    it.finishing.push_back(tk);
  }
  s->fp_wait.clear();
  HIPCHK(hipEventRecord(it.ev, s->stream));
  it.busy = true;
  s->iterations++;
  if (nreq >= 2) s->shared_iters++;
  s->max_reqs_iter = std::max<uint64_t>(s->max_reqs_iter, nreq);
  return FTV_OK;
}

void complete_iteration(ftv_server *s, Iter &it) {
  const int64_t now = ftv_now_ns();
  for (uint64_t tk : it.finishing) {
    Req &r = s->reqs[tk];
    r.t_done = now;
    if (r.rq.kind == FTV_REQ_VOTE && r.slot >= 0) {
      memcpy(&r.stats, (const void *)(s->h_stats + r.slot), sizeof(ftv_stats));
      s->free_slots.push_back(r.slot);
    }
    r.state = Q_DONE;
    // inputs (and caller-owned outputs) leave the budget now; server-owned
    // outputs stay counted until ftv_release
    uint64_t keep = 0;
    if (r.own_cons) keep += r.cons_bytes;
    if (r.own_mask) keep += r.mask_bytes;
    if (r.own_fps) keep += r.nfps * 8;
    s->bytes_in_flight -= (r.in_bytes + r.out_bytes - keep);
    r.out_bytes = keep;
    r.in_bytes = 0;
    s->completed++;
    s->replica_bytes_done += r.replica_bytes;
    s->lat_us.push_back((double)(r.t_done - r.t_arrival) / 1e3);
    s->t_last_done = now;
  }
  it.finishing.clear();
  it.busy = false;
  s->cv_done.notify_all();
}

void fail_all(ftv_server *s, int code) {
  // a HIP failure leaves the stream unusable: finish every request with an error
  const int64_t now = ftv_now_ns();
  for (auto &kv : s->reqs) {
    Req &r = kv.second;
    if (r.state != Q_DONE) {
      r.state = Q_DONE;
      r.status = code;
      r.t_done = now;
    }
  }
  s->queue.clear();
  s->active.clear();
  s->fp_wait.clear();
  for (auto &it : s->ring) {
    it.busy = false;
    it.finishing.clear();
  }
  s->cv_done.notify_all();
}

void server_main(ftv_server *s) {
  (void)hipSetDevice(s->cfg.device);
  std::unique_lock<std::mutex> lk(s->mu);
  bool broken = false;
  for (;;) {
    bool progressed = false;
    if (!broken) admit(s);
    for (int i = 0; i < kRing && !broken; ++i) {
      Iter &it = s->ring[(s->ring_next + i) % kRing];
      if (!it.busy) continue;
      const hipError_t q = hipEventQuery(it.ev);
      if (q == hipSuccess) {
        complete_iteration(s, it);
        progressed = true;
      } else if (q != hipErrorNotReady) {
        (void)hip_fail(q, "server iteration");
        broken = true;
        fail_all(s, FTV_E_HIP);
      }
    }
    if (!broken) admit(s);
    Iter &nx = s->ring[s->ring_next];
    if (!broken && !nx.busy && has_work(s)) {
      if (launch_iteration(s, nx) != FTV_OK) {
        broken = true;
        fail_all(s, FTV_E_HIP);
      }
      s->ring_next = (s->ring_next + 1) % kRing;
      progressed = true;
    }
    bool busy = false;
    for (auto &it : s->ring) busy = busy || it.busy;
    if (s->stop && !has_work(s) && !busy) {
      // requests that can no longer be admitted (outputs never released) end here
      const int64_t now = ftv_now_ns();
      for (uint64_t tk : s->queue) {
        Req &r = s->reqs[tk];
        r.state = Q_DONE;
        r.status = FTV_E_CLOSED;
        r.t_done = now;
      }
      s->queue.clear();
      s->cv_done.notify_all();
      break;
    }
    if (broken && s->stop) break;
    if (progressed) {
      s->t_active = ftv_now_ns();
    } else if (busy || ftv_now_ns() - s->t_active < kSpinNs) {
      // iterations in flight, or work seen within the last millisecond: spin,
      // so that a finished iteration or a new request is noticed within
      // microseconds (a timed sleep of a few microseconds lasts tens of them)
      lk.unlock();
      for (int i = 0; i < 32; ++i) __builtin_ia32_pause();
      lk.lock();
    } else {
      s->cv_work.wait_for(lk, std::chrono::milliseconds(2));
    }
  }
}

void destroy_server(ftv_server *s) {
  (void)hipSetDevice(s->cfg.device);
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  for (auto &it : s->ring) {
    if (it.ev) (void)hipEventDestroy(it.ev);
    if (it.h_buf) (void)hipHostFree(it.h_buf);
    if (it.d_buf) (void)hipFree(it.d_buf);
    if (it.d_queue) (void)hipFree(it.d_queue);
  }
  if (s->d_tasks) (void)hipFree(s->d_tasks);
  if (s->h_tasks) (void)hipHostFree(s->h_tasks);
  if (s->d_acc) (void)hipFree(s->d_acc);
  if (s->h_stats) (void)hipHostFree(s->h_stats);
  s->arena.destroy();
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

}  // namespace

extern "C" {

int ftv_server_create(const ftv_server_cfg *cfg, ftv_server **out) {
  if (!cfg || !out) return fail(FTV_E_INVALID, "NULL argument");
  *out = nullptr;
  if (cfg->max_slots < 1 || cfg->max_slots > 4096 || cfg->max_queue < 1 || cfg->reserved != 0 ||
      cfg->chunk_bytes == 0 || cfg->hbm_budget_bytes == 0)
    return fail(FTV_E_INVALID, "bad server configuration");
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (cfg->device < 0 || cfg->device >= ndev) return fail(FTV_E_INVALID, "no such device");
  HIPCHK(hipSetDevice(cfg->device));
  ftv_server *s = new (std::nothrow) ftv_server();
  if (!s) return fail(FTV_E_NOMEM, "out of host memory");
  s->cfg = *cfg;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, cfg->device) == hipSuccess && prop.multiProcessorCount > 0)
    s->num_cus = prop.multiProcessorCount;
  const uint32_t ns = cfg->max_slots;
  bool ok = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) == hipSuccess &&
            hipMalloc(&s->d_tasks, sizeof(TaskD) * ns) == hipSuccess &&
            hipHostMalloc(&s->h_tasks, sizeof(TaskD) * ns) == hipSuccess &&
            hipMalloc(&s->d_acc, sizeof(uint64_t) * kNumCounters * ns) == hipSuccess &&
            hipHostMalloc(&s->h_stats, sizeof(ftv_stats) * ns, hipHostMallocMapped) == hipSuccess &&
            hipHostGetDevicePointer((void **)&s->d_stats, s->h_stats, 0) == hipSuccess;
  for (auto &it : s->ring)
    ok = ok && hipEventCreateWithFlags(&it.ev, hipEventDisableTiming) == hipSuccess &&
         hipHostMalloc(&it.h_buf, iter_bytes(s), hipHostMallocMapped) == hipSuccess &&
         hipHostGetDevicePointer((void **)&it.h_buf_dev, it.h_buf, 0) == hipSuccess && it.h_buf_dev &&
         hipMalloc(&it.d_buf, iter_bytes(s)) == hipSuccess && hipMalloc(&it.d_queue, 256) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    destroy_server(s);
    return fail(FTV_E_NOMEM, "cannot allocate the server tables");
  }
  int rc = s->arena.init(cfg->arena_bytes);
  if (rc) {
    destroy_server(s);
    return rc;
  }
  memset(s->h_stats, 0, sizeof(ftv_stats) * ns);
  for (int i = (int)ns - 1; i >= 0; --i) s->free_slots.push_back(i);
  s->th = std::thread(server_main, s);
  *out = s;
  return FTV_OK;
}

int ftv_submit(ftv_server *s, const ftv_request *req, uint64_t *ticket) {
  if (!s || !req || !ticket) return fail(FTV_E_INVALID, "NULL argument");
  if (req->reserved != 0) return fail(FTV_E_INVALID, "request.reserved must be 0");
  Req r;
  r.rq = *req;
  r.t_submit = ftv_now_ns();
  r.t_arrival = req->t_arrival_ns ? req->t_arrival_ns : r.t_submit;
  if (req->kind == FTV_REQ_VOTE) {
    ftv_vote_desc d = req->vote;
    d.stats = reinterpret_cast<ftv_stats *>(alignof(ftv_stats) * 64);  // validation only
    TaskD t;
    int rc = make_task(&d, true, &t);
    if (rc) return rc;
    const uint64_t es = (d.dtype == FTV_F32 || d.dtype == FTV_I32) ? 4 : 8;
    r.replica_bytes = d.k * d.n * es;
    r.in_bytes = r.replica_bytes;
    r.out_bytes = d.n * es + d.n;
    if ((!d.consensus || !d.mask) && s->arena.size == 0)
      return fail(FTV_E_NOMEM, "server has no output arena: pass consensus and mask buffers");
    if ((!d.consensus ? Arena::round(d.n * es) : 0) + (!d.mask ? Arena::round(d.n) : 0) > s->arena.size)
      return fail(FTV_E_NOMEM, "request outputs exceed the server output arena");
  } else if (req->kind == FTV_REQ_FINGERPRINT) {
    const uint64_t bb = req->block_bytes;
    if (bb < 4096 || bb > 65536 || (bb & (bb - 1)))
      return fail(FTV_E_INVALID, "block_bytes must be a power of two in [4096, 65536]");
    if (req->fp_bytes && (!req->fp_buf || (uintptr_t)req->fp_buf % 16))
      return fail(FTV_E_ALIGN, "fingerprint buffer must be non-NULL and 16-byte aligned");
    const uint64_t nfps = (req->fp_bytes + bb - 1) / bb;
    r.replica_bytes = req->fp_bytes;
    r.in_bytes = req->fp_bytes;
    r.out_bytes = nfps * 8;
    if (nfps && s->arena.size < Arena::round(nfps * 8))
      return fail(FTV_E_NOMEM, "server has no room for fingerprint outputs");
  } else {
    return fail(FTV_E_INVALID, "unknown request kind");
  }
  if (r.in_bytes + r.out_bytes > s->cfg.hbm_budget_bytes)
    return fail(FTV_E_NOMEM, "request footprint exceeds the server budget");
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return fail(FTV_E_CLOSED, "server is shutting down");
  if (s->queue.size() >= s->cfg.max_queue) {
    s->rejected++;
    return fail(FTV_E_BUSY, "server queue is full");
  }
  r.ticket = s->next_ticket++;
  *ticket = r.ticket;
  const int64_t now = ftv_now_ns();
  note_queue(s, now);
  if (!s->t_first) s->t_first = now;
  s->queue.push_back(r.ticket);
  s->peak_q = std::max<uint64_t>(s->peak_q, s->queue.size());
  s->reqs.emplace(r.ticket, r);
  s->submitted++;
  s->cv_work.notify_one();
  return FTV_OK;
}

int ftv_poll(ftv_server *s, uint64_t ticket, ftv_result *out, int64_t wait_us) {
  if (!s || !out) return fail(FTV_E_INVALID, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(FTV_E_CLOSED, "unknown ticket");
  auto done = [&] {
    auto f = s->reqs.find(ticket);
    return f == s->reqs.end() || f->second.state == Q_DONE;
  };
  if (!done() && wait_us != 0) {
    if (wait_us < 0) s->cv_done.wait(lk, done);
    else s->cv_done.wait_for(lk, std::chrono::microseconds(wait_us), done);
  }
  it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(FTV_E_CLOSED, "ticket released while waiting");
  const Req &r = it->second;
  if (r.state != Q_DONE) return FTV_E_NOTREADY;
  memset(out, 0, sizeof(*out));
  out->status = r.status;
  out->kind = r.rq.kind;
  out->stats = r.stats;
  out->consensus = r.cons;
  out->mask = r.mask;
  out->fps = r.fps;
  out->nfps = r.nfps;
  out->t_arrival_ns = r.t_arrival;
  out->t_submit_ns = r.t_submit;
  out->t_admit_ns = r.t_admit;
  out->t_done_ns = r.t_done;
  out->user_tag = r.rq.user_tag;
  return FTV_OK;
}

int ftv_release(ftv_server *s, uint64_t ticket) {
  if (!s) return fail(FTV_E_INVALID, "NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(FTV_E_CLOSED, "unknown ticket");
  Req &r = it->second;
  if (r.state != Q_DONE) return fail(FTV_E_NOTREADY, "request still in flight");
  free_outputs(s, r);
  // a completed request still counts its server-owned outputs (its inputs
  // left the budget at completion); one ended by a failure before completing
  // still counts all it was admitted with; one never admitted counts nothing
  if (r.admitted) s->bytes_in_flight -= r.in_bytes + r.out_bytes;
  s->reqs.erase(it);
  s->cv_work.notify_one();
  return FTV_OK;
}

int ftv_server_get_stats(ftv_server *s, ftv_server_stats *out) {
  if (!s || !out) return fail(FTV_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  memset(out, 0, sizeof(*out));
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->queued = s->queue.size();
  out->in_flight = s->submitted - s->completed - s->queue.size();
  out->rejected = s->rejected;
  out->bytes_in_flight = s->bytes_in_flight;
  out->peak_bytes_in_flight = s->peak_bytes;
  out->iterations = s->iterations;
  out->peak_queue_depth = s->peak_q;
  out->shared_iterations = s->shared_iters;
  out->max_requests_per_iteration = s->max_reqs_iter;
  const int64_t now = ftv_now_ns();
  double integral = s->q_integral;
  if (s->q_last_t) integral += (double)s->queue.size() * (double)(now - s->q_last_t);
  if (s->t_first && now > s->t_first) out->mean_queue_depth = integral / (double)(now - s->t_first);
  if (!s->lat_us.empty()) {
    std::vector<double> v = s->lat_us;
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) { return v[std::min(v.size() - 1, (size_t)(p * (double)(v.size() - 1) + 0.5))]; };
    out->p50_us = pct(0.50);
    out->p99_us = pct(0.99);
    double sum = 0;
    for (double x : v) sum += x;
    out->mean_us = sum / (double)v.size();
    out->max_us = v.back();
  }
  if (s->t_last_done > s->t_first)
    out->replica_gbps = (double)s->replica_bytes_done / (double)(s->t_last_done - s->t_first);
  return FTV_OK;
}

int ftv_server_destroy(ftv_server *s) {
  if (!s) return FTV_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->th.joinable()) s->th.join();
  destroy_server(s);
  return FTV_OK;
}

}  // extern "C"
