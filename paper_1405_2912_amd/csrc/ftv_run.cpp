// ftv_run.cpp -- redundant execution with light-weight fault tolerance
// (Sec. IV-B, IV-C, IV-D).
//
// A task has several implementations (kernels of processing units), each
// with a profile (runtime, valid runs, runs).  An attempt runs the task on
// the k implementations with the lowest fault-aware runtime that have not
// failed in this call, each into a replica buffer on a stream of its own, and
// waits for each with a deadline of its profiled runtime times a user factor.
// A run that reports a direct fault or misses its deadline is abandoned (its
// replica is not voted; its buffer is reused only once its work has drained)
// and its implementation is excluded; the surviving runs are voted and the
// profiles updated from the vote.  An unresolved vote starts the next attempt
// with re-ranked implementations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "ftv.h"
#include "ftv_common.hpp"
#include "ftv_internal.hpp"

using namespace ftv;

namespace ftv {

// A replica buffer with its stream and events.  Slots are reused across
// calls and freed only with the context: freeing device memory while an
// abandoned run may still write it would be unsafe, and waiting for that run
// would defeat its timeout.
struct Slot {
  void *buf = nullptr;
  uint64_t cap = 0;
  hipStream_t stream{};
  hipEvent_t start{}, end{};
  bool in_use = false;
  bool abandoned = false;  // its last run timed out or failed: reusable once `end` completes
};

struct RunState {
  std::vector<Slot> slots;
  ftv_stats *d_stats = nullptr;
  hipStream_t vote_stream{};
};

void run_state_destroy(RunState *r) {
  if (!r) return;  // the context has synchronised the device
  for (Slot &s : r->slots) {
    if (s.start) (void)hipEventDestroy(s.start);
    if (s.end) (void)hipEventDestroy(s.end);
    if (s.stream) (void)hipStreamDestroy(s.stream);
    if (s.buf) (void)hipFree(s.buf);
  }
  if (r->d_stats) (void)hipFree(r->d_stats);
  if (r->vote_stream) (void)hipStreamDestroy(r->vote_stream);
  delete r;
}

}  // namespace ftv

namespace {

// A free slot of at least `bytes`, or a new one.  An abandoned slot is free
// again once the run it was given to has finished.
int acquire_slot(RunState *rs, uint64_t bytes, uint32_t *out) {
  for (uint32_t i = 0; i < rs->slots.size(); ++i) {
    Slot &s = rs->slots[i];
    if (s.in_use || s.cap < bytes) continue;
    if (s.abandoned) {
      const hipError_t q = hipEventQuery(s.end);
      if (q == hipErrorNotReady) continue;
      (void)hipGetLastError();
      s.abandoned = false;
    }
    s.in_use = true;
    *out = i;
    return FTV_OK;
  }
  Slot s;
  s.cap = bytes;
  if (hipMalloc(&s.buf, bytes ? bytes : 16) != hipSuccess ||
      hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreate(&s.start) != hipSuccess || hipEventCreate(&s.end) != hipSuccess) {
    (void)hipGetLastError();
    if (s.start) (void)hipEventDestroy(s.start);
    if (s.end) (void)hipEventDestroy(s.end);
    if (s.stream) (void)hipStreamDestroy(s.stream);
    if (s.buf) (void)hipFree(s.buf);
    return fail(FTV_E_NOMEM, "cannot allocate a replica buffer");
  }
  s.in_use = true;
  rs->slots.push_back(s);
  *out = (uint32_t)rs->slots.size() - 1;
  return FTV_OK;
}

struct Run {
  uint32_t impl = 0;
  uint32_t slot = 0;
  int state = 0;  // 0 running, 1 finished, 2 direct fault, 3 timed out
  double deadline_s = 0;
};

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

double fault_aware(const ftv_unit &u) { return ftv_fault_aware_runtime(&u); }

}  // namespace

extern "C" {

int ftv_run_redundant(ftv_ctx *ctx, const ftv_impl *impls, uint32_t nimpl, ftv_unit *units, uint32_t nunits,
                      const ftv_redundancy_cfg *cfg, uint64_t n, void *out, ftv_redundancy_report *rep) {
  if (!ctx || !impls || !units || !cfg || !rep) return fail(FTV_E_INVALID, "NULL argument");
  if (cfg->k < 2 || cfg->k > FTV_MAX_K) return fail(FTV_E_K, "k must be in [2, 7]");
  if (cfg->max_attempts < 1) return fail(FTV_E_INVALID, "max_attempts must be >= 1");
  if (!(cfg->timeout_factor >= 0) || std::isinf(cfg->timeout_factor))
    return fail(FTV_E_INVALID, "timeout_factor must be finite and >= 0");
  int rc = check_tol(cfg->dtype, cfg->tol);
  if (rc) return rc;
  if (nimpl < 2) return fail(FTV_E_INVALID, "at least two implementations are needed");
  for (uint32_t i = 0; i < nimpl; ++i) {
    if (!impls[i].run) return fail(FTV_E_INVALID, "implementation without a run function");
    if (impls[i].unit >= nunits) return fail(FTV_E_INVALID, "implementation's unit out of range");
  }
  for (uint32_t u = 0; u < nunits; ++u)
    if (std::isnan(fault_aware(units[u]))) return fail(FTV_E_INVALID, "unit with runtime <= 0 or valid > total");
  if (n && !out) return fail(FTV_E_INVALID, "NULL output");
  const uint64_t bytes = n * (uint64_t)elem_size(cfg->dtype);
  memset(rep, 0, sizeof(*rep));
  rep->verdict = FTV_UNRESOLVED;
  const double t0 = now_s();

  RunState *&rs = ctx_run_state(ctx);
  if (!rs) {
    rs = new (std::nothrow) RunState();
    if (!rs) return fail(FTV_E_NOMEM, "out of host memory");
  }
  if (!rs->d_stats) {
    if (hipMalloc(&rs->d_stats, sizeof(ftv_stats)) != hipSuccess ||
        hipStreamCreateWithFlags(&rs->vote_stream, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      if (rs->d_stats) (void)hipFree(rs->d_stats);
      rs->d_stats = nullptr;
      return fail(FTV_E_NOMEM, "cannot allocate the runner's workspace");
    }
  }
  std::vector<char> failed(nimpl, 0);
  std::vector<Run> runs;
  // a finished run's slot is free at once; an abandoned one when it drains
  auto release_runs = [&]() {
    for (Run &r : runs) {
      Slot &s = rs->slots[r.slot];
      s.in_use = false;
      s.abandoned = r.state != 1;
    }
    runs.clear();
  };

  rc = FTV_OK;
  for (uint32_t attempt = 0; attempt < cfg->max_attempts && rc == FTV_OK; ++attempt) {
    // rank the implementations not failed in this call by their unit's F
    std::vector<uint32_t> order;
    for (uint32_t i = 0; i < nimpl; ++i)
      if (!failed[i]) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
      return fault_aware(units[impls[a].unit]) < fault_aware(units[impls[b].unit]);
    });
    // check intervals: units with F = +infinity outside the k best are passed
    // over; the first one due runs as an extra replica
    if (cfg->check_interval) {
      std::vector<char> seen(nunits, 0);
      const size_t kk = std::min<size_t>(cfg->k, order.size());
      for (size_t j = 0; j < kk; ++j) {
        ftv_unit &u = units[impls[order[j]].unit];
        seen[impls[order[j]].unit] = 1;
        u.skipped = 0;
      }
      int extra = -1;
      for (size_t j = kk; j < order.size(); ++j) {
        const uint32_t ui = impls[order[j]].unit;
        ftv_unit &u = units[ui];
        if (seen[ui] || !std::isinf(fault_aware(u))) continue;
        seen[ui] = 1;
        if (extra < 0 && u.skipped + 1 >= cfg->check_interval) {
          extra = (int)order[j];
          u.skipped = 0;
        } else {
          u.skipped += 1;
        }
      }
      order.resize(kk);
      if (extra >= 0 && order.size() < FTV_MAX_K && order.size() >= 2) order.push_back((uint32_t)extra);
    }
    if (order.size() > cfg->k + (cfg->check_interval ? 1u : 0u)) order.resize(cfg->k);
    if (order.size() < 2) break;
    rep->attempts++;
    // launch every chosen implementation into a replica of its own
    for (uint32_t i : order) {
      Run r;
      r.impl = i;
      rc = acquire_slot(rs, bytes, &r.slot);
      if (rc) break;
      Slot &s = rs->slots[r.slot];
      const ftv_unit &u = units[impls[i].unit];
      const bool profiled = u.runtime > 0 && u.valid > 0;
      const double start = now_s();
      r.deadline_s = (cfg->timeout_factor > 0 && profiled) ? start + u.runtime * cfg->timeout_factor : 0;
      (void)hipEventRecord(s.start, s.stream);
      const int frc = impls[i].run(impls[i].user, s.buf, (void *)s.stream);
      const hipError_t le = hipGetLastError();
      if (hipEventRecord(s.end, s.stream) != hipSuccess) {
        (void)hipGetLastError();
        r.state = 2;
      }
      if (frc != 0 || le != hipSuccess) r.state = 2;
      runs.push_back(r);
    }
    if (rc) break;
    // wait for each run until its deadline
    for (;;) {
      bool pending = false;
      const double t = now_s();
      for (Run &r : runs) {
        if (r.state != 0) continue;
        const hipError_t q = hipEventQuery(rs->slots[r.slot].end);
        if (q == hipSuccess) {
          r.state = 1;
        } else if (q != hipErrorNotReady) {
          (void)hipGetLastError();
          r.state = 2;
        } else if (r.deadline_s > 0 && t > r.deadline_s) {
          r.state = 3;
        } else {
          pending = true;
        }
      }
      if (!pending) break;
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    // failed runs: not valid, excluded for the rest of the call
    std::vector<uint32_t> live;
    for (uint32_t j = 0; j < runs.size(); ++j) {
      const Run &r = runs[j];
      if (r.state == 1) {
        live.push_back(j);
        continue;
      }
      failed[r.impl] = 1;
      units[impls[r.impl].unit].total += 1;
      if (r.state == 2) rep->errors++;
      else rep->timeouts++;
    }
    if (live.size() < 2) {
      release_runs();
      continue;
    }
    ftv_vote_desc d;
    memset(&d, 0, sizeof(d));
    d.k = (uint32_t)live.size();
    d.dtype = cfg->dtype;
    d.n = n;
    d.tol = cfg->tol;
    d.consensus = out;
    d.mask = nullptr;
    d.stats = rs->d_stats;
    for (uint32_t q = 0; q < live.size(); ++q) d.replicas[q] = rs->slots[runs[live[q]].slot].buf;
    ftv_stats st;
    rc = ftv_vote(ctx, &d, (void *)rs->vote_stream);
    if (rc == FTV_OK && (hipMemcpyAsync(&st, rs->d_stats, sizeof(st), hipMemcpyDeviceToHost, rs->vote_stream) !=
                             hipSuccess ||
                         hipStreamSynchronize(rs->vote_stream) != hipSuccess)) {
      (void)hipGetLastError();
      rc = fail(FTV_E_HIP, "reading the vote's stats");
    }
    if (rc == FTV_OK) {
      rep->verdict = st.verdict;
      if (st.verdict != FTV_UNRESOLVED) {
        for (uint32_t q = 0; q < live.size(); ++q) {
          const Run &r = runs[live[q]];
          ftv_unit &u = units[impls[r.impl].unit];
          u.total += 1;
          if (st.disagree[q] == 0) {
            u.valid += 1;
            float ms = 0;
            (void)hipEventElapsedTime(&ms, rs->slots[r.slot].start, rs->slots[r.slot].end);
            const double secs = ms * 1e-3;
            u.runtime = u.runtime <= 0 ? secs : u.runtime + (secs - u.runtime) / (double)u.valid;
          }
        }
        rep->winner_unit = impls[runs[live[st.winner]].impl].unit;
        release_runs();
        break;
      }
    }
    release_runs();
  }
  release_runs();
  rep->seconds = now_s() - t0;
  return rc;
}

}  // extern "C"
