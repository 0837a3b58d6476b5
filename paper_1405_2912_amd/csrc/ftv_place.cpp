// ftv_place.cpp -- placement of the voter across host and device, and the
// redundant voter.
//
// The paper's runtime keeps the voter as kernels for several processing units
// and maps each vote like any other task: it stores past execution times per
// problem size and past fault rates, and picks the unit with the lowest
// fault-aware runtime F = R / (1 - p) (Sec. IV-B), which for the voter
// depends strongly on the data size and on where the results lie (Sec. V-A,
// Fig. 3).  The voter may itself be executed redundantly, preferably not on
// the device that computed the results (Sec. IV-D).
//
// Here the units are the single-threaded host voter, the multi-threaded host
// voter and the MI355X voter.  A database keeps one profile (runtime of valid
// runs, valid runs, runs) per unit, size class (floor of log2 of the replica
// bytes) and data placement (which replicas lie in host memory, where the
// outputs go); a unit's time is the wall time of its whole run, transfers
// included.  A call runs the unit of lowest F after trying every unit once
// per key; a unit with p = 1 is re-tried as an extra, checked run at a fixed
// interval of decisions.  In redundant mode a second unit on the other device
// votes too and the two results must be bit-identical; a third unit settles
// a disagreement, and the one that disagrees with the other two is counted as
// a run that was not valid.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "ftv.h"
#include "ftv_common.hpp"

using namespace ftv;

namespace ftv {
int host_threads(uint32_t threads);
}

namespace {

struct Entry {
  ftv_unit u{0.0, 0, 0, 0};
};

// A grow-only buffer in host (pinned) or device memory.
struct Buf {
  void *p = nullptr;
  uint64_t cap = 0;
  bool dev = false;
  int ensure(uint64_t bytes) {
    if (bytes <= cap) return FTV_OK;
    if (p) (void)(dev ? hipFree(p) : hipHostFree(p));
    p = nullptr;
    cap = 0;
    const uint64_t want = bytes < 256 ? 256 : bytes;
    const hipError_t e = dev ? hipMalloc(&p, want) : hipHostMalloc(&p, want, hipHostMallocDefault);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      return fail(FTV_E_NOMEM, dev ? "cannot allocate the voter's device staging"
                                   : "cannot allocate the voter's host staging");
    }
    cap = want;
    return FTV_OK;
  }
  void release() {
    if (p) (void)(dev ? hipFree(p) : hipHostFree(p));
    p = nullptr;
    cap = 0;
  }
};

// One result set: consensus, mask and stats.
struct Set {
  Buf cons, mask, stats;
  explicit Set(bool dev) {
    cons.dev = mask.dev = stats.dev = dev;
  }
  int ensure(uint64_t cbytes, uint64_t mbytes) {
    int rc = cons.ensure(cbytes);
    if (!rc) rc = mask.ensure(mbytes);
    if (!rc) rc = stats.ensure(sizeof(ftv_stats));
    return rc;
  }
  void release() {
    cons.release();
    mask.release();
    stats.release();
  }
};

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

bool on_host(uint32_t unit) { return unit != FTV_VOTER_GPU; }

}  // namespace

struct ftv_voter_db {
  std::mutex mu;
  uint32_t check_interval = 0;
  uint32_t threads = 0;
  std::map<uint32_t, Entry> prof[FTV_NUM_VOTERS];
  uint32_t inject[FTV_NUM_VOTERS] = {0, 0, 0};
  Buf hrep[FTV_MAX_K];             // host copies of device replicas
  Set hset[3]{Set(false), Set(false), Set(false)};  // host result sets: 0 primary view, 1-2 extra runs
  Set hstage{false};               // host outputs of a host voter bound for device memory
  Set dset{true};                  // device outputs of the GPU voter when they are not the caller's
  ftv_voter_db() {
    for (Buf &b : hrep) b.dev = false;
  }
  ~ftv_voter_db() {
    for (Buf &b : hrep) b.release();
    for (Set &s : hset) s.release();
    hstage.release();
    dset.release();
  }
};

namespace {

uint32_t size_class(uint64_t bytes) {
  uint32_t c = 0;
  while (bytes > 1) {
    bytes >>= 1;
    ++c;
  }
  return c;
}

uint32_t key_of(uint64_t bytes, uint32_t host_mask, int32_t out_memory) {
  return (size_class(bytes) << 8) | (host_mask << 1) | (uint32_t)(out_memory == FTV_MEM_HOST);
}

// Where a run's outputs go.
struct Target {
  void *cons;
  uint8_t *mask;
  ftv_stats *stats;
  bool dev;  // pointers are device memory
};

// One vote of `d` (replica placement `memory`) by `unit` into `dst`.
int run_unit(ftv_ctx *ctx, ftv_voter_db *db, uint32_t unit, const ftv_vote_desc &d, const int32_t *memory,
             const Target &dst, hipStream_t s) {
  const uint64_t es = (uint64_t)elem_size(d.dtype);
  const uint64_t cb = d.consensus ? d.n * es : 0, mb = d.mask ? d.n : 0;
  int rc = FTV_OK;
  if (on_host(unit)) {
    ftv_vote_desc h = d;
    // device replicas come to the host first
    for (uint32_t r = 0; r < d.k; ++r) {
      if (memory[r] != FTV_MEM_DEVICE || d.n == 0) continue;
      rc = db->hrep[r].ensure(d.n * es);
      if (rc) return rc;
      HIPCHK(hipMemcpyAsync(db->hrep[r].p, d.replicas[r], d.n * es, hipMemcpyDeviceToHost, s));
      h.replicas[r] = db->hrep[r].p;
    }
    HIPCHK(hipStreamSynchronize(s));
    Set &stage = db->hstage;
    if (dst.dev) {
      rc = stage.ensure(cb, mb);
      if (rc) return rc;
    }
    h.consensus = d.consensus ? (dst.dev ? stage.cons.p : dst.cons) : nullptr;
    h.mask = d.mask ? (dst.dev ? (uint8_t *)stage.mask.p : dst.mask) : nullptr;
    h.stats = dst.dev ? (ftv_stats *)stage.stats.p : dst.stats;
    rc = ftv_vote_host(&h, unit == FTV_VOTER_HOST1 ? 1u : db->threads);
    if (rc) return rc;
    if (dst.dev) {
      if (cb) HIPCHK(hipMemcpyAsync(dst.cons, h.consensus, cb, hipMemcpyHostToDevice, s));
      if (mb) HIPCHK(hipMemcpyAsync(dst.mask, h.mask, mb, hipMemcpyHostToDevice, s));
      HIPCHK(hipMemcpyAsync(dst.stats, h.stats, sizeof(ftv_stats), hipMemcpyHostToDevice, s));
      HIPCHK(hipStreamSynchronize(s));
    }
    return FTV_OK;
  }
  // the MI355X voter: host replicas are streamed in by ftv_vote_mem
  ftv_vote_desc g = d;
  if (!dst.dev) {
    rc = db->dset.ensure(cb, mb);
    if (rc) return rc;
  }
  g.consensus = d.consensus ? (dst.dev ? dst.cons : db->dset.cons.p) : nullptr;
  g.mask = d.mask ? (dst.dev ? dst.mask : (uint8_t *)db->dset.mask.p) : nullptr;
  g.stats = dst.dev ? dst.stats : (ftv_stats *)db->dset.stats.p;
  rc = ftv_vote_mem(ctx, &g, memory, 64ull << 20, (void *)s);
  if (rc) return rc;
  if (!dst.dev) {
    if (cb) HIPCHK(hipMemcpyAsync(dst.cons, g.consensus, cb, hipMemcpyDeviceToHost, s));
    if (mb) HIPCHK(hipMemcpyAsync(dst.mask, g.mask, mb, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(dst.stats, g.stats, sizeof(ftv_stats), hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  return FTV_OK;
}

// A planted fault (test hook): the run's consensus, else its stats, differ.
int corrupt(const ftv_vote_desc &d, const Target &t, hipStream_t s) {
  if (d.consensus && d.n) {
    uint8_t b = 0;
    if (t.dev) {
      HIPCHK(hipMemcpyAsync(&b, t.cons, 1, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      b ^= 1;
      HIPCHK(hipMemcpyAsync(t.cons, &b, 1, hipMemcpyHostToDevice, s));
      HIPCHK(hipStreamSynchronize(s));
    } else {
      *(uint8_t *)t.cons ^= 1;
    }
    return FTV_OK;
  }
  ftv_stats st;
  if (t.dev) {
    HIPCHK(hipMemcpyAsync(&st, t.stats, sizeof(st), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    st.no_majority += 1;
    HIPCHK(hipMemcpyAsync(t.stats, &st, sizeof(st), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  } else {
    t.stats->no_majority += 1;
  }
  return FTV_OK;
}

// Host view of a result set: the caller's outputs (copied into hset[0] when
// they are device memory) or an extra run's set.
int host_view(const ftv_vote_desc &d, const Target &t, Set &tmp, hipStream_t s, Target *view) {
  if (!t.dev) {
    *view = t;
    return FTV_OK;
  }
  const uint64_t es = (uint64_t)elem_size(d.dtype);
  const uint64_t cb = d.consensus ? d.n * es : 0, mb = d.mask ? d.n : 0;
  int rc = tmp.ensure(cb, mb);
  if (rc) return rc;
  if (cb) HIPCHK(hipMemcpyAsync(tmp.cons.p, t.cons, cb, hipMemcpyDeviceToHost, s));
  if (mb) HIPCHK(hipMemcpyAsync(tmp.mask.p, t.mask, mb, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(tmp.stats.p, t.stats, sizeof(ftv_stats), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  *view = Target{cb ? tmp.cons.p : nullptr, mb ? (uint8_t *)tmp.mask.p : nullptr, (ftv_stats *)tmp.stats.p, false};
  return FTV_OK;
}

bool same_result(const ftv_vote_desc &d, const Target &a, const Target &b) {
  const uint64_t es = (uint64_t)elem_size(d.dtype);
  if (d.consensus && d.n && memcmp(a.cons, b.cons, d.n * es) != 0) return false;
  if (d.mask && d.n && memcmp(a.mask, b.mask, d.n) != 0) return false;
  return memcmp(a.stats, b.stats, sizeof(ftv_stats)) == 0;
}

void record(Entry &e, bool valid, double secs) {
  e.u.total += 1;
  if (!valid) return;
  e.u.valid += 1;
  // runtime: running mean of the valid runs
  e.u.runtime = e.u.runtime <= 0 ? secs : e.u.runtime + (secs - e.u.runtime) / (double)e.u.valid;
}

}  // namespace

extern "C" {

int ftv_voter_db_create(uint32_t check_interval, uint32_t host_threads, ftv_voter_db **out) {
  if (!out) return fail(FTV_E_INVALID, "NULL argument");
  ftv_voter_db *db = new (std::nothrow) ftv_voter_db();
  if (!db) return fail(FTV_E_NOMEM, "out of host memory");
  db->check_interval = check_interval;
  db->threads = host_threads;
  *out = db;
  return FTV_OK;
}

int ftv_voter_db_destroy(ftv_voter_db *db) {
  if (!db) return fail(FTV_E_INVALID, "NULL database");
  delete db;
  return FTV_OK;
}

int ftv_voter_db_profile(ftv_voter_db *db, uint32_t unit, uint64_t bytes, uint32_t host_mask, int32_t out_memory,
                         ftv_unit *out) {
  if (!db || !out) return fail(FTV_E_INVALID, "NULL argument");
  if (unit >= FTV_NUM_VOTERS) return fail(FTV_E_INVALID, "unknown voter unit");
  if (host_mask >= (1u << FTV_MAX_K)) return fail(FTV_E_INVALID, "host_mask has bits beyond replica 6");
  if (out_memory != FTV_MEM_HOST && out_memory != FTV_MEM_DEVICE) return fail(FTV_E_INVALID, "bad out_memory");
  std::lock_guard<std::mutex> lk(db->mu);
  const auto it = db->prof[unit].find(key_of(bytes, host_mask, out_memory));
  *out = it == db->prof[unit].end() ? ftv_unit{0.0, 0, 0, 0} : it->second.u;
  return FTV_OK;
}

int ftv_voter_db_inject(ftv_voter_db *db, uint32_t unit, uint32_t count) {
  if (!db) return fail(FTV_E_INVALID, "NULL database");
  if (unit >= FTV_NUM_VOTERS) return fail(FTV_E_INVALID, "unknown voter unit");
  std::lock_guard<std::mutex> lk(db->mu);
  db->inject[unit] = count;
  return FTV_OK;
}

int ftv_vote_placed(ftv_ctx *ctx, ftv_voter_db *db, const ftv_vote_desc *d, const int32_t *memory,
                    int32_t out_memory, uint32_t avoid, uint32_t flags, void *stream, ftv_place_report *rep) {
  if (!ctx || !db || !d || !memory || !rep) return fail(FTV_E_INVALID, "NULL argument");
  if (d->k < 2 || d->k > FTV_MAX_K) return fail(FTV_E_K, "k must be in [2, 7]");
  int rc = check_tol(d->dtype, d->tol);
  if (rc) return rc;
  if (!d->stats) return fail(FTV_E_INVALID, "stats pointer is NULL");
  if (out_memory != FTV_MEM_HOST && out_memory != FTV_MEM_DEVICE)
    return fail(FTV_E_INVALID, "out_memory must be FTV_MEM_HOST or FTV_MEM_DEVICE");
  if (flags & ~(uint32_t)FTV_PLACE_REDUNDANT) return fail(FTV_E_INVALID, "unknown flag");
  if (avoid >= (1u << FTV_NUM_VOTERS)) return fail(FTV_E_INVALID, "avoid names an unknown unit");
  uint32_t host_mask = 0;
  for (uint32_t r = 0; r < d->k; ++r) {
    if (memory[r] != FTV_MEM_HOST && memory[r] != FTV_MEM_DEVICE)
      return fail(FTV_E_INVALID, "memory[r] must be FTV_MEM_HOST or FTV_MEM_DEVICE");
    if (memory[r] == FTV_MEM_HOST) host_mask |= 1u << r;
  }
  const uint64_t es = (uint64_t)elem_size(d->dtype);
  const uint64_t cb = d->consensus ? d->n * es : 0, mb = d->mask ? d->n : 0;
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(db->mu);
  memset(rep, 0, sizeof(*rep));
  for (int j = 0; j < 3; ++j) rep->unit[j] = -1;
  rep->result_unit = -1;
  const uint32_t key = key_of(d->n * es * d->k, host_mask, out_memory);
  Entry *ent[FTV_NUM_VOTERS];
  for (uint32_t u = 0; u < FTV_NUM_VOTERS; ++u) ent[u] = &db->prof[u][key];

  // ---- decision: untried units first, then by fault-aware runtime ----
  uint32_t allowed = ((1u << FTV_NUM_VOTERS) - 1u) & ~avoid;
  if (!allowed) allowed = (1u << FTV_NUM_VOTERS) - 1u;
  auto F = [&](uint32_t u) -> double {
    const Entry &e = *ent[u];
    if (e.u.total == 0) return -1.0;  // never run for this key: try it
    if (e.u.valid == 0) return std::numeric_limits<double>::infinity();
    return e.u.runtime * ((double)e.u.total / (double)e.u.valid);
  };
  std::vector<uint32_t> order;
  for (uint32_t u = 0; u < FTV_NUM_VOTERS; ++u)
    if (allowed & (1u << u)) order.push_back(u);
  for (uint32_t u = 0; u < FTV_NUM_VOTERS; ++u)
    if (!(allowed & (1u << u))) order.push_back(u);  // avoided units: only when nothing else is left
  std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
    const bool aa = allowed & (1u << a), ab = allowed & (1u << b);
    if (aa != ab) return aa;
    return F(a) < F(b);
  });
  std::vector<uint32_t> usable;   // finite F (or untried)
  int probe = -1;                 // an infinite-F unit due for its check
  for (uint32_t u : order) {
    if (std::isinf(F(u))) {
      Entry &e = *ent[u];
      if (probe < 0 && db->check_interval && e.u.skipped + 1 >= db->check_interval) {
        probe = (int)u;
        e.u.skipped = 0;
      } else {
        e.u.skipped += 1;
      }
    } else {
      usable.push_back(u);
    }
  }
  if (usable.empty()) {
    if (probe < 0) return fail(FTV_E_MISMATCH, "every voter unit has failed for this size and placement");
    usable.push_back((uint32_t)probe);  // nothing else: the due unit runs as the primary
    probe = -1;
  }
  const bool redundant = (flags & FTV_PLACE_REDUNDANT) != 0;

  const Target caller{d->consensus, d->mask, d->stats, out_memory == FTV_MEM_DEVICE};
  auto run = [&](uint32_t u, const Target &dst, double *secs) {
    const double t0 = now_s();
    int r = run_unit(ctx, db, u, *d, memory, dst, s);
    if (r == FTV_OK && db->inject[u]) {
      db->inject[u] -= 1;
      r = corrupt(*d, dst, s);
    }
    *secs = now_s() - t0;
    const uint32_t j = rep->runs++;
    rep->unit[j] = (int32_t)u;
    rep->seconds[j] = *secs;
    return r;
  };
  auto extra_target = [&](int i, Target *t) {
    Set &st = db->hset[i];
    int r = st.ensure(cb, mb);
    if (r) return r;
    *t = Target{cb ? st.cons.p : nullptr, mb ? (uint8_t *)st.mask.p : nullptr, (ftv_stats *)st.stats.p, false};
    return FTV_OK;
  };

  // ---- primary: the best unit; a unit that fails directly is replaced by the next ----
  size_t next = 0;
  uint32_t prim = 0;
  double tp = 0;
  for (;;) {
    if (next >= usable.size()) return rc ? rc : fail(FTV_E_MISMATCH, "no voter unit left");
    prim = usable[next++];
    rc = run(prim, caller, &tp);
    if (rc == FTV_OK) break;
    record(*ent[prim], false, 0);
    if (rep->runs >= 3) return rc;
  }
  rep->result_unit = (int32_t)prim;
  if (!redundant && probe < 0) {
    record(*ent[prim], true, tp);
    return FTV_OK;
  }
  Target accepted;  // host view of the result the call returns
  rc = host_view(*d, caller, db->hset[0], s, &accepted);
  if (rc) return rc;

  // ---- redundant: a second voter, on the other device than the primary if possible ----
  auto ran = [&](uint32_t u) {
    for (uint32_t j = 0; j < rep->runs; ++j)
      if (rep->unit[j] == (int32_t)u) return true;
    return false;
  };
  int second = -1;
  if (redundant) {
    // preference: not avoided and on the other device; not avoided; avoided on the other device; any
    for (int pass = 0; pass < 4 && second < 0; ++pass)
      for (size_t i = next; i < usable.size() && second < 0; ++i) {
        const uint32_t u = usable[i];
        const bool ok_avoid = pass >= 2 || (allowed & (1u << u));
        const bool ok_dev = (pass % 2) == 1 || on_host(u) != on_host(prim);
        if (ok_avoid && ok_dev && !ran(u)) second = (int)u;
      }
    if (second < 0 && probe >= 0) {
      second = probe;
      probe = -1;
      rep->probed = 1;
    }
  }
  if (second < 0) {
    record(*ent[prim], true, tp);
  } else {
    Target st2;
    rc = extra_target(1, &st2);
    if (rc) return rc;
    double t2 = 0;
    const int rc2 = run((uint32_t)second, st2, &t2);
    const bool agree = rc2 == FTV_OK && same_result(*d, accepted, st2);
    rep->agreed = agree ? 1 : 0;
    if (agree) {
      record(*ent[prim], true, tp);
      record(*ent[second], true, t2);
    } else {
      // a third voter settles it: a unit not run yet, or a due probe
      int third = -1;
      for (uint32_t u : usable)
        if (third < 0 && !ran(u)) third = (int)u;
      if (third < 0 && probe >= 0) {
        third = probe;
        probe = -1;
        rep->probed = 1;
      }
      if (third < 0 || rep->runs >= 3) {
        if (rc2 != FTV_OK) {  // the second voter failed directly: the primary stands alone
          record(*ent[prim], true, tp);
          record(*ent[second], false, 0);
          return FTV_OK;
        }
        return fail(FTV_E_MISMATCH, "the two voters disagree and no third unit is left");
      }
      Target st3;
      rc = extra_target(2, &st3);
      if (rc) return rc;
      double t3 = 0;
      const int rc3 = run((uint32_t)third, st3, &t3);
      if (rc3 == FTV_OK && same_result(*d, accepted, st3)) {
        record(*ent[prim], true, tp);
        record(*ent[third], true, t3);
        record(*ent[second], false, 0);
      } else if (rc3 == FTV_OK && rc2 == FTV_OK && same_result(*d, st2, st3)) {
        // the primary was the odd one out: the agreed result replaces it
        record(*ent[prim], false, 0);
        record(*ent[second], true, t2);
        record(*ent[third], true, t3);
        if (caller.dev) {
          if (cb) HIPCHK(hipMemcpyAsync(caller.cons, st2.cons, cb, hipMemcpyHostToDevice, s));
          if (mb) HIPCHK(hipMemcpyAsync(caller.mask, st2.mask, mb, hipMemcpyHostToDevice, s));
          HIPCHK(hipMemcpyAsync(caller.stats, st2.stats, sizeof(ftv_stats), hipMemcpyHostToDevice, s));
          HIPCHK(hipStreamSynchronize(s));
        } else {
          if (cb) memcpy(caller.cons, st2.cons, cb);
          if (mb) memcpy(caller.mask, st2.mask, mb);
          memcpy(caller.stats, st2.stats, sizeof(ftv_stats));
        }
        rep->result_unit = second;
      } else {
        return fail(FTV_E_MISMATCH, "three voters gave three different results");
      }
    }
  }

  // ---- a unit with p = 1 due for its check votes too, checked against the result ----
  if (probe >= 0 && rep->runs < 3) {
    Target pt;
    rc = extra_target((int)rep->runs, &pt);
    if (rc) return rc;
    double tq = 0;
    const int qrc = run((uint32_t)probe, pt, &tq);
    rep->probed = 1;
    record(*ent[probe], qrc == FTV_OK && same_result(*d, accepted, pt), tq);
  }
  return FTV_OK;
}

}  // extern "C"
