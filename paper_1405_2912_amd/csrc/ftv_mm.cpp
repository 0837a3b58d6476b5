// ftv_mm.cpp -- memory areas with siblings and versions (Sec. IV-A, IV-C).
//
// The paper's memory management unit: a registered area has copies in host
// and device memory ("siblings"), each tagged with a version that a write
// increases by one; a request returns a sibling with the highest version in
// the requested memory, creating one by copy when that memory has none.  In
// fault-tolerant mode an existing sibling is only handed out while another
// highest-version sibling exists, so a kernel that runs into a fault never
// destroys the last good copy; a release with ok = 0 invalidates the sibling
// the kernel used (Fig. 1).  ftv_mm_check validates the highest-version
// siblings against each other by block fingerprints (the fingerprint kernel
// of ftv_blocks.hip, then a per-block vote on the device) and invalidates the
// minority.  Device-to-device copies use the streaming copy kernel of
// ftv_copy.hip (the runtime's copy reached about half its rate on MI355X).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "ftv.h"
#include "ftv_common.hpp"
#include "ftv_internal.hpp"

using namespace ftv;

namespace {

struct Sib {
  void *ptr = nullptr;
  int memory = FTV_MEM_HOST;
  bool valid = true;
  bool writing = false;
  uint32_t readers = 0;
  uint64_t version = 0;
  bool caller = false;  // the registered area: never freed by the manager
};

struct Area {
  uint64_t bytes = 0;
  std::vector<Sib> sibs;
};

}  // namespace

struct ftv_mm {
  int device = -1;
  int num_cus = 256;
  bool ft = false;
  std::mutex mu;
  std::vector<Area> areas;
  // ftv_mm_check workspace (grown on demand)
  void *staging = nullptr;
  uint64_t staging_bytes = 0;
  uint64_t *d_fps = nullptr;
  uint64_t fps_cap = 0;
  uint32_t *d_res = nullptr;   // vote result: flags per sibling + unresolved count
  uint32_t *h_res = nullptr;   // pinned copy
};

namespace {

constexpr size_t kResBytes = 4 * (FTV_MM_MAX_SIBLINGS + 2) + 8;

uint64_t newest(const Area &a) {
  uint64_t v = 0;
  for (const Sib &s : a.sibs)
    if (s.valid && s.version > v) v = s.version;
  return v;
}

// Valid, highest-version siblings not being written, in index order.
std::vector<uint32_t> candidates(const Area &a) {
  const uint64_t v = newest(a);
  std::vector<uint32_t> c;
  for (uint32_t i = 0; i < a.sibs.size(); ++i)
    if (a.sibs[i].valid && !a.sibs[i].writing && a.sibs[i].version == v) c.push_back(i);
  return c;
}

void free_sib(const ftv_mm *mm, Sib &s) {
  if (s.caller || !s.ptr) return;
  if (s.memory == FTV_MEM_DEVICE) (void)hipFree(s.ptr);
  else std::free(s.ptr);
  s.ptr = nullptr;
  (void)mm;
}

int alloc_sib(ftv_mm *mm, uint64_t bytes, int memory, void **out) {
  *out = nullptr;
  if (memory == FTV_MEM_DEVICE) {
    if (hipSetDevice(mm->device) != hipSuccess || hipMalloc(out, bytes) != hipSuccess) {
      (void)hipGetLastError();
      *out = nullptr;
      return fail(FTV_E_NOMEM, "cannot allocate a device sibling");
    }
    return FTV_OK;
  }
  const uint64_t rounded = (bytes + 4095) / 4096 * 4096;
  *out = std::aligned_alloc(4096, rounded);
  if (!*out) return fail(FTV_E_NOMEM, "cannot allocate a host sibling");
  return FTV_OK;
}

// Copy the area's bytes from sibling src to sibling dst; a host destination
// is complete when this returns.
int copy_sib(ftv_mm *mm, const Area &a, const Sib &src, Sib &dst, hipStream_t stream) {
  if (src.memory == FTV_MEM_HOST && dst.memory == FTV_MEM_HOST) {
    std::memcpy(dst.ptr, src.ptr, a.bytes);
    return FTV_OK;
  }
  HIPCHK(hipSetDevice(mm->device));
  if (src.memory == FTV_MEM_DEVICE && dst.memory == FTV_MEM_DEVICE) {
    HIPCHK(launch_copy(dst.ptr, src.ptr, a.bytes, mm->num_cus, stream));
    return FTV_OK;
  }
  const hipMemcpyKind kind = src.memory == FTV_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost;
  HIPCHK(hipMemcpyAsync(dst.ptr, src.ptr, a.bytes, kind, stream));
  if (dst.memory == FTV_MEM_HOST) HIPCHK(hipStreamSynchronize(stream));
  return FTV_OK;
}

// A sibling in `memory` holding the newest data, made by copy: the
// lowest-indexed stale or invalid sibling there that nobody uses, else a new
// one.  The copy source is a candidate in the same memory if there is one.
int new_sibling(ftv_mm *mm, Area &a, int memory, const std::vector<uint32_t> &cands,
                hipStream_t stream, uint32_t *out) {
  const uint64_t v = newest(a);
  uint32_t src = cands[0];
  for (uint32_t i : cands)
    if (a.sibs[i].memory == memory) {
      src = i;
      break;
    }
  int slot = -1;
  for (uint32_t i = 0; i < a.sibs.size(); ++i) {
    const Sib &s = a.sibs[i];
    if (s.memory == memory && !(s.valid && s.version == v) && s.readers == 0 && !s.writing) {
      slot = (int)i;
      break;
    }
  }
  if (slot < 0) {
    if (a.sibs.size() >= FTV_MM_MAX_SIBLINGS) return fail(FTV_E_NOMEM, "too many siblings for one area");
    Sib s;
    s.memory = memory;
    int rc = alloc_sib(mm, a.bytes, memory, &s.ptr);
    if (rc) return rc;
    a.sibs.push_back(s);
    slot = (int)a.sibs.size() - 1;
  }
  Sib &d = a.sibs[slot];
  int rc = copy_sib(mm, a, a.sibs[src], d, stream);
  if (rc) {
    d.valid = false;
    return rc;
  }
  d.version = v;
  d.valid = true;
  *out = (uint32_t)slot;
  return FTV_OK;
}

int check_area(ftv_mm *mm, uint32_t area, Area **out) {
  if (!mm) return fail(FTV_E_INVALID, "NULL manager");
  if (area >= mm->areas.size()) return fail(FTV_E_INVALID, "unknown area");
  *out = &mm->areas[area];
  return FTV_OK;
}

}  // namespace

extern "C" {

int ftv_mm_create(int device, int fault_tolerant, ftv_mm **out) {
  if (!out) return fail(FTV_E_INVALID, "NULL argument");
  *out = nullptr;
  if (fault_tolerant != 0 && fault_tolerant != 1) return fail(FTV_E_INVALID, "fault_tolerant must be 0 or 1");
  if (device < -1) return fail(FTV_E_INVALID, "device must be >= -1");
  if (device >= 0) {
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device >= ndev) return fail(FTV_E_INVALID, "no such device");
  }
  ftv_mm *mm = new (std::nothrow) ftv_mm();
  if (!mm) return fail(FTV_E_NOMEM, "out of host memory");
  mm->device = device;
  mm->ft = fault_tolerant != 0;
  if (device >= 0) {
    int cus = 0;
    const bool ok = hipSetDevice(device) == hipSuccess &&
                    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
                    hipMalloc((void **)&mm->d_res, kResBytes) == hipSuccess &&
                    hipHostMalloc((void **)&mm->h_res, kResBytes) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      ftv_mm_destroy(mm);
      return fail(FTV_E_NOMEM, "cannot allocate the manager's workspace");
    }
    if (cus > 0) mm->num_cus = cus;
  }
  *out = mm;
  return FTV_OK;
}

int ftv_mm_destroy(ftv_mm *mm) {
  if (!mm) return FTV_OK;
  if (mm->device >= 0) {
    (void)hipSetDevice(mm->device);
    (void)hipDeviceSynchronize();
  }
  for (Area &a : mm->areas)
    for (Sib &s : a.sibs) free_sib(mm, s);
  if (mm->staging) (void)hipFree(mm->staging);
  if (mm->d_fps) (void)hipFree(mm->d_fps);
  if (mm->d_res) (void)hipFree(mm->d_res);
  if (mm->h_res) (void)hipHostFree(mm->h_res);
  delete mm;
  return FTV_OK;
}

int ftv_mm_register(ftv_mm *mm, void *host_ptr, uint64_t bytes, uint32_t *area) {
  if (!mm || !host_ptr || !area) return fail(FTV_E_INVALID, "NULL argument");
  if (bytes == 0) return fail(FTV_E_INVALID, "an area needs at least one byte");
  std::lock_guard<std::mutex> lk(mm->mu);
  Area a;
  a.bytes = bytes;
  Sib s;
  s.ptr = host_ptr;
  s.memory = FTV_MEM_HOST;
  s.version = 1;
  s.caller = true;
  a.sibs.push_back(s);
  mm->areas.push_back(std::move(a));
  *area = (uint32_t)(mm->areas.size() - 1);
  return FTV_OK;
}

int ftv_mm_request(ftv_mm *mm, uint32_t area, int memory, int access, void *stream, void **ptr,
                   uint32_t *sibling) {
  if (!ptr || !sibling) return fail(FTV_E_INVALID, "NULL argument");
  if (memory != FTV_MEM_HOST && memory != FTV_MEM_DEVICE) return fail(FTV_E_INVALID, "bad memory kind");
  if (access < FTV_ACC_READ || access > FTV_ACC_READWRITE) return fail(FTV_E_INVALID, "bad access");
  if (!mm) return fail(FTV_E_INVALID, "NULL manager");
  if (memory == FTV_MEM_DEVICE && mm->device < 0)
    return fail(FTV_E_INVALID, "host-only manager: no device memory");
  std::lock_guard<std::mutex> lk(mm->mu);
  Area *a = nullptr;
  int rc = check_area(mm, area, &a);
  if (rc) return rc;
  const std::vector<uint32_t> cands = candidates(*a);
  if (cands.empty()) {
    for (const Sib &s : a->sibs)
      if (s.valid && s.writing) return fail(FTV_E_BUSY, "the newest sibling is being written");
    return fail(FTV_E_INVALID, "no valid sibling is left");
  }
  const bool writes = (access & FTV_ACC_WRITE) != 0;
  int pick = -1;
  for (uint32_t i : cands) {
    const Sib &s = a->sibs[i];
    if (s.memory == memory && !(writes && s.readers)) {
      pick = (int)i;
      break;
    }
  }
  // fault-tolerant mode keeps a second highest-version sibling as the backup
  if (pick >= 0 && mm->ft && cands.size() < 2) pick = -1;
  if (pick < 0) {
    uint32_t slot = 0;
    rc = new_sibling(mm, *a, memory, cands, (hipStream_t)stream, &slot);
    if (rc) return rc;
    pick = (int)slot;
  }
  Sib &s = a->sibs[pick];
  if (writes) s.writing = true;
  else s.readers++;
  *ptr = s.ptr;
  *sibling = (uint32_t)pick;
  return FTV_OK;
}

int ftv_mm_release(ftv_mm *mm, uint32_t area, uint32_t sibling, int ok) {
  if (ok != 0 && ok != 1) return fail(FTV_E_INVALID, "ok must be 0 or 1");
  if (!mm) return fail(FTV_E_INVALID, "NULL manager");
  std::lock_guard<std::mutex> lk(mm->mu);
  Area *a = nullptr;
  int rc = check_area(mm, area, &a);
  if (rc) return rc;
  if (sibling >= a->sibs.size()) return fail(FTV_E_INVALID, "unknown sibling");
  Sib &s = a->sibs[sibling];
  if (s.writing) {
    s.writing = false;
    if (ok) s.version = newest(*a) + 1;
    else s.valid = false;
    return FTV_OK;
  }
  if (s.readers == 0) return fail(FTV_E_INVALID, "sibling is not in use");
  s.readers--;
  if (!ok) s.valid = false;
  return FTV_OK;
}

int ftv_mm_siblings(ftv_mm *mm, uint32_t area, ftv_sibling_info *out, uint32_t cap, uint32_t *count) {
  if (!count || (cap && !out)) return fail(FTV_E_INVALID, "NULL argument");
  if (!mm) return fail(FTV_E_INVALID, "NULL manager");
  std::lock_guard<std::mutex> lk(mm->mu);
  Area *a = nullptr;
  int rc = check_area(mm, area, &a);
  if (rc) return rc;
  *count = (uint32_t)a->sibs.size();
  for (uint32_t i = 0; i < a->sibs.size() && i < cap; ++i) {
    const Sib &s = a->sibs[i];
    ftv_sibling_info &o = out[i];
    memset(&o, 0, sizeof(o));
    o.ptr = s.ptr;
    o.memory = s.memory;
    o.valid = s.valid ? 1 : 0;
    o.version = s.version;
    o.readers = s.readers;
    o.writing = s.writing ? 1 : 0;
    o.caller = s.caller ? 1 : 0;
  }
  return FTV_OK;
}

int ftv_mm_check(ftv_mm *mm, uint32_t area, uint64_t block_bytes, void *stream,
                 ftv_mm_check_result *out) {
  if (!out) return fail(FTV_E_INVALID, "NULL argument");
  if (!mm) return fail(FTV_E_INVALID, "NULL manager");
  if (mm->device < 0) return fail(FTV_E_INVALID, "host-only manager: fingerprints need the device");
  if (block_bytes < 4096 || block_bytes > 65536 || (block_bytes & (block_bytes - 1)))
    return fail(FTV_E_INVALID, "block_bytes must be a power of two in [4096, 65536]");
  std::lock_guard<std::mutex> lk(mm->mu);
  Area *a = nullptr;
  int rc = check_area(mm, area, &a);
  if (rc) return rc;
  memset(out, 0, sizeof(*out));
  const std::vector<uint32_t> cands = candidates(*a);
  const uint64_t nblocks = (a->bytes + block_bytes - 1) / block_bytes;
  out->checked = (uint32_t)cands.size();
  out->blocks = nblocks;
  if (cands.size() < 2) return FTV_OK;
  if (nblocks > 0x7fffffffull) return fail(FTV_E_INVALID, "too many blocks");
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipSetDevice(mm->device));
  const uint64_t m = cands.size();
  if (mm->fps_cap < m * nblocks) {
    HIPCHK(hipStreamSynchronize(s));
    if (mm->d_fps) (void)hipFree(mm->d_fps);
    mm->d_fps = nullptr;
    mm->fps_cap = 0;
    if (hipMalloc(&mm->d_fps, 8 * m * nblocks) != hipSuccess) {
      (void)hipGetLastError();
      mm->d_fps = nullptr;
      return fail(FTV_E_NOMEM, "cannot allocate the fingerprint workspace");
    }
    mm->fps_cap = m * nblocks;
  }
  bool any_host = false;
  for (uint32_t i : cands) any_host = any_host || a->sibs[i].memory == FTV_MEM_HOST;
  if (any_host && mm->staging_bytes < a->bytes) {
    HIPCHK(hipStreamSynchronize(s));
    if (mm->staging) (void)hipFree(mm->staging);
    mm->staging = nullptr;
    mm->staging_bytes = 0;
    if (hipMalloc(&mm->staging, a->bytes) != hipSuccess) {
      (void)hipGetLastError();
      mm->staging = nullptr;
      return fail(FTV_E_NOMEM, "cannot allocate the staging buffer");
    }
    mm->staging_bytes = a->bytes;
  }
  // fingerprint rows: device siblings first, up to FTV_MAX_K of them per
  // launch, then host siblings one at a time through the staging buffer
  // (stream order keeps each staging copy after the previous fingerprints)
  std::vector<uint32_t> order;
  for (uint32_t i : cands)
    if (a->sibs[i].memory == FTV_MEM_DEVICE) order.push_back(i);
  const uint64_t ndev = order.size();
  for (uint32_t i : cands)
    if (a->sibs[i].memory == FTV_MEM_HOST) order.push_back(i);
  for (uint64_t j0 = 0; j0 < ndev; j0 += FTV_MAX_K) {
    const void *bufs[FTV_MAX_K];
    const uint32_t g = (uint32_t)std::min<uint64_t>(FTV_MAX_K, ndev - j0);
    for (uint32_t q = 0; q < g; ++q) bufs[q] = a->sibs[order[j0 + q]].ptr;
    HIPCHK(launch_fingerprints(bufs, g, a->bytes, block_bytes, mm->d_fps + j0 * nblocks, s));
  }
  for (uint64_t j = ndev; j < m; ++j) {
    HIPCHK(hipMemcpyAsync(mm->staging, a->sibs[order[j]].ptr, a->bytes, hipMemcpyHostToDevice, s));
    HIPCHK(launch_fingerprint(mm->staging, a->bytes, block_bytes, mm->d_fps + j * nblocks, s));
  }
  HIPCHK(launch_fp_vote(mm->d_fps, (uint32_t)m, nblocks, mm->d_res, mm->num_cus, s));
  const size_t res_words = (m + 1) / 2 * 2 + 2;
  HIPCHK(hipMemcpyAsync(mm->h_res, mm->d_res, 4 * res_words, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  uint64_t unresolved = 0;
  memcpy(&unresolved, mm->h_res + (m + 1) / 2 * 2, 8);
  out->unresolved = unresolved;
  for (uint64_t j = 0; j < m; ++j)
    if (mm->h_res[j]) {
      a->sibs[order[j]].valid = false;
      out->invalidated++;
    }
  return FTV_OK;
}

}  // extern "C"
