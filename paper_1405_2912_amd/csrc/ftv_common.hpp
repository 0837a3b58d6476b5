// ftv_common.hpp -- host-side error handling and validation shared by the
// C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "ftv.h"
#include "ftv_internal.hpp"

namespace ftv {

extern thread_local std::string g_err;

// Record `msg` as the thread's last error and return `code`.
int fail(int code, const std::string &msg);
// Record a HIP error (and clear HIP's sticky error) and return FTV_E_HIP.
int hip_fail(hipError_t e, const char *what);

int check_tol(int dtype, const ftv_tol &t);
TolD to_tol_d(int dtype, const ftv_tol &t);
// Validate a vote descriptor into a device task record; strict = the batched
// alignment rules.
int make_task(const ftv_vote_desc *d, bool strict, TaskD *out);

// [p, p + len) as a byte range; a NULL pointer or zero length is empty.
struct Span {
  const void *p;
  uint64_t len;
};
// FTV_E_INVALID if an output range shares a byte with an input range or with
// another output range (inputs may overlap each other).
int check_disjoint(const Span *outs, int nouts, const Span *ins, int nins);
// The overlap rule of one vote descriptor: consensus, mask and stats against
// the replicas and each other.  Also rejects n above 2^60.
int check_vote_overlaps(const ftv_vote_desc *d);

// State of ftv_run_redundant kept in a context (abandoned replicas); freed
// with the context after the device has been synchronised.
struct RunState;
void run_state_destroy(RunState *r);
RunState *&ctx_run_state(ftv_ctx *c);

}  // namespace ftv

#define HIPCHK(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return ftv::hip_fail(e_, #call); \
  } while (0)
