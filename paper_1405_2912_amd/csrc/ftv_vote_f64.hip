// ftv_vote_f64.hip -- per-task vote kernels for f64 values (see ftv_vote_task.hpp).
#include "ftv_vote_task.hpp"

namespace ftv {

hipError_t launch_vote_task_f64(const TaskD &t, const VoteWs &ws, int num_cus, hipStream_t s, bool finalize) {
  switch ((t.spec / 8) % 3) {
    case FTV_TOL_EXACT: return launch_vec<FTV_F64, FTV_TOL_EXACT>(t, ws, num_cus, s, finalize);
    case FTV_TOL_ULP: return launch_vec<FTV_F64, FTV_TOL_ULP>(t, ws, num_cus, s, finalize);
    case FTV_TOL_REL: return launch_vec<FTV_F64, FTV_TOL_REL>(t, ws, num_cus, s, finalize);
  }
  return hipErrorInvalidValue;
}

}  // namespace ftv
