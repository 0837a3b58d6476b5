// ftv_vote_i32.hip -- per-task vote kernels for i32 values (see ftv_vote_task.hpp).
#include "ftv_vote_task.hpp"

namespace ftv {

hipError_t launch_vote_task_i32(const TaskD &t, const VoteWs &ws, int num_cus, hipStream_t s, bool finalize) {
  return launch_vec<FTV_I32, FTV_TOL_EXACT>(t, ws, num_cus, s, finalize);
}

}  // namespace ftv
