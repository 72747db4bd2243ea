// Instantiation of the forward-evaluation kernels for K = 4 points per lane, up to 4 input variables.
#include "eval_impl.h"

namespace tgp {
template hipError_t launch_eval_kv<4, 4>(const EvalArgs&, int, bool, int, int64_t, hipStream_t);
template int occupancy_eval_kv<4, 4>(int, bool, int);
}  // namespace tgp
