// Instantiation of the adjoint kernel for K = 3 points per lane, up to 8 input variables.
#include "adjoint_impl.h"

namespace tgp {
template hipError_t launch_adjoint_kv<3, 8>(const AdjArgs&, int, int64_t, hipStream_t);
}  // namespace tgp
