// Forward-evaluation launch dispatch and the finalize kernel; the kernel
// templates live in eval_impl.h and are instantiated one (K, VM) pair per
// source file (eval_k*_v*.hip) so they compile in parallel.
#include <hip/hip_runtime.h>

#include "tgp_kernels.h"

namespace tgp {

template <int K, int VM>
hipError_t launch_eval_kv(const EvalArgs& a, int NO, bool pred, int bw, int64_t grid, hipStream_t s);

__global__ void finalize_kernel(FinalArgs a) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.P) return;
  const int st = a.info[t * kInfoStride + kInfoStatus];
  if (a.mse) a.mse[t] = st == 0 ? (float)(a.acc[t] * a.inv_D) : __builtin_nanf("");
  if (a.tree_status) a.tree_status[t] = st;
}

hipError_t launch_eval(const EvalArgs& a, int K, int VM, int NO, bool pred, int block_waves, int64_t grid,
                       hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (K == 16 && VM == 2) return launch_eval_kv<16, 2>(a, NO, pred, block_waves, grid, s);
  if (K == 8) {
    switch (VM) {
      case 2: return launch_eval_kv<8, 2>(a, NO, pred, block_waves, grid, s);
      case 4: return launch_eval_kv<8, 4>(a, NO, pred, block_waves, grid, s);
      case 8: return launch_eval_kv<8, 8>(a, NO, pred, block_waves, grid, s);
      default: return launch_eval_kv<8, 16>(a, NO, pred, block_waves, grid, s);
    }
  }
  switch (VM) {
    case 2: return launch_eval_kv<4, 2>(a, NO, pred, block_waves, grid, s);
    case 4: return launch_eval_kv<4, 4>(a, NO, pred, block_waves, grid, s);
    case 8: return launch_eval_kv<4, 8>(a, NO, pred, block_waves, grid, s);
    default: return launch_eval_kv<4, 16>(a, NO, pred, block_waves, grid, s);
  }
}

hipError_t launch_finalize(const FinalArgs& a, hipStream_t s) {
  if (a.P <= 0) return hipSuccess;
  finalize_kernel<<<(unsigned)((a.P + 255) / 256), 256, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace tgp
