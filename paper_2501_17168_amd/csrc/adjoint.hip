// Adjoint launch dispatch and the zero-fill kernel used before gradient accumulation.
#include <hip/hip_runtime.h>

#include "tgp_kernels.h"

namespace tgp {

template <int K, int VM>
hipError_t launch_adjoint_kv(const AdjArgs& a, int block_waves, int64_t grid, hipStream_t s);

hipError_t launch_adjoint(const AdjArgs& a, int K, int VM, int block_waves, int64_t grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (K == 2) {
    switch (VM) {
      case 2: return launch_adjoint_kv<2, 2>(a, block_waves, grid, s);
      case 4: return launch_adjoint_kv<2, 4>(a, block_waves, grid, s);
      case 8: return launch_adjoint_kv<2, 8>(a, block_waves, grid, s);
      default: return launch_adjoint_kv<2, 16>(a, block_waves, grid, s);
    }
  }
  if (K == 3) {
    switch (VM) {
      case 2: return launch_adjoint_kv<3, 2>(a, block_waves, grid, s);
      case 4: return launch_adjoint_kv<3, 4>(a, block_waves, grid, s);
      case 8: return launch_adjoint_kv<3, 8>(a, block_waves, grid, s);
      default: return launch_adjoint_kv<3, 16>(a, block_waves, grid, s);
    }
  }
  switch (VM) {
    case 2: return launch_adjoint_kv<4, 2>(a, block_waves, grid, s);
    case 4: return launch_adjoint_kv<4, 4>(a, block_waves, grid, s);
    case 8: return launch_adjoint_kv<4, 8>(a, block_waves, grid, s);
    default: return launch_adjoint_kv<4, 16>(a, block_waves, grid, s);
  }
}

// Zero rows x cols of a row-major float matrix with leading dimension ld
// (a fill kernel rather than a memset, so the call can sit in a captured graph).
__global__ void zero_f32_kernel(float* p, int64_t rows, int64_t cols, int64_t ld) {
  const int64_t n = rows * cols;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / cols, c = i - r * cols;
    p[r * ld + c] = 0.0f;
  }
}

hipError_t launch_zero_f32(float* p, int64_t rows, int64_t cols, int64_t ld, hipStream_t s) {
  if (!p || rows <= 0 || cols <= 0) return hipSuccess;
  const int64_t n = rows * cols;
  const int64_t blocks = n / 256 + 1 < 65536 ? n / 256 + 1 : 65536;
  zero_f32_kernel<<<(unsigned)blocks, 256, 0, s>>>(p, rows, cols, ld);
  return hipGetLastError();
}

}  // namespace tgp
