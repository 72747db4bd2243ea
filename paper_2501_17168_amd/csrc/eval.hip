// Forward-evaluation launch dispatch and the finalize kernel; the kernel
// templates live in eval_impl.h and are instantiated one (K, VM) pair per
// source file (eval_k*_v*.hip) so they compile in parallel.
#include <hip/hip_runtime.h>

#include <atomic>

#include "tgp_kernels.h"

namespace tgp {

template <int K, int VM>
hipError_t launch_eval_kv(const EvalArgs& a, int NO, bool pred, int bw, int64_t grid, hipStream_t s);
template <int K, int VM>
int occupancy_eval_kv(int NO, bool pred, int bw);

// Workgroup = 64 consecutive trees x segs segments. Thread (tree t, segment
// g) adds tiles g, g + segs, g + 2 segs, ... of tree t in float64, in
// increasing order; segment sums are then added in increasing g. The order
// is fixed by (ntiles, segs) alone, so the fitness is bitwise reproducible.
// Loads are coalesced: for one tile, consecutive threads read consecutive
// trees.
constexpr int kFinTrees = 64;

__global__ __launch_bounds__(1024) void finalize_kernel(FinalArgs a) {
  __shared__ double s_seg[16][kFinTrees];
  const int tl = threadIdx.x % kFinTrees;
  const int g = threadIdx.x / kFinTrees;
  const int64_t t = (int64_t)blockIdx.x * kFinTrees + tl;
  int st = 0;
  if (t < a.P) st = a.info[t * kInfoStride + kInfoStatus];
  double sum = 0.0;
  if (a.mse && t < a.P && st == 0)
    for (int64_t j = g; j < a.ntiles; j += a.segs) sum += a.part[j * a.P + t];
  if (a.segs > 1) {
    s_seg[g][tl] = sum;
    __syncthreads();
    if (g == 0)
      for (int k = 1; k < a.segs; ++k) sum += s_seg[k][tl];
  }
  if (g != 0 || t >= a.P) return;
  if (a.mse) a.mse[t] = st == 0 ? (float)(sum * a.inv_D) : __builtin_nanf("");
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

namespace {
int occupancy_eval(int K, int VM, int NO, bool pred, int bw) {
  if (K == 16 && VM == 2) return occupancy_eval_kv<16, 2>(NO, pred, bw);
  if (K == 8) {
    switch (VM) {
      case 2: return occupancy_eval_kv<8, 2>(NO, pred, bw);
      case 4: return occupancy_eval_kv<8, 4>(NO, pred, bw);
      case 8: return occupancy_eval_kv<8, 8>(NO, pred, bw);
      default: return occupancy_eval_kv<8, 16>(NO, pred, bw);
    }
  }
  switch (VM) {
    case 2: return occupancy_eval_kv<4, 2>(NO, pred, bw);
    case 4: return occupancy_eval_kv<4, 4>(NO, pred, bw);
    case 8: return occupancy_eval_kv<4, 8>(NO, pred, bw);
    default: return occupancy_eval_kv<4, 16>(NO, pred, bw);
  }
}
}  // namespace

int eval_resident_waves(int K, int VM, int NO, bool pred, int bw) {
  // cached per instantiation and workgroup shape: index (K, VM, NO, pred, bw)
  static std::atomic<int> cache[3][4][kMaxOutNarrow + 1][2][3];
  const int ki = K == 16 ? 2 : (K == 8 ? 1 : 0);
  const int vi = VM <= 2 ? 0 : (VM <= 4 ? 1 : (VM <= 8 ? 2 : 3));
  const int oi = (NO < 1 ? 1 : (NO > kMaxOutNarrow ? kMaxOutNarrow + 1 : NO)) - 1;
  const int bi = bw >= 4 ? 2 : (bw >= 2 ? 1 : 0);
  std::atomic<int>& c = cache[ki][vi][oi][pred ? 1 : 0][bi];
  int w = c.load(std::memory_order_relaxed);
  if (w == 0) {
    w = occupancy_eval(K, VM, NO, pred, bw) * bw;
    if (w <= 0) w = K >= 16 ? 8 : (K >= 8 ? 8 : 12);  // runtime gave no answer: a conservative count
    c.store(w, std::memory_order_relaxed);
  }
  return w;
}

hipError_t launch_finalize(const FinalArgs& a, hipStream_t s) {
  if (a.P <= 0) return hipSuccess;
  if (a.segs < 1 || a.segs > 16 || (a.segs & (a.segs - 1))) return hipErrorInvalidValue;
  finalize_kernel<<<(unsigned)((a.P + kFinTrees - 1) / kFinTrees), kFinTrees * a.segs, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace tgp
