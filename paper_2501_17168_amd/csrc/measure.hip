// Measurement helpers (not part of the evaluated method).
//
// 1. Operator throughput: a straight-line compiled loop applies one operator
//    to 8 independent chains per lane over a full-occupancy grid, so its rate
//    is what a compiled (not interpreted) evaluator would reach for that
//    operator. Rates relative to add give each operator's cost in VALU
//    issue slots, the unit of the interpreter's roofline.
// 2. Kernel timing: when enabled, the forward path records a HIP event pair
//    around each evaluation-kernel launch on the caller's stream.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "tgp.h"
#include "tgp_isa.h"
#include "tgp_kernels.h"

namespace tgp {

namespace {

template <int OP>
__device__ __forceinline__ float step(float x, float y) {
  if constexpr (OP == kOpAdd) return x + y;
  else if constexpr (OP == kOpSub) return x - y;
  else if constexpr (OP == kOpMul) return x * y;
  else if constexpr (OP == kOpDiv) return fabsf(x) < kDivTau ? 1.0f : y / x;          // x <- 1.3 / x
  else if constexpr (OP == kOpSin) return sinf(x);
  else if constexpr (OP == kOpCos) return cosf(x);
  else if constexpr (OP == kOpTanh) return tanhf(x);
  else if constexpr (OP == kOpExp) {
    const float c = x > kExpClamp ? kExpClamp : (x < -kExpClamp ? -kExpClamp : x);
    return expf(c) - y;                                                                 // one extra sub
  } else if constexpr (OP == kOpLog) return logf(fabsf(x) + kLogEps);
  else if constexpr (OP == kOpMax) return fmaxf(x, y);
  else if constexpr (OP == kOpMin) return fminf(x, y);
  else return tanf(x) * y;                                                              // one extra mul
}

template <int OP>
__global__ __launch_bounds__(256) void opcost_kernel(float* out, int iters, float y) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  float x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = 0.5f + 0.01f * (float)((t + k) & 63);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = step<OP>(x[k], y);
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k];
  out[t] = s;
}

std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_prof_ev;

}  // namespace

void profile_before(hipStream_t s, void** token) {
  *token = nullptr;
  std::lock_guard<std::mutex> g(g_prof_mu);
  if (!g_prof_on) return;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return;
  if (hipEventCreate(&b) != hipSuccess) {
    hipEventDestroy(a);
    return;
  }
  hipEventRecord(a, s);
  g_prof_ev.emplace_back(a, b);
  *token = (void*)b;
}

void profile_after(hipStream_t s, void* token) {
  if (token) hipEventRecord((hipEvent_t)token, s);
}

}  // namespace tgp

using namespace tgp;

extern "C" {

__attribute__((visibility("default"))) tgp_status tgp_op_rate(int32_t op, double* ops_per_s) {
  if (!ops_per_s || op < 0 || op >= kNumOps) return TGP_E_ARG;
  const int threads = 256, blocks = 4096, iters = 2048;
  float* out = nullptr;
  if (hipMalloc(&out, sizeof(float) * threads * blocks) != hipSuccess) return TGP_E_HIP;
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  auto launch = [&](hipStream_t s) {
    switch (op) {
#define TGP_OPC(O) case O: opcost_kernel<O><<<blocks, threads, 0, s>>>(out, iters, O == kOpDiv ? 1.3f : (O == kOpMul ? 0.99999f : (O == kOpExp ? 1.5f : (O == kOpTan ? 0.25f : 0.001f)))); break;
      TGP_OPC(0) TGP_OPC(1) TGP_OPC(2) TGP_OPC(3) TGP_OPC(4) TGP_OPC(5)
      TGP_OPC(6) TGP_OPC(7) TGP_OPC(8) TGP_OPC(9) TGP_OPC(10) TGP_OPC(11)
#undef TGP_OPC
    }
  };
  launch(0);  // warm-up
  float best = 1e30f;
  for (int r = 0; r < 3; ++r) {
    hipEventRecord(e0, 0);
    launch(0);
    hipEventRecord(e1, 0);
    hipEventSynchronize(e1);
    float ms = 0;
    hipEventElapsedTime(&ms, e0, e1);
    best = ms < best ? ms : best;
  }
  const hipError_t err = hipGetLastError();
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(out);
  if (err != hipSuccess) return TGP_E_HIP;
  *ops_per_s = (double)threads * blocks * iters * 8 / (best * 1e-3);
  return TGP_OK;
}

__attribute__((visibility("default"))) tgp_status tgp_profile(int32_t enable) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof_on = enable != 0;
  return TGP_OK;
}

__attribute__((visibility("default"))) tgp_status tgp_profile_read(double* total_ms, int64_t* launches) {
  if (!total_ms || !launches) return TGP_E_ARG;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  {
    std::lock_guard<std::mutex> g(g_prof_mu);
    ev.swap(g_prof_ev);
  }
  double tot = 0.0;
  tgp_status st = TGP_OK;
  for (auto& p : ev) {
    float ms = 0.0f;
    if (hipEventSynchronize(p.second) != hipSuccess || hipEventElapsedTime(&ms, p.first, p.second) != hipSuccess)
      st = TGP_E_HIP;
    tot += ms;
    hipEventDestroy(p.first);
    hipEventDestroy(p.second);
  }
  *total_ms = tot;
  *launches = (int64_t)ev.size();
  return st;
}

}  // extern "C"
