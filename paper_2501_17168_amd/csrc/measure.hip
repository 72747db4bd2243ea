// Measurement helpers (not part of the evaluated method).
//
// 1. Operator cost: a straight-line compiled loop applies one operator to 8
//    independent streams of spread inputs per lane over a full-occupancy
//    grid. Its time above a reference loop without the operator, in units
//    of one extra add, is the operator's cost in VALU issue slots as a
//    compiled (not interpreted) evaluator would pay it: the unit of the
//    interpreter's roofline.
// 2. Kernel timing: when enabled, the forward path records a HIP event pair
//    around each evaluation-kernel launch on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "tgp.h"
#include "interp.h"
#include "ops.h"
#include "tgp_isa.h"
#include "tgp_kernels.h"

namespace tgp {

namespace {

// Each lane walks its own Weyl sequence u += golden-ratio constant, mapped
// to x in [-R, R): fresh, spread inputs every step, so the lanes of a wave
// take an operator's data-dependent branches as they would on real data
// (iterating x = f(x) instead would converge and keep every lane on one
// branch). OP < 0 are the references: kNull adds x; kUnit first runs x
// through kUnitOps dependent FMAs (no folding possible), so (kUnit - kNull)
// / kUnitOps is the time of one issue slot. (A single extra instruction
// partly hides in the loop's latency and would understate the slot.)
constexpr int kNull = -2, kUnit = -1, kUnitOps = 32;

template <int OP>
__device__ __forceinline__ float apply(float x, float c) {
  if constexpr (OP == kNull) return x;
  else if constexpr (OP == kUnit) {
#pragma unroll
    for (int r = 0; r < kUnitOps; ++r) x = fmaf(x, c, 0.25f);
    return x;
  }
  else if constexpr (OP == kOpAdd) return x + c;
  else if constexpr (OP == kOpSub) return x - c;
  else if constexpr (OP == kOpMul) return x * c;
  else if constexpr (OP == kOpDiv) return fabsf(x) < kDivTau ? 1.0f : c / x;
  else if constexpr (OP == kOpSin) return sinf(x);
  else if constexpr (OP == kOpCos) return cosf(x);
  else if constexpr (OP == kOpTanh) return tanhf(x);
  else if constexpr (OP == kOpExp) return exp_clamped(x);
  else if constexpr (OP == kOpLog) return log_positive(fabsf(x) + kLogEps);
  else if constexpr (OP == kOpMax) return fmaxf(x, c);
  else if constexpr (OP == kOpMin) return fminf(x, c);
  else return tanf(x);
}

template <int OP>
__global__ __launch_bounds__(256) void opcost_kernel(float* out, int iters, float c, float scale) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t u[8];
  float acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    u[k] = (t * 8u + (uint32_t)k) * 2654435761u;
    acc[k] = 0.0f;
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      u[k] += 0x9E3779B9u;
      const float x = (float)(int32_t)u[k] * scale;
      acc[k] += apply<OP>(x, c);
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += acc[k];
  out[t] = s;
}

// y[i] = the interpreter's unary operator U applied to x[i] (as the
// evaluation kernels apply it).
template <int U>
__global__ __launch_bounds__(256) void op_apply_kernel(const float* __restrict__ x, float* __restrict__ y,
                                                       int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = interp::un_op<U>(x[i]);
}

std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_prof_ev;    // recorded, not yet read
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_prof_pool;  // read, kept for reuse

}  // namespace

// Event pairs are reused from one read to the next, so that a profiled call
// costs two event records on the host, not two event creations.
void profile_before(hipStream_t s, void** token) {
  *token = nullptr;
  std::lock_guard<std::mutex> g(g_prof_mu);
  if (!g_prof_on) return;
  hipEvent_t a, b;
  if (!g_prof_pool.empty()) {
    a = g_prof_pool.back().first;
    b = g_prof_pool.back().second;
    g_prof_pool.pop_back();
  } else {
    if (hipEventCreate(&a) != hipSuccess) return;
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      return;
    }
  }
  (void)hipEventRecord(a, s);
  g_prof_ev.emplace_back(a, b);
  *token = (void*)b;
}

void profile_after(hipStream_t s, void* token) {
  if (token) hipEventRecord((hipEvent_t)token, s);
}

}  // namespace tgp

using namespace tgp;

extern "C" {

__attribute__((visibility("default"))) tgp_status tgp_op_cost(int32_t op, double* slots) {
  if (!slots || op < 0 || op >= kNumOps) return TGP_E_ARG;
  const int threads = 256, blocks = 4096, iters = 512;
  float* out = nullptr;
  if (hipMalloc(&out, sizeof(float) * threads * blocks) != hipSuccess) return TGP_E_HIP;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    hipFree(out);
    return TGP_E_HIP;
  }
  // input ranges: [-20, 20) for exp (its clamp range), [-8, 8) otherwise
  const float two31 = 4.656612873e-10f;  // 2^-31
  auto launch = [&](int which) {
    const float scale = (which == kOpExp ? 20.0f : 8.0f) * two31;
    switch (which) {
#define TGP_OPC(O) case O: opcost_kernel<O><<<blocks, threads, 0, 0>>>(out, iters, 0.75f, scale); break;
      TGP_OPC(kNull) TGP_OPC(kUnit)
      TGP_OPC(0) TGP_OPC(1) TGP_OPC(2) TGP_OPC(3) TGP_OPC(4) TGP_OPC(5)
      TGP_OPC(6) TGP_OPC(7) TGP_OPC(8) TGP_OPC(9) TGP_OPC(10) TGP_OPC(11)
#undef TGP_OPC
    }
  };
  auto best_ms = [&](int which) {
    launch(which);  // warm-up
    float best = 1e30f;
    for (int r = 0; r < 3; ++r) {
      hipEventRecord(e0, 0);
      launch(which);
      hipEventRecord(e1, 0);
      hipEventSynchronize(e1);
      float ms = 0;
      hipEventElapsedTime(&ms, e0, e1);
      best = ms < best ? ms : best;
    }
    return (double)best;
  };
  const double t_null = best_ms(kNull), t_unit = best_ms(kUnit), t_op = best_ms(op);
  const hipError_t err = hipGetLastError();
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(out);
  if (err != hipSuccess) return TGP_E_HIP;
  *slots = (t_op - t_null) / ((t_unit - t_null) / kUnitOps);
  return TGP_OK;
}

__attribute__((visibility("default"))) tgp_status tgp_op_apply(int32_t op, const float* x, float* y, int64_t n,
                                                               hipStream_t stream) {
  if (n < 0 || (n > 0 && (!x || !y))) return TGP_E_ARG;
  int u = -1;
  switch (op) {
    case kOpSin: u = 0; break;
    case kOpCos: u = 1; break;
    case kOpTanh: u = 2; break;
    case kOpExp: u = 3; break;
    case kOpLog: u = 4; break;
    case kOpTan: u = 5; break;
    default: return TGP_E_ARG;
  }
  if (n == 0) return TGP_OK;
  const int threads = 256;
  const unsigned blocks = (unsigned)std::min<int64_t>((n + threads - 1) / threads, 16384);
  switch (u) {
    case 0: op_apply_kernel<0><<<blocks, threads, 0, stream>>>(x, y, n); break;
    case 1: op_apply_kernel<1><<<blocks, threads, 0, stream>>>(x, y, n); break;
    case 2: op_apply_kernel<2><<<blocks, threads, 0, stream>>>(x, y, n); break;
    case 3: op_apply_kernel<3><<<blocks, threads, 0, stream>>>(x, y, n); break;
    case 4: op_apply_kernel<4><<<blocks, threads, 0, stream>>>(x, y, n); break;
    default: op_apply_kernel<5><<<blocks, threads, 0, stream>>>(x, y, n); break;
  }
  return hipGetLastError() == hipSuccess ? TGP_OK : TGP_E_HIP;
}

__attribute__((visibility("default"))) tgp_status tgp_profile(int32_t enable) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof_on = enable != 0;
  if (!g_prof_on) {  // release the reusable pairs (recorded ones wait for the next read)
    for (auto& p : g_prof_pool) {
      (void)hipEventDestroy(p.first);
      (void)hipEventDestroy(p.second);
    }
    g_prof_pool.clear();
  }
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
  }
  {
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (auto& p : ev) {
      if (g_prof_on) {
        g_prof_pool.push_back(p);
      } else {
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
      }
    }
  }
  *total_ms = tot;
  *launches = (int64_t)ev.size();
  return st;
}

}  // extern "C"
