// Fitness evaluation for callers that cannot allocate: the scratch that
// tgp_eval_mse takes as a caller-owned workspace comes instead from a
// file-scope device array of fixed size (each device that runs the library
// holds its own copy until the process ends).
//
// In host code the array's name is a host-side stand-in, not a device
// address: the address is looked up once per device with
// hipGetSymbolAddress, with that device current, and only that address is
// handed to the kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "tgp.h"

namespace {

constexpr size_t kScratchBytes = (size_t)TGP_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_scratch[kMaxDevices];  // device address of `scratch` on each device, once looked up

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Address of the current device's copy of `scratch`.
tgp_status scratch_ptr(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return TGP_E_HIP;
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return TGP_E_HIP;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return TGP_OK;
}

}  // namespace

extern "C" __attribute__((visibility("default"))) tgp_status tgp_eval_mse_noalloc(
    const tgp_pop* pop, const tgp_data* data, const tgp_cfg* cfg, float* mse, int32_t* tree_status,
    hipStream_t stream) {
  // the regular call's argument checks: without a workspace it returns TGP_E_WORKSPACE for
  // valid arguments, and the argument's error otherwise; it enqueues nothing either way
  const tgp_status pre = tgp_eval_mse(pop, data, cfg, mse, tree_status, nullptr, 0, stream);
  if (pre != TGP_E_WORKSPACE) return pre;
  const size_t need = tgp_workspace_bytes(pop, data, 1, 0);
  if (need == 0) return TGP_E_ARG;
  if (need > kScratchBytes) return TGP_E_TOO_LARGE;
  void* ws = nullptr;
  const tgp_status st = scratch_ptr(&ws);
  if (st != TGP_OK) return st;
  return tgp_eval_mse(pop, data, cfg, mse, tree_status, ws, kScratchBytes, stream);
}
