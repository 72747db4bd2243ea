// Autotuner for the evaluation schedule.
//
// The paper switches between its hybrid and data-parallel fitness modes by
// comparing the number of data points with the GPU's core count (§III-C,
// "Choose Parallelism Adaptively"; the crossover is measured in §V-B). Here
// the choice is measured instead: every candidate (schedule x points per
// lane x waves per workgroup x trees per unit) is timed on the caller's own
// population and data, and the fastest is cached under the shape key
// (P, Lmax, V, D, n_out, gradient flag) for the rest of the process. The
// gradient call has one schedule (point-major); its candidates are the
// points per lane (2 or 4), the workgroup shape and the trees per unit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "tgp_autotune.h"
#include "tgp_isa.h"

namespace tgp {

namespace {

using Key = std::tuple<int64_t, int32_t, int32_t, int64_t, int32_t, int32_t>;
std::mutex g_mu;
std::map<Key, tgp_cfg> g_cache;

Key key_of(const tgp_pop* pop, const tgp_data* d, int n_out, bool grad) {
  return Key(pop->P, pop->Lmax, d->V, d->D, n_out, grad ? 1 : 0);
}

}  // namespace

bool autotune_lookup(const tgp_pop* pop, const tgp_data* d, int n_out, bool grad, tgp_cfg* out) {
  std::lock_guard<std::mutex> g(g_mu);
  auto it = g_cache.find(key_of(pop, d, n_out, grad));
  if (it == g_cache.end()) return false;
  *out = it->second;
  return true;
}

tgp_status autotune_run(const tgp_pop* pop, const tgp_data* d, int n_out, bool grad, tgp_cfg* out, void* ws,
                        size_t ws_bytes, hipStream_t s) {
  if (pop->P == 0) {
    *out = grad ? tgp_cfg{TGP_MODE_POINT_MAJOR, 1, 4, 1, 0} : tgp_cfg{TGP_MODE_TREE_MAJOR, 1, 8, 1, 0};
    return TGP_OK;
  }
  float* mse = nullptr;
  float* gv = nullptr;
  float* gx = nullptr;
  if (hipMalloc(&mse, sizeof(float) * (size_t)pop->P) != hipSuccess) return TGP_E_HIP;
  if (grad && (hipMalloc(&gv, sizeof(float) * (size_t)pop->P * pop->row_stride) != hipSuccess ||
               hipMalloc(&gx, sizeof(float) * (size_t)d->V * d->ldx) != hipSuccess)) {
    hipFree(mse);
    if (gv) hipFree(gv);
    return TGP_E_HIP;
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    hipFree(mse);
    if (gv) hipFree(gv);
    if (gx) hipFree(gx);
    return TGP_E_HIP;
  }
  auto run = [&](const tgp_cfg& c) {
    return grad ? tgp_eval_mse_grad(pop, d, &c, nullptr, mse, gv, gx, nullptr, ws, ws_bytes, s)
                : tgp_internal_forward(pop, d, &c, n_out, mse, ws, ws_bytes, s);
  };
  std::vector<tgp_cfg> cands;
  if (grad) {
    for (int k : {4, 2})
      for (int bw : {1, 2})
        for (int tpu : {1, 4, 16, 64}) cands.push_back(tgp_cfg{TGP_MODE_POINT_MAJOR, bw, k, tpu, 0});
  } else {
    for (int k : {16, 8, 4}) {
      if (k == 16 && d->V > 2) continue;
      if (k == 8 && d->V > 8) continue;
      if (k > 4 && n_out > kMaxOutNarrow) continue;  // many outputs: 4 points per lane only
      for (int bw : {1, 2, 4}) cands.push_back(tgp_cfg{TGP_MODE_TREE_MAJOR, bw, k, 1, 0});
      for (int tpu : {1, 4, 16, 64})
        cands.push_back(tgp_cfg{TGP_MODE_POINT_MAJOR, 4, k, tpu, 0});
      for (int bw : {1, 4})
        for (int tpu : {1, 2, 4}) cands.push_back(tgp_cfg{TGP_MODE_PERSISTENT, bw, k, tpu, 0});
      cands.push_back(tgp_cfg{TGP_MODE_PERSISTENT, 4, k, 1, TGP_FLAG_STATIC_ORDER});
    }
  }
  tgp_cfg best{};
  float best_ms = 1e30f;
  tgp_status st = TGP_OK;
  for (const tgp_cfg& c : cands) {
    // warm-up, then the median of three timed runs
    st = run(c);
    if (st != TGP_OK) break;
    float t[3];
    for (int r = 0; r < 3; ++r) {
      hipEventRecord(e0, s);
      run(c);
      hipEventRecord(e1, s);
      if (hipEventSynchronize(e1) != hipSuccess) { st = TGP_E_HIP; break; }
      hipEventElapsedTime(&t[r], e0, e1);
    }
    if (st != TGP_OK) break;
    std::sort(t, t + 3);
    if (t[1] < best_ms) {
      best_ms = t[1];
      best = c;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(mse);
  if (gv) hipFree(gv);
  if (gx) hipFree(gx);
  if (st != TGP_OK) return st;
  {
    std::lock_guard<std::mutex> g(g_mu);
    g_cache[key_of(pop, d, n_out, grad)] = best;
  }
  *out = best;
  return TGP_OK;
}

}  // namespace tgp
