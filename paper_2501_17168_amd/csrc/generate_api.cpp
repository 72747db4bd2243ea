// C-ABI entry of random tree generation: host-side checks, then one launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "tgp.h"
#include "tgp_generate.h"

using namespace tgp;

extern "C" {

__attribute__((visibility("default"))) tgp_status tgp_generate(const tgp_gen_cfg* g, int64_t P, int32_t Lmax,
                                                               float* out_type, float* out_value,
                                                               float* out_size, int64_t out_stride,
                                                               int32_t* attempts, hipStream_t stream) {
  if (!g) return TGP_E_ARG;
  if (P < 0 || Lmax < 1 || out_stride < Lmax) return TGP_E_SHAPE;
  if (Lmax > 1024 || P > INT32_MAX) return TGP_E_UNSUPPORTED;
  if (g->method < TGP_GEN_GROW || g->method > TGP_GEN_RAMPED) return TGP_E_ARG;
  if (g->depth_min < 0 || g->depth_max < g->depth_min) return TGP_E_ARG;
  if (g->depth_max > kMaxGenDepth) return TGP_E_UNSUPPORTED;
  if (g->V < 1 || g->V > 16) return TGP_E_ARG;
  if (!g->funcs || g->n_funcs < 1 || g->n_funcs > 12) return TGP_E_ARG;
  if (!std::isfinite(g->const_lo) || !std::isfinite(g->const_hi) || !(g->const_lo < g->const_hi))
    return TGP_E_ARG;
  if (g->attempts_per_depth < 1) return TGP_E_ARG;
  if (g->first_tree < 0 || g->first_tree + P > (int64_t)1 << 32) return TGP_E_ARG;
  if (!(g->p_func <= 1.0f) || !(g->p_const <= 1.0f)) return TGP_E_ARG;  // also rejects NaN
  GenArgs a{};
  for (int f = 0; f < g->n_funcs; ++f) {
    if (g->funcs[f] < 0 || g->funcs[f] > 11) return TGP_E_ARG;
    for (int e = 0; e < f; ++e)
      if (g->funcs[e] == g->funcs[f]) return TGP_E_ARG;
    a.funcs[f] = g->funcs[f];
  }
  if (P == 0) return TGP_OK;
  if (!out_type || !out_value || !out_size) return TGP_E_ARG;
  a.P = P;
  a.first_tree = g->first_tree;
  a.Lmax = Lmax;
  a.V = g->V;
  a.method = g->method;
  a.d_min = g->depth_min;
  a.d_max = g->depth_max;
  a.n_funcs = g->n_funcs;
  a.lo = g->const_lo;
  a.hi = g->const_hi;
  a.p_func = g->p_func >= 0.0f ? g->p_func : (float)g->n_funcs / (float)(g->n_funcs + g->V + 1);
  a.p_const = g->p_const >= 0.0f ? g->p_const : 1.0f / (float)(g->V + 1);
  a.attempts_per_depth = g->attempts_per_depth;
  a.key0 = (uint32_t)(g->seed & 0xFFFFFFFFu);
  a.key1 = (uint32_t)(g->seed >> 32);
  a.out_t = out_type;
  a.out_v = out_value;
  a.out_s = out_size;
  a.out_ld = out_stride;
  a.attempts = attempts;
  return launch_generate(a, stream) == hipSuccess ? TGP_OK : TGP_E_HIP;
}

}  // extern "C"
