#pragma once
// Forward evaluation: run every tree's program on every data point, then
// reduce the squared errors to one fitness per tree (§III-C), or write the
// per-point predictions (multi-output inference, §IV-C).
//
// Mapping (gfx950, wave64). A wave owns a point tile of 64*K points, K per
// lane: lane l holds points tile*64K + j*64 + l, j < K, so every load of X,
// Y and every prediction store is a coalesced 256-byte row. All lanes of a
// wave run the same tree, so the program counter, the dispatch and every
// operand index are wave-uniform: the program is read with scalar loads
// (the counterpart of the paper's constant-memory broadcast of a tree) and
// dispatched with scalar branches, while the vector ALUs only do the node
// arithmetic on K points per lane.
//
// Work units: tree-major gives each workgroup one tree and block_waves
// consecutive tiles; point-major gives each workgroup block_waves tiles and
// a run of trees, loading the X tile once; persistent waves pull
// (tree chunk, tile) units from a counter, with trees ordered longest
// length bucket first.
//
// Reduction: per lane, float32 residual and square, float64 sum over its K
// points; float64 wave reduction; one float64 atomic per (wave, tree).
#include <hip/hip_runtime.h>
#include <math.h>

#include "interp.h"
#include "tgp_kernels.h"

namespace tgp {

namespace {

using namespace interp;

// Sum of this lane's K squared residuals, pairwise in float32 (all terms
// are non-negative, so the relative error is below log2(K) ulp).
template <int K>
__device__ __forceinline__ float lane_sum_sq(const float (&sq)[K]) {
  float t[K];
#pragma unroll
  for (int j = 0; j < K; ++j) t[j] = sq[j];
#pragma unroll
  for (int w = K / 2; w >= 1; w /= 2)
#pragma unroll
    for (int j = 0; j < w; ++j) t[j] += t[j + w];
  return t[0];
}

template <int K, int VM, int NO>
__device__ __forceinline__ void load_x(const EvalArgs& a, Regs<K, VM, NO>& s, int64_t p0) {
#pragma unroll
  for (int v = 0; v < VM; ++v) {
    if (v < a.V) {
      const float* xr = a.X + (int64_t)v * a.ldx;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const int64_t p = p0 + j * kWave;
        s.X[v][j] = p < a.D ? xr[p] : 0.0f;
      }
    } else {
#pragma unroll
      for (int j = 0; j < K; ++j) s.X[v][j] = 0.0f;
    }
  }
}

// Output o of the tree at point slot j: a tree without Modi nodes predicts
// (root, 0, ..., 0); the root value is the accumulator A.
template <int K, int VM, int NO>
__device__ __forceinline__ float out_val(const Regs<K, VM, NO>& s, int nmodi, int o, int j) {
  return nmodi ? s.O[o][j] : (o == 0 ? s.A[j] : 0.0f);
}

// Evaluate tree t on the tile whose first point for this lane is p0.
//
// Fitness reduction: squared residuals in float32, summed pairwise per lane
// and over the wave by DPP (all terms non-negative: relative error below
// (log2 K + 6) float32 ulp, under 6e-7), then added in float64 across
// waves. If the float32 wave sum overflows, the tile is summed again in
// float64 (terms that are themselves infinite give the same result).
template <int K, int VM, int NO, bool PRED>
__device__ __forceinline__ void eval_tree(const EvalArgs& a, Regs<K, VM, NO>& s, float* spill, int64_t t,
                                          int64_t p0, int lane) {
  const int32_t* inf = a.info + t * kInfoStride;
  const int status = __builtin_amdgcn_readfirstlane(inf[kInfoStatus]);
  if (status != 0) {
    if constexpr (PRED) {
      for (int o = 0; o < a.n_out; ++o) {
        float* pr = a.pred + (t * a.n_out + o) * a.ldp;
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const int64_t p = p0 + j * kWave;
          if (p < a.D) pr[p] = __builtin_nanf("");
        }
      }
    }
    return;
  }
  const int nmodi = __builtin_amdgcn_readfirstlane(inf[kInfoNModi]);
  if (nmodi) {
#pragma unroll
    for (int q = 0; q < NO; ++q)
#pragma unroll
      for (int j = 0; j < K; ++j) s.O[q][j] = 0.0f;
  }
  // every program starts by loading A
  run_program<K, VM, NO>((prog_ptr)(a.prog + t * a.pstride), s, spill);

  if constexpr (PRED) {
#pragma unroll
    for (int o = 0; o < NO; ++o) {
      if (o < a.n_out) {
        float* pr = a.pred + (t * a.n_out + o) * a.ldp;
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const int64_t p = p0 + j * kWave;
          if (p < a.D) pr[p] = out_val(s, nmodi, o, j);
        }
      }
    }
  }
  if (!a.Y) return;
  float lane_sum = 0.0f;
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    if (o < a.n_out) {
      const float* yr = a.Y + (int64_t)o * a.ldy;
      float sq[K];
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const int64_t p = p0 + j * kWave;
        const float e = p < a.D ? out_val(s, nmodi, o, j) - yr[p] : 0.0f;
        sq[j] = e * e;
      }
      lane_sum += lane_sum_sq<K>(sq);
    }
  }
  const float tot32 = wave_sum_f32(lane_sum);
  double tot = (double)tot32;
  if (__builtin_isinf(tot32)) {
    double l64 = 0.0;
#pragma unroll
    for (int o = 0; o < NO; ++o) {
      if (o < a.n_out) {
        const float* yr = a.Y + (int64_t)o * a.ldy;
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const int64_t p = p0 + j * kWave;
          const float e = p < a.D ? out_val(s, nmodi, o, j) - yr[p] : 0.0f;
          l64 += (double)(e * e);
        }
      }
    }
    tot = wave_sum_f64(l64);
  }
  if (lane == 0) unsafeAtomicAdd(&a.acc[t], tot);
}

}  // namespace

template <int K, int VM, int NO, bool PRED>
__global__ __launch_bounds__(256) void eval_kernel(EvalArgs a) {
  // per wave: LDS spill slots 4..7
  extern __shared__ float s_lds[];
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  const int W = blockDim.x / kWave;
  float* spill = s_lds + wv * (kLdsFloatsPerWave<K>) + lane;
  Regs<K, VM, NO> s;
  constexpr int kTile = K * kWave;
  const bool persistent = a.mode == TGP_MODE_PERSISTENT;

  int cur_tile = -1;
  for (int iter = 0;; ++iter) {
    // ---- next work unit: a point tile and a run [t0, t1) of tree slots ----
    int tile;
    int64_t t0, t1;
    if (persistent) {
      // queue j hands out units j, j + nq, j + 2 nq, ... in order (longest trees first)
      const int j = (int)(blockIdx.x % (unsigned)a.nq);
      int k = 0;
      if (lane == 0) k = atomicAdd(a.queue + j * kQueueStride, 1);
      k = __builtin_amdgcn_readfirstlane(__shfl(k, 0, kWave));
      const int64_t u = (int64_t)j + (int64_t)a.nq * k;
      if (u >= a.n_units) break;
      tile = (int)(u % a.ntiles);
      t0 = (int64_t)(u / a.ntiles) * a.tpu;
      t1 = min(a.P, t0 + a.tpu);
    } else {
      if (iter > 0) break;
      const int64_t b = blockIdx.x;
      const int g = (int)(b % a.ngroups);
      tile = g * W + wv;
      t0 = (b / a.ngroups) * a.tpu;
      t1 = min(a.P, t0 + a.tpu);
      if (tile >= a.ntiles) break;
    }
    const int64_t p0 = (int64_t)tile * kTile + lane;
    if (tile != cur_tile) {
      load_x<K, VM, NO>(a, s, p0);
      cur_tile = tile;
    }
    for (int64_t k = t0; k < t1; ++k) {
      const int64_t t = persistent ? (int64_t)__builtin_amdgcn_readfirstlane(a.order[k]) : k;
      if (t < 0 || t >= a.P) continue;
      eval_tree<K, VM, NO, PRED>(a, s, spill, t, p0, lane);
    }
  }
}

template <int K, int VM, int NO, bool PRED>
inline hipError_t launch_eval_t(const EvalArgs& a, int block_waves, int64_t grid, hipStream_t s) {
  const size_t lds = (size_t)block_waves * kLdsFloatsPerWave<K> * sizeof(float);
  eval_kernel<K, VM, NO, PRED><<<dim3((unsigned)grid), dim3(block_waves * kWave), lds, s>>>(a);
  return hipGetLastError();
}

template <int K, int VM>
hipError_t launch_eval_kv(const EvalArgs& a, int NO, bool pred, int bw, int64_t grid, hipStream_t s) {
  if (NO == 1) return pred ? launch_eval_t<K, VM, 1, true>(a, bw, grid, s) : launch_eval_t<K, VM, 1, false>(a, bw, grid, s);
  return pred ? launch_eval_t<K, VM, kMaxOut, true>(a, bw, grid, s) : launch_eval_t<K, VM, kMaxOut, false>(a, bw, grid, s);
}

}  // namespace tgp
