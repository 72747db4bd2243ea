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
// a run of trees; persistent waves are bound to one tile each and pull
// chunks of trees, longest length bucket first, from that tile's queue.
// A wave loads its tile of X and Y once per unit (once per life in the
// persistent schedule) and keeps it in registers.
//
// Latency: while one tree runs, the wave already has the header of the
// next one and is loading the one after; the next tree's first program
// word is requested before the current tree's reduction. These prefetches
// are vector loads (broadcast of one address), whose in-order completion
// lets them stay in flight across the interpreter's scalar-load waits;
// the persistent queue's next chunk is requested one chunk ahead.
//
// Reduction: per lane, float32 residual and square; pairwise lane sum and
// DPP wave sum in float32; one float64 partial per (tree, tile), written by
// lane 0 and summed in a fixed order by the finalize kernel.
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

// The wave's point tile: X in the interpreter registers, Y beside it.
template <int K, int NO>
struct TileY {
  float y[NO][K];
};

template <int K, int VM, int NO>
__device__ __forceinline__ void load_tile(const EvalArgs& a, Regs<K, VM, NO>& s, TileY<K, NO>& ty, int64_t p0) {
#pragma unroll
  for (int v = 0; v < VM; ++v) {
    const float* xr = a.X + (int64_t)(v < a.V ? v : 0) * a.ldx;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int64_t p = p0 + j * kWave;
      // canonical (a signaling NaN becomes quiet), as the interpreter's max/min assume
      s.X[v][j] = __builtin_canonicalizef((v < a.V && p < a.D) ? xr[p] : 0.0f);
    }
  }
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    const float* yr = a.Y ? a.Y + (int64_t)(o < a.ny ? o : 0) * a.ldy : nullptr;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int64_t p = p0 + j * kWave;
      ty.y[o][j] = (yr && o < a.ny && p < a.D) ? yr[p] : 0.0f;
    }
  }
}

// Output o of the tree at point slot j: a tree without Modi nodes predicts
// (root, 0, ..., 0); the root value is the accumulator A.
template <int K, int VM, int NO>
__device__ __forceinline__ float out_val(const Regs<K, VM, NO>& s, bool modi, int o, int j) {
  return modi ? s.O[o][j] : (o == 0 ? s.A[j] : 0.0f);
}

// Broadcast loads: every lane reads the same address with a vector load;
// the value is taken from lane 0 when it is needed.
__device__ __forceinline__ uint32_t bcast_load_u32(const int32_t* p) { return (uint32_t)*p; }
__device__ __forceinline__ uint2 bcast_load_u64(const uint2* p) { return *p; }
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ unsigned long long uniform64(uint2 v) {
  return (unsigned long long)uniform(v.x) | ((unsigned long long)uniform(v.y) << 32);
}

// Evaluate the tree with header `hdr` on the tile whose first point for this
// lane is p0, starting from its already-loaded first program word. Between
// the program and the reduction, `between()` runs (the next prefetch).
//
// Fitness reduction (accuracy: hit counts, exact): squared residuals in float32, summed pairwise per lane
// and over the wave by DPP (all terms non-negative: relative error below
// (log2 K + 6) float32 ulp, under 6e-7). If the float32 wave sum overflows,
// the tile is summed again in float64 (terms that are themselves infinite
// give the same result). The tile's sum is stored as the (tree, tile)
// partial; the finalize kernel adds a tree's partials in float64 in a fixed
// order, so the fitness does not depend on which wave finished first.
template <int K, int VM, int NO, bool PRED, class Between>
__device__ __forceinline__ void eval_tree(const EvalArgs& a, Regs<K, VM, NO>& s, const TileY<K, NO>& ty,
                                          float* spill, uint32_t hdr, unsigned long long first, int64_t p0,
                                          int64_t tile, int lane, Between between) {
  const int64_t t = hdr & kHdrTree;
  if (hdr & kHdrInvalid) {
    between();
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
  const bool modi = (hdr & kHdrModi) != 0;
  if (modi) {
#pragma unroll
    for (int q = 0; q < NO; ++q)
#pragma unroll
      for (int j = 0; j < K; ++j) s.O[q][j] = 0.0f;
  }
  // every program starts by loading A
  run_from<K, VM, NO, false, false, true>((prog_ptr)(a.prog + t * a.pstride), first, s, spill);
  between();

  if constexpr (PRED) {
#pragma unroll
    for (int o = 0; o < NO; ++o) {
      if (o < a.n_out) {
        float* pr = a.pred + (t * a.n_out + o) * a.ldp;
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const int64_t p = p0 + j * kWave;
          if (p < a.D) pr[p] = out_val(s, modi, o, j);
        }
      }
    }
  }
  if (!a.Y) return;
  if (a.loss == kLossAccuracy) {
    // class = first index of the largest output, NaN below every number; a hit when it
    // equals the label (row 0 of Y). Counts are exact in float32.
    float hits = 0.0f;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      float best = out_val(s, modi, 0, j);
      int cls = 0;
#pragma unroll
      for (int o = 1; o < NO; ++o) {
        const float v = out_val(s, modi, o, j);
        if (o < a.n_out && (v > best || (best != best && v == v))) {
          best = v;
          cls = o;
        }
      }
      const int64_t p = p0 + j * kWave;
      hits += (p < a.D && (float)cls == ty.y[0][j]) ? 1.0f : 0.0f;
    }
    const float tot = wave_sum_f32(hits);
    if (lane == 0) a.part[tile * a.P + t] = (double)tot;
    return;
  }
  float lane_sum = 0.0f;
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    if (o < a.n_out) {
      float sq[K];
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const int64_t p = p0 + j * kWave;
        const float e = p < a.D ? out_val(s, modi, o, j) - ty.y[o][j] : 0.0f;
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
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const int64_t p = p0 + j * kWave;
          const float e = p < a.D ? out_val(s, modi, o, j) - ty.y[o][j] : 0.0f;
          l64 += (double)(e * e);
        }
      }
    }
    tot = wave_sum_f64(l64);
  }
  if (lane == 0) a.part[tile * a.P + t] = tot;
}

// Positions of the trees one wave evaluates on its tile.
//   contiguous (tree-major, point-major): trees k in [k, kend), header from
//   the tree record;
//   persistent: chunks of tpu positions of the length-sorted order. Chunk
//   numbers come round-robin in snake order (round r gives wave j of the
//   tile's n waves chunk r n + j, or r n + n - 1 - j on odd rounds, so the
//   longest chunk of each round goes to a different end and every wave's
//   total is within about one chunk of the others) or, dynamic, from the
//   tile's counter, with the pop for the chunk after the current one
//   always in flight. A tile's chunks are split over nsub interleaved
//   sub-queues so that no counter is shared by too many waves.
struct Cursor {
  int64_t k, kend, P;
  int tpu;
  int round, j, n;    // round-robin: round, wave in tile, waves per tile (n = 0: no further chunks)
  int32_t* q;         // dynamic: this wave's sub-queue counter
  int sub, nsub;      // dynamic: sub-queue s of a tile hands out chunks s, s + nsub, ...
  int pending;        // dynamic, lane 0: result of the in-flight pop

  __device__ __forceinline__ int pop_issue(int lane) const {
    int r = 0;
    if (lane == 0) r = atomicAdd(q, 1);
    return r;
  }
  __device__ __forceinline__ void enter(int64_t c) {
    k = c * tpu;
    kend = min(P, k + tpu);
    if (k >= P) k = P;
  }
  __device__ __forceinline__ int64_t snake() const {
    return (int64_t)round * n + ((round & 1) ? n - 1 - j : j);
  }
  // next position, or P when there is none
  __device__ __forceinline__ int64_t next(int lane) {
    if (k + 1 < kend) return ++k;
    if (q) {
      const int c = (int)uniform((uint32_t)__shfl(pending, 0, kWave));
      pending = pop_issue(lane);
      enter((int64_t)c * nsub + sub);
    } else if (n > 0) {
      ++round;
      enter(snake());
    } else {
      k = P;
    }
    return k;
  }
};

}  // namespace

template <int K, int VM, int NO, bool PRED>
__global__ __launch_bounds__(256) void eval_kernel(EvalArgs a) {
  // per wave: LDS spill slots 4..7
  extern __shared__ float s_lds[];
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
  const int W = blockDim.x / kWave;
  float* spill = s_lds + wv * (kLdsFloatsPerWave<K>) + lane;
  Regs<K, VM, NO> s;
  TileY<K, NO> ty;
  constexpr int kTile = K * kWave;
  const bool persistent = a.mode == TGP_MODE_PERSISTENT;

  // ---- this wave's tile and first position ----
  int tile;
  Cursor cur;
  cur.P = a.P;
  cur.tpu = a.tpu;
  cur.pending = 0;
  cur.q = nullptr;
  cur.n = 0;
  if (persistent) {
    const int64_t gw = (int64_t)blockIdx.x * W + wv;
    if (gw >= (int64_t)a.ntiles * a.wpt) return;
    tile = (int)(gw % a.ntiles);
    if (a.dynamic) {
      cur.nsub = a.nsub;
      cur.sub = (int)((gw / a.ntiles) % a.nsub);
      cur.q = a.queue + ((int64_t)tile * a.nsub + cur.sub) * kQueueStride;
      const int c0 = (int)uniform((uint32_t)__shfl(cur.pop_issue(lane), 0, kWave));
      cur.pending = cur.pop_issue(lane);
      cur.enter((int64_t)c0 * cur.nsub + cur.sub);
    } else {
      cur.n = a.wpt;
      cur.j = (int)(gw / a.ntiles);
      cur.round = 0;
      cur.enter(cur.snake());
    }
    if (cur.k >= a.P) return;
  } else {
    const int64_t b = blockIdx.x;
    const int g = (int)(b % a.ngroups);
    tile = g * W + wv;
    if (tile >= a.ntiles) return;
    cur.enter(b / a.ngroups);
    if (cur.k >= a.P) return;
  }
  const int64_t p0 = (int64_t)tile * kTile + lane;
  load_tile<K, VM, NO>(a, s, ty, p0);

  // header of position k: the order entry (queue mode) or the tree record
  auto hdr_ptr = [&](int64_t k) -> const int32_t* {
    return persistent ? a.order + k : a.info + k * kInfoStride + kInfoHdr;
  };
  auto first_ptr = [&](uint32_t hdr) -> const uint2* {
    return a.prog + (int64_t)(hdr & kHdrTree) * a.pstride;
  };

  // pipeline: header of position k1 and first word of its tree are being
  // loaded (vh1, vf1); header of position k2 is being loaded (vh2)
  uint32_t hdr = uniform(bcast_load_u32(hdr_ptr(cur.k)));
  unsigned long long first = 0;
  if (!(hdr & kHdrInvalid)) first = uniform64(bcast_load_u64(first_ptr(hdr)));
  int64_t k1 = cur.next(lane);
  uint32_t vh1 = k1 < a.P ? bcast_load_u32(hdr_ptr(k1)) : kHdrInvalid;
  for (;;) {
    const int64_t k2 = k1 < a.P ? cur.next(lane) : a.P;
    const uint32_t vh2 = k2 < a.P ? bcast_load_u32(hdr_ptr(k2)) : kHdrInvalid;
    uint32_t h1 = kHdrInvalid;
    uint2 vf1 = make_uint2(0u, 0u);
    auto between = [&]() {
      // the next tree's header has arrived by now; request its first word
      h1 = k1 < a.P ? uniform(vh1) : kHdrInvalid;
      if (!(h1 & kHdrInvalid)) vf1 = bcast_load_u64(first_ptr(h1));
    };
    eval_tree<K, VM, NO, PRED>(a, s, ty, spill, hdr, first, p0, tile, lane, between);
    if (k1 >= a.P) break;
    hdr = h1;
    first = (h1 & kHdrInvalid) ? 0ull : uniform64(vf1);
    k1 = k2;
    vh1 = vh2;
  }
}

template <int K, int VM, int NO, bool PRED>
inline hipError_t launch_eval_t(const EvalArgs& a, int block_waves, int64_t grid, hipStream_t s) {
  const size_t lds = (size_t)block_waves * kLdsFloatsPerWave<K> * sizeof(float);
  eval_kernel<K, VM, NO, PRED><<<dim3((unsigned)grid), dim3(block_waves * kWave), lds, s>>>(a);
  return hipGetLastError();
}

// Workgroups of block_waves waves that one CU holds at once for this instantiation
// (registers, LDS and the launch bound), or 0 when the runtime cannot say.
template <int K, int VM, int NO, bool PRED>
inline int occupancy_eval_t(int block_waves) {
  const size_t lds = (size_t)block_waves * kLdsFloatsPerWave<K> * sizeof(float);
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, eval_kernel<K, VM, NO, PRED>, block_waves * kWave, lds) !=
      hipSuccess)
    return 0;
  return n;
}

template <int K, int VM, int NO>
inline hipError_t launch_eval_kvo(const EvalArgs& a, bool pred, int bw, int64_t grid, hipStream_t s) {
  return pred ? launch_eval_t<K, VM, NO, true>(a, bw, grid, s) : launch_eval_t<K, VM, NO, false>(a, bw, grid, s);
}

template <int K, int VM, int NO>
inline int occupancy_eval_kvo(bool pred, int bw) {
  return pred ? occupancy_eval_t<K, VM, NO, true>(bw) : occupancy_eval_t<K, VM, NO, false>(bw);
}

// The output accumulators are instantiated for exactly n_out outputs (1..4), so a
// three-output population carries three accumulators, not four. Populations of 5 to
// kMaxOut outputs (classification with many classes) run at 4 points per lane with
// kMaxOut accumulators.
template <int K, int VM>
hipError_t launch_eval_kv(const EvalArgs& a, int NO, bool pred, int bw, int64_t grid, hipStream_t s) {
  switch (NO) {
    case 1: return launch_eval_kvo<K, VM, 1>(a, pred, bw, grid, s);
    case 2: return launch_eval_kvo<K, VM, 2>(a, pred, bw, grid, s);
    case 3: return launch_eval_kvo<K, VM, 3>(a, pred, bw, grid, s);
    case 4: return launch_eval_kvo<K, VM, 4>(a, pred, bw, grid, s);
    default:
      if constexpr (K == 4) return launch_eval_kvo<K, VM, kMaxOut>(a, pred, bw, grid, s);
      return hipErrorInvalidValue;
  }
}

template <int K, int VM>
int occupancy_eval_kv(int NO, bool pred, int bw) {
  switch (NO) {
    case 1: return occupancy_eval_kvo<K, VM, 1>(pred, bw);
    case 2: return occupancy_eval_kvo<K, VM, 2>(pred, bw);
    case 3: return occupancy_eval_kvo<K, VM, 3>(pred, bw);
    case 4: return occupancy_eval_kvo<K, VM, 4>(pred, bw);
    default:
      if constexpr (K == 4) return occupancy_eval_kvo<K, VM, kMaxOut>(pred, bw);
      return 0;
  }
}

}  // namespace tgp
