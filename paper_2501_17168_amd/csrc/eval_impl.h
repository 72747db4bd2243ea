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

#include "tgp_kernels.h"

namespace tgp {

namespace {

constexpr int kWave = 64;

template <int K>
constexpr int kLdsFloatsPerWave = (kMaxSlots - kRegSlots) * K * kWave;

template <int K, int VM, int NO>
struct Regs {
  float A[K];
  float T[K];
  float r[K];
  float R[kRegSlots][K];
  float X[VM][K];
  float O[NO][K];
};

template <int B>
__device__ __forceinline__ float bin_op(float a, float b) {
  if constexpr (B == 0) return a + b;
  else if constexpr (B == 1) return a - b;
  else if constexpr (B == 2) return a * b;
  else if constexpr (B == 3) return fabsf(b) < kDivTau ? 1.0f : a / b;
  else if constexpr (B == 4) return fmaxf(a, b);
  else return fminf(a, b);
}

template <int U>
__device__ __forceinline__ float un_op(float a) {
  if constexpr (U == 0) return sinf(a);
  else if constexpr (U == 1) return cosf(a);
  else if constexpr (U == 2) return tanhf(a);
  else if constexpr (U == 3) {
    const float c = a > kExpClamp ? kExpClamp : (a < -kExpClamp ? -kExpClamp : a);
    return expf(c);
  } else if constexpr (U == 4) return logf(fabsf(a) + kLogEps);
  else return tanf(a);
}

// value of source S for point slot j
template <int S, int K, int VM, int NO>
__device__ __forceinline__ float src_val(const Regs<K, VM, NO>& s, int j, float cv, const float* spill, int aux) {
  if constexpr (S == kSrcC) return cv;
  else if constexpr (S < kSrcRM) return s.R[S - kSrcR0][j];
  else if constexpr (S == kSrcRM) return spill[((aux & (kMaxSlots - 1)) - kRegSlots) * (K * kWave) + j * kWave];
  else return s.X[(S - kSrcX0) < VM ? (S - kSrcX0) : 0][j];
}

template <int K, int VM, int NO>
__device__ __forceinline__ void add_out(Regs<K, VM, NO>& s, int o) {
  // selects rather than branches, so every register index stays static
#pragma unroll
  for (int q = 0; q < NO; ++q) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const float sum = s.O[q][j] + s.r[j];
      s.O[q][j] = (q == o) ? sum : s.O[q][j];
    }
  }
}

// program words live in device memory that no kernel writes while it is
// being interpreted; the constant address space lets the compiler read them
// with scalar loads
typedef const __attribute__((address_space(4))) unsigned long long* prog_ptr;

// Interpret one program on this lane's K points. `spill` points at this
// wave's LDS spill area [kMaxSlots - kRegSlots][K][64], offset by the lane.
// The next instruction word is fetched while the current one executes; the
// empty asm statements pin where the compiler waits for that scalar load
// (at the end of the iteration, not right after issuing it).
template <int K, int VM, int NO>
__device__ __forceinline__ void run_program(prog_ptr prog, Regs<K, VM, NO>& s, float* spill) {
  unsigned long long ins = prog[0];
  asm volatile("" : "+s"(ins));
  // one exit (after the latch), so the loop is a single-entry single-exit
  // region made only of uniform branches
  bool done = false;
  for (;;) {
    ++prog;
    const unsigned long long nxt = prog[0];
    const uint32_t w = (uint32_t)ins;
    const float cv = __uint_as_float((uint32_t)(ins >> 32));
    const int c = (int)(w & 0xffffu);
    const int aux = (int)(w >> 16);
    int un = -1;

#define TGP_SRC_CASE(BASE, S, STMT)                                   \
  case (BASE) + (S): {                                                \
    if constexpr ((S) < kSrcX0 || (S) - kSrcX0 < VM) {                \
      _Pragma("unroll") for (int j = 0; j < K; ++j) {                 \
        const float v = src_val<(S), K, VM, NO>(s, j, cv, spill, aux); \
        STMT;                                                         \
      }                                                               \
    }                                                                 \
  } break;
#define TGP_SRC_CASES(BASE, STMT)                                                             \
  TGP_SRC_CASE(BASE, 0, STMT) TGP_SRC_CASE(BASE, 1, STMT) TGP_SRC_CASE(BASE, 2, STMT)       \
  TGP_SRC_CASE(BASE, 3, STMT) TGP_SRC_CASE(BASE, 4, STMT) TGP_SRC_CASE(BASE, 5, STMT)       \
  TGP_SRC_CASE(BASE, 6, STMT) TGP_SRC_CASE(BASE, 7, STMT) TGP_SRC_CASE(BASE, 8, STMT)       \
  TGP_SRC_CASE(BASE, 9, STMT) TGP_SRC_CASE(BASE, 10, STMT) TGP_SRC_CASE(BASE, 11, STMT)     \
  TGP_SRC_CASE(BASE, 12, STMT) TGP_SRC_CASE(BASE, 13, STMT) TGP_SRC_CASE(BASE, 14, STMT)    \
  TGP_SRC_CASE(BASE, 15, STMT) TGP_SRC_CASE(BASE, 16, STMT) TGP_SRC_CASE(BASE, 17, STMT)    \
  TGP_SRC_CASE(BASE, 18, STMT) TGP_SRC_CASE(BASE, 19, STMT) TGP_SRC_CASE(BASE, 20, STMT)    \
  TGP_SRC_CASE(BASE, 21, STMT)

#define TGP_BT_CASE(B)                                                                      \
  case kBT + 2 * (B):                                                                       \
    _Pragma("unroll") for (int j = 0; j < K; ++j) s.A[j] = bin_op<(B)>(s.A[j], s.T[j]);     \
    break;                                                                                  \
  case kBT + 2 * (B) + 1:                                                                   \
    _Pragma("unroll") for (int j = 0; j < K; ++j) s.A[j] = bin_op<(B)>(s.T[j], s.A[j]);     \
    break;                                                                                  \
  case kMB + 2 * (B):                                                                       \
    _Pragma("unroll") for (int j = 0; j < K; ++j) {                                         \
      s.r[j] = bin_op<(B)>(s.A[j], s.T[j]);                                                 \
      s.A[j] = s.T[j];                                                                      \
    }                                                                                       \
    break;                                                                                  \
  case kMB + 2 * (B) + 1:                                                                   \
    _Pragma("unroll") for (int j = 0; j < K; ++j) s.r[j] = bin_op<(B)>(s.T[j], s.A[j]);     \
    break;

// Unary (transcendental) cases only record which function to apply: the
// library implementations branch per lane, and keeping those divergent
// branches out of the dispatch switch keeps the switch a purely scalar
// branch tree (no per-lane flow merges that copy the register state).
#define TGP_UN_CASE(U)     \
  case kUN + (U):          \
    un = (U);              \
    break;                 \
  case kMU + (U):          \
    un = (U) | 8;          \
    break;

    switch (c) {
      TGP_SRC_CASES(kLD, s.A[j] = v)
      TGP_SRC_CASES(kTLD, s.T[j] = v)
      TGP_SRC_CASES(kADD, s.A[j] = s.A[j] + v)
      TGP_SRC_CASES(kMUL, s.A[j] = s.A[j] * v)
      TGP_SRC_CASES(kMAX, s.A[j] = fmaxf(s.A[j], v))
      TGP_SRC_CASES(kMIN, s.A[j] = fminf(s.A[j], v))
      TGP_SRC_CASES(kSUBA, s.A[j] = s.A[j] - v)
      TGP_SRC_CASES(kSUBR, s.A[j] = v - s.A[j])
      case kSPL + 0:
#pragma unroll
        for (int j = 0; j < K; ++j) s.R[0][j] = s.A[j];
        break;
      case kSPL + 1:
#pragma unroll
        for (int j = 0; j < K; ++j) s.R[1][j] = s.A[j];
        break;
      case kSPL + 2:
#pragma unroll
        for (int j = 0; j < K; ++j) s.R[2][j] = s.A[j];
        break;
      case kSPL + 3:
#pragma unroll
        for (int j = 0; j < K; ++j) s.R[3][j] = s.A[j];
        break;
      case kSPLM: {
        float* dst = spill + ((aux & (kMaxSlots - 1)) - kRegSlots) * (K * kWave);
#pragma unroll
        for (int j = 0; j < K; ++j) dst[j * kWave] = s.A[j];
      } break;
      case kTA:
#pragma unroll
        for (int j = 0; j < K; ++j) s.T[j] = s.A[j];
        break;
      TGP_BT_CASE(0)
      TGP_BT_CASE(1)
      TGP_BT_CASE(2)
      TGP_BT_CASE(3)
      TGP_BT_CASE(4)
      TGP_BT_CASE(5)
      TGP_UN_CASE(0)
      TGP_UN_CASE(1)
      TGP_UN_CASE(2)
      TGP_UN_CASE(3)
      TGP_UN_CASE(4)
      TGP_UN_CASE(5)
      case kACC:
        add_out<K, VM, NO>(s, aux);
        break;
      default:  // kEND (or any word that is not an instruction)
        done = true;
        break;
    }
#undef TGP_SRC_CASE
#undef TGP_SRC_CASES
#undef TGP_BT_CASE
#undef TGP_UN_CASE
    if (un >= 0) {
      float t[K];
      switch (un & 7) {
        case 0:
#pragma unroll
          for (int j = 0; j < K; ++j) t[j] = un_op<0>(s.A[j]);
          break;
        case 1:
#pragma unroll
          for (int j = 0; j < K; ++j) t[j] = un_op<1>(s.A[j]);
          break;
        case 2:
#pragma unroll
          for (int j = 0; j < K; ++j) t[j] = un_op<2>(s.A[j]);
          break;
        case 3:
#pragma unroll
          for (int j = 0; j < K; ++j) t[j] = un_op<3>(s.A[j]);
          break;
        case 4:
#pragma unroll
          for (int j = 0; j < K; ++j) t[j] = un_op<4>(s.A[j]);
          break;
        default:
#pragma unroll
          for (int j = 0; j < K; ++j) t[j] = un_op<5>(s.A[j]);
          break;
      }
      if (un & 8) {
#pragma unroll
        for (int j = 0; j < K; ++j) s.r[j] = t[j];
      } else {
#pragma unroll
        for (int j = 0; j < K; ++j) s.A[j] = t[j];
      }
    }
    unsigned long long n2 = nxt;
    asm volatile("" : "+s"(n2));
    ins = n2;
    if (done) break;
  }
}

__device__ __forceinline__ double wave_sum_f64(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
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

// Evaluate tree t on the tile whose first point for this lane is p0.
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
#pragma unroll
  for (int q = 0; q < NO; ++q)
#pragma unroll
    for (int j = 0; j < K; ++j) s.O[q][j] = 0.0f;
#pragma unroll
  for (int j = 0; j < K; ++j) s.A[j] = 0.0f;
  run_program<K, VM, NO>((prog_ptr)(a.prog + t * a.pstride), s, spill);
  // outputs: a tree without Modi nodes predicts (root, 0, ..., 0)
  if (nmodi == 0) {
#pragma unroll
    for (int j = 0; j < K; ++j) s.O[0][j] = s.A[j];
  }

  double sse = 0.0;
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    if (o < a.n_out) {
      if constexpr (PRED) {
        float* pr = a.pred + (t * a.n_out + o) * a.ldp;
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const int64_t p = p0 + j * kWave;
          if (p < a.D) pr[p] = s.O[o][j];
        }
      }
      if (a.Y) {
        const float* yr = a.Y + (int64_t)o * a.ldy;
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const int64_t p = p0 + j * kWave;
          if (p < a.D) {
            const float e = s.O[o][j] - yr[p];
            sse += (double)(e * e);
          }
        }
      }
    }
  }
  if (a.Y) {
    sse = wave_sum_f64(sse);
    if (lane == 0) unsafeAtomicAdd(&a.acc[t], sse);
  }
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
      int u = 0;
      if (lane == 0) u = atomicAdd(a.queue, 1);
      u = __builtin_amdgcn_readfirstlane(__shfl(u, 0, kWave));
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
