#pragma once
// The wave-uniform interpreter shared by the forward and adjoint kernels:
// per-lane register state, operator semantics and the dispatch loop over a
// compiled program (instruction set in tgp_isa.h).
#include <hip/hip_runtime.h>
#include <math.h>

#include "ops.h"
#include "tgp_kernels.h"

namespace tgp {
namespace interp {

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

// max / min of canonical values. Every value the interpreter holds is the
// result of an IEEE operation, a finite constant or a canonicalized X load,
// so no operand is a signaling NaN; the hardware max/min then already has
// fmax/fmin semantics (a quiet NaN operand is ignored) and the compiler's
// per-operand canonicalization (two extra instructions per point) is not
// needed.
__device__ __forceinline__ float vmax(float a, float b) {
  float r;
  asm("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ float vmin(float a, float b) {
  float r;
  asm("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

template <int B>
__device__ __forceinline__ float bin_op(float a, float b) {
  if constexpr (B == 0) return a + b;
  else if constexpr (B == 1) return a - b;
  else if constexpr (B == 2) return a * b;
  else if constexpr (B == 3) return fabsf(b) < kDivTau ? 1.0f : a / b;
  else if constexpr (B == 4) return vmax(a, b);
  else return vmin(a, b);
}

template <int U>
__device__ __forceinline__ float un_op(float a) {
  if constexpr (U == 0) return sinf(a);
  else if constexpr (U == 1) return cosf(a);
  else if constexpr (U == 2) return tanhf(a);
  else if constexpr (U == 3) return exp_clamped(a);
  else if constexpr (U == 4) return log_positive(fabsf(a) + kLogEps);
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
  if constexpr (NO <= kMaxOutNarrow) {
    // selects rather than branches, so every register index stays static
#pragma unroll
    for (int q = 0; q < NO; ++q) {
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const float sum = s.O[q][j] + s.r[j];
        s.O[q][j] = (q == o) ? sum : s.O[q][j];
      }
    }
  } else {
    // many outputs: branch on the (wave-uniform) index, K adds instead of NO x K selects.
    // The empty asm names the output, so the branches are not merged into one block with
    // a computed register index (which would move the accumulators to scratch).
#pragma unroll
    for (int q = 0; q < NO; ++q) {
      if (q == o) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
          s.O[q][j] += s.r[j];
          asm volatile("; output %1 point %2" : "+v"(s.O[q][j]) : "n"(q), "n"(j));
        }
      }
    }
  }
}

// program words live in device memory that no kernel writes while it is
// being interpreted; the constant address space lets the compiler read them
// with scalar loads
typedef const __attribute__((address_space(4))) unsigned long long* prog_ptr;

// One action: v = f(A) for the unary function in bits 0..2 of `un`; a Modi
// node's value goes to r while A keeps the child value it hands up, any
// other node's replaces A. Unary (transcendental) functions run here, after
// the dispatch switch: the library implementations branch per lane, and
// keeping those divergent branches out of the switch keeps the switch a
// purely scalar branch tree (no per-lane flow merges that copy the register
// state). The empty asm on the rare Modi side keeps the compiler from
// flattening the two sides into 2K per-lane selects on every action (that
// measured 3% slower on the batched workload; applying f to A in place with a
// saved copy for Modi measured slower still, at more registers).
template <int K, int VM, int NO>
__device__ __forceinline__ void apply_unary(Regs<K, VM, NO>& s, int un) {
  float v[K];
#pragma unroll
  for (int j = 0; j < K; ++j) v[j] = s.A[j];
  switch (un & 7) {
    case 0:
#pragma unroll
      for (int j = 0; j < K; ++j) v[j] = un_op<0>(v[j]);
      break;
    case 1:
#pragma unroll
      for (int j = 0; j < K; ++j) v[j] = un_op<1>(v[j]);
      break;
    case 2:
#pragma unroll
      for (int j = 0; j < K; ++j) v[j] = un_op<2>(v[j]);
      break;
    case 3:
#pragma unroll
      for (int j = 0; j < K; ++j) v[j] = un_op<3>(v[j]);
      break;
    case 4:
#pragma unroll
      for (int j = 0; j < K; ++j) v[j] = un_op<4>(v[j]);
      break;
    default:
#pragma unroll
      for (int j = 0; j < K; ++j) v[j] = un_op<5>(v[j]);
      break;
  }
  if (un & kActModi) {
    asm volatile("");
#pragma unroll
    for (int j = 0; j < K; ++j) s.r[j] = v[j];
  } else {
#pragma unroll
    for (int j = 0; j < K; ++j) s.A[j] = v[j];
  }
}

// Interpret one program on this lane's K points. `spill` points at this
// wave's LDS spill area [kMaxSlots - kRegSlots][K][64], offset by the lane.
// The next instruction word is fetched while the current one executes; the
// empty asm statements pin where the compiler waits for that scalar load
// (at the end of the iteration, not right after issuing it).
// With BOUNDED, exactly `count` instructions run (a subtree's code range,
// which has no END of its own); otherwise the program runs up to the word
// that carries the stop action (its last) or an END.
// DUAL (forward programs only) applies a word's second action; gradient
// programs hold capture levels in those bits.
// run_from takes the first instruction word already loaded (`first`, equal
// to prog[0]); run_program loads it.
// With CAPTURE (the adjoint's runs), after every word whose capture level
// (tgp_isa.h) equals `cap_level`, A is pushed on the wave's capture stack:
// value c sits at cap[c * K * 64 + j * 64] (cap offset by the lane), *csp
// counts the values, and pushes beyond cap_limit are dropped (the plan sizes
// every tree's sweep within the limit).
template <int K, int VM, int NO, bool BOUNDED = false, bool CAPTURE = false, bool DUAL = false>
__device__ __forceinline__ void run_from(prog_ptr prog, unsigned long long first, Regs<K, VM, NO>& s, float* spill,
                                         int count = 0, float* cap = nullptr, int* csp = nullptr, int cap_level = 0,
                                         int cap_limit = 0) {
  if (BOUNDED && count <= 0) return;
  // `first` is wave-uniform; say so, so that it can live in scalar registers
  // (the builtin returns int: widen the low half through uint32_t, or a word with bit 31 set
  // would fill the payload half with ones)
  unsigned long long ins = (unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)first) |
                           ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(first >> 32)) << 32);
  asm volatile("" : "+s"(ins));
  int left = count;
  // one exit (after the latch), so the loop is a single-entry single-exit
  // region made only of uniform branches. `act` (scalar) is 0 for the
  // common case; otherwise it carries a unary function to apply
  // (kActUn | index, kActModi for the Modi register) and/or kActStop.
  for (;;) {
    ++prog;
    const unsigned long long nxt = prog[0];
    const uint32_t w = (uint32_t)ins;
    const float cv = __uint_as_float((uint32_t)(ins >> 32));
    const int c = word_case(w);
    const int aux = (int)((w >> kAuxShift) & kAuxMask);
    int act = (int)((w >> kActShift) & 63u);

    if (w & (kSpillFlag | kPreLoadFlag)) {
    // spill A first (the word starts a second-evaluated subtree)
    if (w & kSpillFlag) {
      switch ((w >> kSpillShift) & 7u) {
        case 0:
#pragma unroll
          for (int j = 0; j < K; ++j) s.R[0][j] = s.A[j];
          break;
        case 1:
#pragma unroll
          for (int j = 0; j < K; ++j) s.R[1][j] = s.A[j];
          break;
        case 2:
#pragma unroll
          for (int j = 0; j < K; ++j) s.R[2][j] = s.A[j];
          break;
        case 3:
#pragma unroll
          for (int j = 0; j < K; ++j) s.R[3][j] = s.A[j];
          break;
        default: {
          float* dst = spill + ((int)((w >> kSpillShift) & 7u) - kRegSlots) * (K * kWave);
#pragma unroll
          for (int j = 0; j < K; ++j) dst[j * kWave] = s.A[j];
        } break;
      }
    }
    // then load a variable (the first operand of a binary node over two leaves)
    if (w & kPreLoadFlag) {
      const int var = (int)((w >> kPreLoadShift) & 15u);
#pragma unroll
      for (int v = 0; v < VM; ++v)
        if (v == var) {
#pragma unroll
          for (int j = 0; j < K; ++j) s.A[j] = s.X[v][j];
        }
    }
    }

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

#define TGP_MB_CASE(B)                                                                      \
  case kMB + 2 * (B):                                                                       \
    _Pragma("unroll") for (int j = 0; j < K; ++j) {                                         \
      s.r[j] = bin_op<(B)>(s.A[j], s.T[j]);                                                 \
      s.A[j] = s.T[j];                                                                      \
    }                                                                                       \
    break;                                                                                  \
  case kMB + 2 * (B) + 1:                                                                   \
    _Pragma("unroll") for (int j = 0; j < K; ++j) s.r[j] = bin_op<(B)>(s.T[j], s.A[j]);     \
    break;

// Unary functions are applied after the switch, from the word's action bits
// (apply_unary).
    switch (c) {
      TGP_SRC_CASES(kLD, s.A[j] = v)
      TGP_SRC_CASES(kTLD, s.T[j] = v)
      TGP_SRC_CASES(kADD, s.A[j] = s.A[j] + v)
      TGP_SRC_CASES(kMUL, s.A[j] = s.A[j] * v)
      TGP_SRC_CASES(kMAX, s.A[j] = vmax(s.A[j], v))
      TGP_SRC_CASES(kMIN, s.A[j] = vmin(s.A[j], v))
      TGP_SRC_CASES(kSUBA, s.A[j] = s.A[j] - v)
      TGP_SRC_CASES(kSUBR, s.A[j] = v - s.A[j])
      TGP_SRC_CASES(kDIVA, s.A[j] = bin_op<3>(s.A[j], v))
      TGP_SRC_CASES(kDIVR, s.A[j] = bin_op<3>(v, s.A[j]))
      TGP_MB_CASE(0)
      TGP_MB_CASE(1)
      TGP_MB_CASE(2)
      TGP_MB_CASE(3)
      TGP_MB_CASE(4)
      TGP_MB_CASE(5)
      case kACC:
        add_out<K, VM, NO>(s, (int)(ins >> 32));
        break;
      case kNOP:
        break;
      default:  // kEND (or any word that is not an instruction)
        act = kActStop;
        break;
    }
#undef TGP_SRC_CASE
#undef TGP_SRC_CASES
#undef TGP_MB_CASE
    if (BOUNDED) {
      if (--left == 0) act |= kActStop;
    }
    // keep act an opaque scalar: otherwise the compiler threads the per-case
    // constants through boolean phis held as 64-bit lane masks
    asm volatile("" : "+s"(act));
    if (act & kActUn) {
      apply_unary<K, VM, NO>(s, act);
      // DUAL (forward programs): the word's second action
      if (DUAL && (w & kAct2Flag)) {
        int un2 = act2_of(w);
        asm volatile("" : "+s"(un2));
        apply_unary<K, VM, NO>(s, un2);
      }
    }
    if constexpr (CAPTURE) {
      if ((w & kCapFlag) && capture_level(w) == cap_level) {
        const int c = *csp;
        if (c < cap_limit) {
          float* dst = cap + c * (K * kWave);
#pragma unroll
          for (int j = 0; j < K; ++j) dst[j * kWave] = s.A[j];
        }
        *csp = c + 1;
      }
    }
    unsigned long long n2 = nxt;
    asm volatile("" : "+s"(n2));
    ins = n2;
    if (act & kActStop) break;
  }
}

template <int K, int VM, int NO, bool BOUNDED = false, bool CAPTURE = false>
__device__ __forceinline__ void run_program(prog_ptr prog, Regs<K, VM, NO>& s, float* spill, int count = 0,
                                            float* cap = nullptr, int* csp = nullptr, int cap_level = 0,
                                            int cap_limit = 0) {
  if (BOUNDED && count <= 0) return;
  run_from<K, VM, NO, BOUNDED, CAPTURE>(prog, prog[0], s, spill, count, cap, csp, cap_level, cap_limit);
}

// 64-bit DPP move: row_shr / row_bcast as in the GCN data-parallel
// primitives; lanes with no source, or outside row_mask, read 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, true));
}

// Sum over the 64 lanes (all active), returned in every lane: row shifts by
// 1, 2, 4, 8 leave each row's sum in its lane 15; two row broadcasts carry
// the row sums up to lane 63. VALU only (no LDS round trips).
constexpr int kRowShr = 0x110, kRowBcast15 = 0x142, kRowBcast31 = 0x143;

__device__ __forceinline__ double wave_sum_f64(double v) {
  v += dpp_f64<kRowShr + 1, 0xf>(v);
  v += dpp_f64<kRowShr + 2, 0xf>(v);
  v += dpp_f64<kRowShr + 4, 0xf>(v);
  v += dpp_f64<kRowShr + 8, 0xf>(v);
  v += dpp_f64<kRowBcast15, 0xa>(v);
  v += dpp_f64<kRowBcast31, 0xc>(v);
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ float wave_sum_f32(float v) {
  v += dpp_f32<kRowShr + 1, 0xf>(v);
  v += dpp_f32<kRowShr + 2, 0xf>(v);
  v += dpp_f32<kRowShr + 4, 0xf>(v);
  v += dpp_f32<kRowShr + 8, 0xf>(v);
  v += dpp_f32<kRowBcast15, 0xa>(v);
  v += dpp_f32<kRowBcast31, 0xc>(v);
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

}  // namespace interp
}  // namespace tgp
