#pragma once
// Float32 exp and log for the protected operators of the function set, on
// the domains those operators give them (exp: arguments clamped to
// [-kExpClamp, kExpClamp]; log: arguments |x| + kLogEps, never below
// kLogEps), so the general library paths for overflow, underflow and
// subnormal arguments are not needed.
//
// Both use the hardware base-2 instructions with the classic compensated
// change of base:
//   exp(x) = 2^n * 2^f, with x*log2(e) = n + f, n an integer; x*log2(e) is
//     carried as a float32 head and the tail fma(x, L, -head) +
//     x*(log2(e) - L), L = log2(e) rounded to float32, so f keeps the bits
//     the head loses;
//   log(y) = log2(y) * ln(2), the product taken as a head and a tail the
//     same way (ln(2) = M + (ln(2) - M), M a float32 just below ln(2)).
// Accuracy is checked on the device against float64 over dense samples of
// both domains (tests/test_gpu_ops.py): exp within 0.85 ulp, log within
// 2.4 ulp (the hardware base-2 log's error), inside the 4 ulp that the
// float32 envelopes assume of the math library.
#include <hip/hip_runtime.h>

#include "tgp_isa.h"

namespace tgp {

// log2(e) and ln(2) as a float32 head and the float32 rounding of the remainder (the ln(2) head
// rounded down)
constexpr float kLog2eHi = 0x1.715476p+0f;   // bits 0x3fb8aa3b
constexpr float kLog2eLo = 0x1.4ae0cp-26f;   // bits 0x32a57060
constexpr float kLn2Hi = 0x1.62e42ep-1f;     // bits 0x3f317217 (ln(2) rounded down)
constexpr float kLn2Lo = 0x1.efa39ep-25f;    // bits 0x3377d1cf

// exp of the clamped argument: NaN stays NaN, everything else is clamped to
// [-kExpClamp, kExpClamp] first.
__device__ __forceinline__ float exp_clamped(float a) {
  // head - n must stay a plain (exact) subtraction: contracted into fma(x, L, -n) it would carry
  // the head's rounding error a second time
#pragma clang fp contract(off)
  const float x = a > kExpClamp ? kExpClamp : (a < -kExpClamp ? -kExpClamp : a);
  const float head = x * kLog2eHi;
  const float n = __builtin_rintf(head);
  const float tail = __builtin_fmaf(x, kLog2eLo, __builtin_fmaf(x, kLog2eHi, -head));
  const float f = (head - n) + tail;
  return __builtin_amdgcn_ldexpf(__builtin_amdgcn_exp2f(f), (int)n);
}

// log(y) for y >= kLogEps (a positive normal number), +inf or NaN.
__device__ __forceinline__ float log_positive(float y) {
  const float l2 = __builtin_amdgcn_logf(y);
  const float head = l2 * kLn2Hi;
  const float tail = __builtin_fmaf(l2, kLn2Lo, __builtin_fmaf(l2, kLn2Hi, -head));
  const float r = head + tail;
  return __builtin_fabsf(l2) < __builtin_inff() ? r : l2;
}

}  // namespace tgp
