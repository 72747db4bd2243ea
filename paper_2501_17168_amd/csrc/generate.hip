// Random tree generation in the padded prefix encoding (§III-A): grow,
// full and ramped half-and-half, one tree per thread (the paper runs
// initialisation one individual per GPU thread).
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011),
// counter (tree, attempt, position, 0), key (seed low, seed high); the four
// words of one call serve one node, mapped to [0, 1) as (w >> 8) * 2^-24.
//
// A thread fills slots in prefix order from a stack of open child slots
// (each with its depth). Node sizes come out of the same forward pass: a
// function node opened when the slot stack held S entries closes when the
// stack is back to S - 1, and its size is the distance travelled since.
// Both stacks live in LDS, one short column per thread; a depth limit of at
// most kMaxGenDepth bounds them. The thread writes each node's type and
// value as it goes, and each size when its subtree closes; an attempt that
// outgrows Lmax starts over (later attempts overwrite the row). Finally
// the wave writes the NaN padding of its 64 rows, one row at a time, with
// coalesced stores.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "tgp.h"
#include "tgp_generate.h"

namespace tgp {
namespace {

constexpr int kGenThreads = 256;
constexpr int kStack = kMaxGenDepth + 2;

constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;  // Philox4x32 multipliers
constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;  // key increments per round

struct U4 {
  uint32_t x, y, z, w;
};

__device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint32_t hi0 = __umulhi(kM0, c.x), lo0 = kM0 * c.x;
    const uint32_t hi1 = __umulhi(kM1, c.z), lo1 = kM1 * c.z;
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
  }
  return c;
}

__device__ inline float unit(uint32_t w) { return (float)(w >> 8) * 5.9604644775390625e-08f; }

__device__ inline int arity_of(int op) { return (op <= 3 || op == 9 || op == 10) ? 2 : 1; }

__global__ __launch_bounds__(kGenThreads) void generate_kernel(GenArgs a) {
  // constants are lo + (hi - lo) * u with each operation rounded: no fused multiply-add
#pragma clang fp contract(off)
  __shared__ uint8_t slot_depth[kStack][kGenThreads];  // open child slots (depths)
  __shared__ int16_t open_pos[kStack][kGenThreads];    // open function nodes: position ...
  __shared__ uint8_t open_mark[kStack][kGenThreads];   // ... and slot-stack size at which it closes
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int64_t i = (int64_t)blockIdx.x * kGenThreads + tid;  // output row
  const int64_t wave_first = i - lane;
  const bool active = i < a.P;
  int len = 0;
  if (active) {
    const uint32_t t = (uint32_t)(a.first_tree + i);
    int depth = a.d_max;
    bool full = a.method == TGP_GEN_FULL;
    if (a.method == TGP_GEN_RAMPED) {
      depth = a.d_min + (int)((t >> 1) % (uint32_t)(a.d_max - a.d_min + 1));
      full = (t & 1u) == 0;
    }
    float* __restrict__ ot = a.out_t + i * a.out_ld;
    float* __restrict__ ov = a.out_v + i * a.out_ld;
    float* __restrict__ os = a.out_s + i * a.out_ld;
    const float span = a.hi - a.lo;
    uint32_t attempt = 0;
    for (;;) {
      int ns = 1, no = 0, n = 0;  // slot-stack size, open-node stack size, nodes placed
      slot_depth[0][tid] = 0;
      bool ok = true;
      while (ns > 0) {
        if (n == a.Lmax) {
          ok = false;
          break;
        }
        const int h = slot_depth[--ns][tid];
        const U4 r = philox4x32_10(U4{t, attempt, (uint32_t)n, 0u}, a.key0, a.key1);
        const float u0 = unit(r.x), u1 = unit(r.y), u2 = unit(r.z);
        const bool is_func = full ? h < depth : (h < depth && (h == 0 || u0 < a.p_func));
        if (is_func) {
          const int f = min((int)floorf(u1 * (float)a.n_funcs), a.n_funcs - 1);
          const int op = a.funcs[f];
          ot[n] = 2.0f;
          ov[n] = (float)op;
          // closes when the slot stack is back to its size before this node's slot was popped
          open_pos[no][tid] = (int16_t)n;
          open_mark[no][tid] = (uint8_t)ns;
          ++no;
          const int ar = arity_of(op);
          for (int c = 0; c < ar; ++c) slot_depth[ns++][tid] = (uint8_t)(h + 1);
        } else {
          if (u1 < a.p_const) {
            ot[n] = 1.0f;
            ov[n] = a.lo + span * u2;
          } else {
            ot[n] = 0.0f;
            ov[n] = (float)min((int)floorf(u2 * (float)a.V), a.V - 1);
          }
          os[n] = 1.0f;
        }
        ++n;
        // every function node whose subtree is now complete gets its size
        while (no > 0 && (int)open_mark[no - 1][tid] == ns) {
          --no;
          const int p = open_pos[no][tid];
          os[p] = (float)(n - p);
        }
      }
      ++attempt;
      if (ok) {
        len = n;
        break;
      }
      if (attempt % (uint32_t)a.attempts_per_depth == 0 && depth > 0) --depth;
    }
    if (a.attempts) a.attempts[i] = (int32_t)attempt;
  }
  // NaN padding of the wave's rows, coalesced: row by row, lanes over columns
  const float nan = __builtin_nanf("");
  const int nrows = (int)min<int64_t>(64, a.P - wave_first);
  for (int rr = 0; rr < nrows; ++rr) {
    const int from = __shfl(len, rr);
    float* __restrict__ ot = a.out_t + (wave_first + rr) * a.out_ld;
    float* __restrict__ ov = a.out_v + (wave_first + rr) * a.out_ld;
    float* __restrict__ os = a.out_s + (wave_first + rr) * a.out_ld;
    for (int p = from + lane; p < a.Lmax; p += 64) {
      ot[p] = nan;
      ov[p] = nan;
      os[p] = nan;
    }
  }
}

}  // namespace

hipError_t launch_generate(const GenArgs& a, hipStream_t s) {
  if (a.P <= 0) return hipSuccess;
  const int64_t grid = (a.P + kGenThreads - 1) / kGenThreads;
  hipLaunchKernelGGL(generate_kernel, dim3((unsigned)grid), dim3(kGenThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace tgp
