#pragma once
// Fitness gradient by a reverse sweep over each tree, with recomputation.
//
// L = sum_t g_t * mse_t. For every (tree, point tile) a wave
//   1. runs the tree's forward program once: output, residual e, the
//      fitness contribution and the output adjoint gbar = g_t * 2 e / D;
//   2. walks the tree's adjoint records (one per function node, pre-order
//      with the smaller child first). A record takes its adjoint either
//      from the previous record or from the pending stack, recomputes the
//      values of its function children by re-running their code ranges of
//      the forward program (their code is contiguous), forms the partial
//      derivatives and hands each child its adjoint: a variable leaf adds it
//      to the lane's grad_X accumulator, a constant leaf adds the wave's sum
//      to grad_value, a function child becomes the next record's adjoint or
//      waits on the pending stack (at most log2(len) entries deep).
// Nothing is stored per point beyond the current path's adjoints. A Modi
// node for output o hands gbar_o * df/dchild to its children and passes its
// own adjoint on to its rightmost child, whose value it forwards.
//
// Work units are point-major: each workgroup holds block_waves tiles and a
// run of trees, so grad_X accumulates in registers across the run and is
// written with one float atomic per (lane, point, variable) at the end.
#include <hip/hip_runtime.h>
#include <math.h>

#include "interp.h"
#include "tgp_kernels.h"

namespace tgp {

namespace {

using namespace interp;

typedef const __attribute__((address_space(4))) uint32_t* rec_ptr;

// partial derivatives of op at (a, b); b unused for unary ops
__device__ __forceinline__ void partials(int op, float a, float b, float& da, float& db) {
  da = 1.0f;
  db = 0.0f;
  switch (op) {
    case kOpAdd: db = 1.0f; break;
    case kOpSub: db = -1.0f; break;
    case kOpMul: da = b; db = a; break;
    case kOpDiv: {
      const bool small = fabsf(b) < kDivTau;
      const float r = 1.0f / b;
      da = small ? 0.0f : r;
      db = small ? 0.0f : -a * r * r;
    } break;
    case kOpMax: {
      const bool pa = (a >= b) || isnan(b);
      da = pa ? 1.0f : 0.0f;
      db = pa ? 0.0f : 1.0f;
    } break;
    case kOpMin: {
      const bool pa = (a <= b) || isnan(b);
      da = pa ? 1.0f : 0.0f;
      db = pa ? 0.0f : 1.0f;
    } break;
    case kOpSin: da = cosf(a); break;
    case kOpCos: da = -sinf(a); break;
    case kOpTanh: {
      const float th = tanhf(a);
      da = 1.0f - th * th;
    } break;
    case kOpExp: da = (a >= -kExpClamp && a <= kExpClamp) ? exp_clamped(a) : 0.0f; break;
    case kOpLog: da = a == 0.0f ? 0.0f : copysignf(1.0f, a) / (fabsf(a) + kLogEps); break;
    default: {  // tan
      const float tn = tanf(a);
      da = 1.0f + tn * tn;
    } break;
  }
}


// The same partial derivatives when the node's own value v is at hand (own):
// exp, tanh and tan take it instead of calling the library again. v came from
// the same float32 argument through the same function, so the result is
// bitwise the one partials() gives.
__device__ __forceinline__ void partials_own(int op, float a, float b, float v, bool own, float& da, float& db) {
  if (own && op == kOpExp) {
    da = (a >= -kExpClamp && a <= kExpClamp) ? v : 0.0f;
    db = 0.0f;
  } else if (own && op == kOpTanh) {
    da = 1.0f - v * v;
    db = 0.0f;
  } else if (own && op == kOpTan) {
    da = 1.0f + v * v;
    db = 0.0f;
  } else {
    partials(op, a, b, da, db);
  }
}

template <int K, int VM, int NO>
struct AdjState {
  Regs<K, VM, NO> s;
  float gx[VM][K];  // grad_X accumulators for this lane's points
};

template <int K, int VM, int NO>
__device__ __forceinline__ void load_x_adj(const AdjArgs& a, Regs<K, VM, NO>& s, int64_t p0) {
#pragma unroll
  for (int v = 0; v < VM; ++v) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int64_t p = p0 + j * kWave;
      s.X[v][j] = __builtin_canonicalizef((v < a.V && p < a.D) ? a.X[(int64_t)v * a.ldx + p] : 0.0f);
    }
  }
}

// value of a leaf child for this lane's K points
template <int K, int VM, int NO>
__device__ __forceinline__ void leaf_value(const Regs<K, VM, NO>& s, int kind, int var, uint32_t bits, float out[K]) {
  if (kind == kKindConst) {
#pragma unroll
    for (int j = 0; j < K; ++j) out[j] = __uint_as_float(bits);
  } else {
#pragma unroll
    for (int v = 0; v < VM; ++v)
      if (v == var) {
#pragma unroll
        for (int j = 0; j < K; ++j) out[j] = s.X[v][j];
      }
  }
}

// a leaf child receives its adjoint
template <int K, int VM, int NO>
__device__ __forceinline__ void leaf_adjoint(const AdjArgs& a, AdjState<K, VM, NO>& st, int64_t t, int64_t p0,
                                             int lane, int kind, int var, uint32_t node, const float adj[K]) {
  if (kind == kKindVar) {
#pragma unroll
    for (int v = 0; v < VM; ++v)
      if (v == var) {
#pragma unroll
        for (int j = 0; j < K; ++j) st.gx[v][j] += adj[j];
      }
  } else if (kind == kKindConst && a.grad_value) {
    float sum = 0.0f;
#pragma unroll
    for (int j = 0; j < K; ++j) sum += (p0 + j * kWave < a.D) ? adj[j] : 0.0f;
    sum = wave_sum_f32(sum);
    if (lane == 0) atomicAdd(&a.grad_value[t * a.gv_stride + node], sum);
  }
}

// After a tree's forward run: the fitness partial of the tile (a float64 sum of the
// float32 squared residuals over the points and outputs) and the output adjoints
// gbar[o] = g_t * 2 (out_o - Y_o) / D. A tree without Modi nodes predicts
// (root, 0, ..., 0); outputs at or beyond n_out, and points past D, get 0.
template <int K, int VM, int NO>
__device__ __forceinline__ double output_adjoints(const AdjArgs& a, const Regs<K, VM, NO>& s, bool modi, float gt,
                                                  int64_t p0, float (&gbar)[NO][K]) {
  double sse = 0.0;
#pragma unroll
  for (int o = 0; o < NO; ++o) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int64_t p = p0 + j * kWave;
      gbar[o][j] = 0.0f;
      if (o < a.n_out && p < a.D) {
        const float out = modi ? s.O[o][j] : (o == 0 ? s.A[j] : 0.0f);
        const float e = out - a.Y[(int64_t)o * a.ldy + p];
        sse += (double)(e * e);
        gbar[o][j] = gt * 2.0f * e * a.inv_D;
      }
    }
  }
  return sse;
}

// The output adjoint of Modi output mo (wave-uniform) at point slot j.
template <int K, int NO>
__device__ __forceinline__ float out_adjoint(const float (&gbar)[NO][K], int mo, int j) {
  float v = gbar[0][j];
#pragma unroll
  for (int o = 1; o < NO; ++o) v = (mo == o) ? gbar[o][j] : v;
  return v;
}

// The trees among c0 .. c0 + 63 (below t1) that are valid and whose records are in format `fmt`,
// as a wave-uniform bit mask: one load per lane and a ballot, so that a sweep skips the other
// sweep's trees without a dependent scalar load per tree.
__device__ __forceinline__ unsigned long long trees_of_format(const AdjArgs& a, int64_t c0, int64_t t1, int lane,
                                                              int fmt) {
  const int64_t t = c0 + lane;
  bool want = false;
  if (t < t1) {
    const int32_t* inf = a.info + t * kInfoStride;
    want = inf[kInfoStatus] == 0 && inf[kInfoAdjFmt] == fmt;
  }
  return __ballot(want);
}

}  // namespace

template <int K, int VM, int NO>
__global__ __launch_bounds__(256) void adjoint_kernel(AdjArgs a) {
  extern __shared__ float s_lds[];
  constexpr int kTile = K * kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  const int W = blockDim.x / kWave;
  const int per_wave = (kMaxSlots - kRegSlots + a.pend_slots) * K * kWave;
  float* spill = s_lds + wv * per_wave + lane;
  float* pend = spill + (kMaxSlots - kRegSlots) * K * kWave;

  const int64_t b = blockIdx.x;
  const int g = (int)(b % a.ngroups);
  const int tile = g * W + wv;
  if (tile >= a.ntiles) return;
  const int64_t t0 = (b / a.ngroups) * a.tpu;
  const int64_t t1 = min(a.P, t0 + a.tpu);
  const int64_t p0 = (int64_t)tile * kTile + lane;

  AdjState<K, VM, NO> st;
  Regs<K, VM, NO>& s = st.s;
  load_x_adj<K, VM, NO>(a, s, p0);
#pragma unroll
  for (int v = 0; v < VM; ++v)
#pragma unroll
    for (int j = 0; j < K; ++j) st.gx[v][j] = 0.0f;

  bool swept = false;  // this wave swept a tree (otherwise it has no grad_X to add)
  for (int64_t c0 = t0; c0 < t1; c0 += kWave)
  for (unsigned long long m = trees_of_format(a, c0, t1, lane, kAdjFmtRecompute); m; m &= m - 1) {
    const int64_t t = c0 + __builtin_ctzll(m);
    const int32_t* inf = a.info + t * kInfoStride;
    swept = true;
    const int nmodi = __builtin_amdgcn_readfirstlane(inf[kInfoNModi]);
    const int nint = __builtin_amdgcn_readfirstlane(inf[kInfoNInternal]);
    const int plen = __builtin_amdgcn_readfirstlane(inf[kInfoProgLen]);
    const float gt = a.grad_mse ? a.grad_mse[t] : 1.0f;
    prog_ptr prog = (prog_ptr)(a.prog + t * a.pstride);
    rec_ptr recs = (rec_ptr)(a.adj + t * (int64_t)a.Lmax * kAdjWords);

    float gbar[NO][K], cur[K];
    int sp = 0;
    // Step q = -1 is the forward pass (the whole program but its END); step
    // q >= 0 is adjoint record q. Every interpreter run of the tree happens
    // at the one call site below, so the kernel holds one copy of the
    // interpreter's dispatch code.
    for (int q = -1; q < nint; ++q) {
      uint32_t w0 = 0, w1 = 0, w2 = 0, w3 = 0, w4 = 0;
      int op = 0, ar = 0, k1 = kKindNone, k2 = kKindNone, v1 = 0, v2 = 0;
      float va[K], vb[K];
#pragma unroll
      for (int j = 0; j < K; ++j) va[j] = vb[j] = 0.0f;
      // interpreter runs of this step: start, length, destination (0: va, 1: vb, 2: forward)
      uint32_t rs0 = 0, rl0 = 0, rs1 = 0, rl1 = 0;
      int nrun = 0, d0 = 2, d1 = 1;
      if (q < 0) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
          s.A[j] = 0.0f;
#pragma unroll
          for (int o = 0; o < NO; ++o) s.O[o][j] = 0.0f;
        }
        nrun = 1;
        rs0 = 0;
        rl0 = (uint32_t)(plen - 1);
        d0 = 2;
      } else {
        w0 = recs[kAdjWords * q];
        w1 = recs[kAdjWords * q + 1];
        w2 = recs[kAdjWords * q + 2];
        w3 = recs[kAdjWords * q + 3];
        w4 = recs[kAdjWords * q + 4];
        op = w0 & 15;
        ar = (w0 >> 4) & 3;
        k1 = (w0 >> 10) & 3;
        k2 = (w0 >> 12) & 3;
        v1 = (w0 >> 14) & 15;
        v2 = (w0 >> 18) & 15;
        // children values (not needed for add / sub)
        if (op != kOpAdd && op != kOpSub) {
          if (k1 == kKindFunc) {
            rs0 = w1;
            rl0 = w2;
            d0 = 0;
            nrun = 1;
          } else {
            leaf_value<K, VM, NO>(s, k1, v1, w2, va);
          }
          if (ar == 2) {
            if (k2 == kKindFunc) {
              if (nrun == 0) {
                rs0 = w3;
                rl0 = w4;
                d0 = 1;
              } else {
                rs1 = w3;
                rl1 = w4;
                d1 = 1;
              }
              ++nrun;
            } else {
              leaf_value<K, VM, NO>(s, k2, v2, w4, vb);
            }
          }
        }
      }
#pragma nounroll
      for (int r = 0; r < nrun; ++r) {
        const uint32_t rs = r == 0 ? rs0 : rs1, rl = r == 0 ? rl0 : rl1;
        const int dst = r == 0 ? d0 : d1;
        run_program<K, VM, NO, true>(prog + rs, s, spill, (int)rl);
        if (dst == 0) {
#pragma unroll
          for (int j = 0; j < K; ++j) va[j] = s.A[j];
        } else if (dst == 1) {
#pragma unroll
          for (int j = 0; j < K; ++j) vb[j] = s.A[j];
        }
      }

      if (q < 0) {
        // ---- forward: outputs, fitness, output adjoints ----
        const double sse = wave_sum_f64(output_adjoints<K, VM, NO>(a, s, nmodi != 0, gt, p0, gbar));
        if (lane == 0) a.part[tile * a.P + t] = sse;
        if (nint == 0) {  // the tree is a single leaf
          const uint2 ins = a.prog[t * a.pstride];
          const int src = word_case(ins.x) - kLD;
          if (src >= kSrcX0)
            leaf_adjoint<K, VM, NO>(a, st, t, p0, lane, kKindVar, src - kSrcX0, 0u, gbar[0]);
          else
            leaf_adjoint<K, VM, NO>(a, st, t, p0, lane, kKindConst, 0, 0u, gbar[0]);
        }
#pragma unroll
        for (int j = 0; j < K; ++j) cur[j] = nmodi ? 0.0f : gbar[0][j];
        continue;
      }

      // ---- adjoint record q ----
      const int modi = (w0 >> 6) & 1, c2first = (w0 >> 7) & 1, mo = (int)((w0 >> 22) & 3);
      const int pop = (w0 >> 8) & 1, push = (w0 >> 9) & 1;
      float adj[K];
      if (pop) {
        sp = sp > 0 ? sp - 1 : 0;
#pragma unroll
        for (int j = 0; j < K; ++j) adj[j] = pend[(sp * K + j) * kWave];
      } else {
#pragma unroll
        for (int j = 0; j < K; ++j) adj[j] = cur[j];
      }
      float a1[K], a2[K];
#pragma unroll
      for (int j = 0; j < K; ++j) {
        float da, db;
        partials(op, va[j], vb[j], da, db);
        const float base = modi ? out_adjoint<K, NO>(gbar, mo, j) : adj[j];
        a1[j] = base * da;
        a2[j] = base * db;
        if (modi) {  // the handed-up value is the rightmost child's
          if (ar == 2) a2[j] += adj[j];
          else a1[j] += adj[j];
        }
      }
      // leaves take their adjoint now; function children go on
      if (k1 != kKindFunc) leaf_adjoint<K, VM, NO>(a, st, t, p0, lane, k1, v1, w1, a1);
      if (ar == 2 && k2 != kKindFunc) leaf_adjoint<K, VM, NO>(a, st, t, p0, lane, k2, v2, w3, a2);
      if (push) {  // both children are function nodes
        const float* second = c2first ? a1 : a2;
        const float* first = c2first ? a2 : a1;
        if (sp < a.pend_slots) {
#pragma unroll
          for (int j = 0; j < K; ++j) pend[(sp * K + j) * kWave] = second[j];
          ++sp;
        }
#pragma unroll
        for (int j = 0; j < K; ++j) cur[j] = first[j];
      } else if (k1 == kKindFunc) {
#pragma unroll
        for (int j = 0; j < K; ++j) cur[j] = a1[j];
      } else if (ar == 2 && k2 == kKindFunc) {
#pragma unroll
        for (int j = 0; j < K; ++j) cur[j] = a2[j];
      }
    }
  }

  // ---- grad_X: one atomic per (lane, point, variable) for the whole run ----
  if (a.grad_X && swept) {
#pragma unroll
    for (int v = 0; v < VM; ++v) {
      if (v < a.V) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const int64_t p = p0 + j * kWave;
          if (p < a.D) atomicAdd(&a.grad_X[(int64_t)v * a.ldx + p], st.gx[v][j]);
        }
      }
    }
  }
}

// Heavy-path sweep (trees whose records are in the heavy-path format).
// Per (tree, tile): one run of the whole program gives the output, the
// fitness partial and the captures of the root path; the records then walk
// each path top down. At a record the children's values are popped from the
// capture stack (light child on top, heavy child below it), the partials
// formed, leaves take their adjoints, the light child's adjoint waits on the
// pending stack, and the heavy child's adjoint and value become the current
// ones. At the end of a path the most recently parked light child is taken
// and its code range run once at its light depth, which captures its own
// path and leaves its value in A. Every function node is thus interpreted
// once per path head above it (the root's run included), instead of once
// per function ancestor. The next record is loaded while the current one is
// worked on.
// Wave LDS: `cap` values (captures from the bottom, pending adjoints from the
// top; during a run the tree's spill slots beyond the four in registers sit
// just below the pending adjoints), then `cap` ints of pending code ranges.
__device__ __forceinline__ uint4 load_path_record(rec_ptr p) { return make_uint4(p[0], p[1], p[2], p[3]); }

template <int K, int VM, int NO>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(K >= 3 ? 3 : 4))) void adjoint_path_kernel(
    AdjArgs a) {
  extern __shared__ float s_lds[];
  constexpr int kTile = K * kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int W = blockDim.x / kWave;
  const int CAP = a.cap;
  const int per_wave = CAP * K * kWave;
  float* vals = s_lds + wv * per_wave + lane;
  int* pinfo = (int*)(s_lds + W * per_wave) + wv * CAP;

  const int64_t b = blockIdx.x;
  const int g = (int)(b % a.ngroups);
  const int tile = g * W + wv;
  if (tile >= a.ntiles) return;
  const int64_t t0 = (b / a.ngroups) * a.tpu;
  const int64_t t1 = min(a.P, t0 + a.tpu);
  const int64_t p0 = (int64_t)tile * kTile + lane;

  AdjState<K, VM, NO> st;
  Regs<K, VM, NO>& s = st.s;
  load_x_adj<K, VM, NO>(a, s, p0);
#pragma unroll
  for (int v = 0; v < VM; ++v)
#pragma unroll
    for (int j = 0; j < K; ++j) st.gx[v][j] = 0.0f;

  bool swept = false;  // this wave swept a tree (otherwise it has no grad_X to add)
  for (int64_t c0 = t0; c0 < t1; c0 += kWave)
  for (unsigned long long m = trees_of_format(a, c0, t1, lane, kAdjFmtPath); m; m &= m - 1) {
    const int64_t t = c0 + __builtin_ctzll(m);
    const int32_t* inf = a.info + t * kInfoStride;
    swept = true;
    const int nmodi = __builtin_amdgcn_readfirstlane(inf[kInfoNModi]);
    const int nint = __builtin_amdgcn_readfirstlane(inf[kInfoNInternal]);
    const int plen = __builtin_amdgcn_readfirstlane(inf[kInfoProgLen]);
    // spill slots in LDS: those beyond the four in registers
    const int xslots = max(__builtin_amdgcn_readfirstlane(inf[kInfoNeed]) - kRegSlots, 0);
    const float gt = a.grad_mse ? a.grad_mse[t] : 1.0f;
    prog_ptr prog = (prog_ptr)(a.prog + t * a.pstride);
    rec_ptr recs = (rec_ptr)(a.adj + t * (int64_t)a.Lmax * kAdjWords);

    float gbar[NO][K], cur[K], curv[K];
    int csp = 0, psp = 0, q = 0;
    // the run ahead: the whole program but its END (the root's), or a light head's code range
    uint32_t rs = 0, rl = (uint32_t)(plen - 1);
    int rlev = 0;
    bool root = true;
    uint4 rn = make_uint4(0u, 0u, 0u, 0u);  // the next record, loaded ahead
    for (;;) {
      if (root) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
          s.A[j] = 0.0f;
#pragma unroll
          for (int o = 0; o < NO; ++o) s.O[o][j] = 0.0f;
        }
        if (nint > 0) rn = load_path_record(recs);
      }
      // the kernel's one interpreter call site; the run's LDS spill slots sit just below the
      // pending adjoints, above every capture the run can push
      float* spill = vals + (CAP - psp - xslots) * (K * kWave);
      run_program<K, VM, NO, true, true>(prog + rs, s, spill, (int)rl, vals, &csp, rlev, CAP - psp - xslots);
      if (root) {
        root = false;
        // ---- forward: outputs, fitness partial, output adjoints ----
        const double sse = wave_sum_f64(output_adjoints<K, VM, NO>(a, s, nmodi != 0, gt, p0, gbar));
        if (lane == 0) a.part[tile * a.P + t] = sse;
        if (nint == 0) {  // the tree is a single leaf
          const uint2 ins = a.prog[t * a.pstride];
          const int src = word_case(ins.x) - kLD;
          if (src >= kSrcX0)
            leaf_adjoint<K, VM, NO>(a, st, t, p0, lane, kKindVar, src - kSrcX0, 0u, gbar[0]);
          else
            leaf_adjoint<K, VM, NO>(a, st, t, p0, lane, kKindConst, 0, 0u, gbar[0]);
          break;
        }
#pragma unroll
        for (int j = 0; j < K; ++j) cur[j] = nmodi ? 0.0f : gbar[0][j];
      }
      // the run's value is the current node's own value: the root's, or the light head's
#pragma unroll
      for (int j = 0; j < K; ++j) curv[j] = s.A[j];
      // ---- records down to the end of a path ----
      bool run_next = false;
      while (q < nint) {
        const uint32_t w0 = rn.x, w1 = rn.y, w2 = rn.z, w3 = rn.w;
        ++q;
        const int op = w0 & 15, ar = (w0 >> 4) & 3, modi = (w0 >> 6) & 1, mo = (int)((w3 >> 16) & 3);
        const int pat = (w0 >> 7) & 15;
        const int va_var = (w0 >> 11) & 15, vb_var = (w0 >> 15) & 15;
        const int eop = (w0 >> 19) & 1;
        const uint32_t node_a = w0 >> 22, node_b = w3 & 0xffffu;
        const float ca = __uint_as_float(w1), cb = __uint_as_float(w2);
        // children values by pattern: the light child's capture is on top, the heavy child's
        // below it; a record with both pops two
        float vh[K], va[K], vb[K];
#pragma unroll
        for (int j = 0; j < K; ++j) vb[j] = 0.0f;
        const float* top = vals + (csp - 1) * (K * kWave);
        const float* below = vals + (csp - 2) * (K * kWave);
        switch (pat) {
          case kPatHL:
          case kPatLH: {
            float vl[K];
#pragma unroll
            for (int j = 0; j < K; ++j) {
              vl[j] = top[j * kWave];
              vh[j] = below[j * kWave];
            }
            csp -= 2;
#pragma unroll
            for (int j = 0; j < K; ++j) {
              va[j] = pat == kPatHL ? vh[j] : vl[j];
              vb[j] = pat == kPatHL ? vl[j] : vh[j];
            }
          } break;
          case kPatHV:
          case kPatHC:
          case kPatH:
#pragma unroll
            for (int j = 0; j < K; ++j) va[j] = vh[j] = top[j * kWave];
            csp -= 1;
            if (pat == kPatHV) leaf_value<K, VM, NO>(s, kKindVar, vb_var, 0u, vb);
            if (pat == kPatHC)
#pragma unroll
              for (int j = 0; j < K; ++j) vb[j] = cb;
            break;
          case kPatVH:
          case kPatCH:
#pragma unroll
            for (int j = 0; j < K; ++j) vb[j] = vh[j] = top[j * kWave];
            csp -= 1;
            if (pat == kPatVH) leaf_value<K, VM, NO>(s, kKindVar, va_var, 0u, va);
            else
#pragma unroll
              for (int j = 0; j < K; ++j) va[j] = ca;
            break;
          case kPatVV:
          case kPatVC:
          case kPatV:
            leaf_value<K, VM, NO>(s, kKindVar, va_var, 0u, va);
            if (pat == kPatVV) leaf_value<K, VM, NO>(s, kKindVar, vb_var, 0u, vb);
            if (pat == kPatVC)
#pragma unroll
              for (int j = 0; j < K; ++j) vb[j] = cb;
            break;
          default:  // kPatCV, kPatCC, kPatC
#pragma unroll
            for (int j = 0; j < K; ++j) va[j] = ca;
            if (pat == kPatCV) leaf_value<K, VM, NO>(s, kKindVar, vb_var, 0u, vb);
            if (pat == kPatCC)
#pragma unroll
              for (int j = 0; j < K; ++j) vb[j] = cb;
            break;
        }
        // the next record, loaded while this one is worked on
        if (q < nint) rn = load_path_record(recs + q * kPathWords);
        float a1[K], a2[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
          float da, db;
          partials_own(op, va[j], vb[j], curv[j], !modi, da, db);
          const float base = modi ? out_adjoint<K, NO>(gbar, mo, j) : cur[j];
          a1[j] = base * da;
          a2[j] = base * db;
          if (modi) {  // the handed-up value is the rightmost child's
            if (ar == 2) a2[j] += cur[j];
            else a1[j] += cur[j];
          }
        }
        // adjoints by pattern: leaves take theirs now, the light child's waits on the pending
        // stack with its code range, the heavy child's becomes the current one
        auto park = [&](const float* al, uint32_t info) {
          if (csp + psp + 1 <= CAP) {
            float* dadj = vals + (CAP - 1 - psp) * (K * kWave);
#pragma unroll
            for (int j = 0; j < K; ++j) dadj[j * kWave] = al[j];
            pinfo[psp] = (int)info;
          }
          ++psp;
        };
        auto follow = [&](const float* ah) {
#pragma unroll
          for (int j = 0; j < K; ++j) {
            cur[j] = ah[j];
            curv[j] = vh[j];
          }
        };
        switch (pat) {
          case kPatHL: park(a2, w2); follow(a1); break;
          case kPatLH: park(a1, w1); follow(a2); break;
          case kPatHV: leaf_adjoint<K, VM, NO>(a, st, t, p0, lane, kKindVar, vb_var, 0u, a2); follow(a1); break;
          case kPatVH: leaf_adjoint<K, VM, NO>(a, st, t, p0, lane, kKindVar, va_var, 0u, a1); follow(a2); break;
          case kPatHC: leaf_adjoint<K, VM, NO>(a, st, t, p0, lane, kKindConst, 0, node_b, a2); follow(a1); break;
          case kPatCH: leaf_adjoint<K, VM, NO>(a, st, t, p0, lane, kKindConst, 0, node_a, a1); follow(a2); break;
          case kPatVV:
            leaf_adjoint<K, VM, NO>(a, st, t, p0, lane, kKindVar, va_var, 0u, a1);
            leaf_adjoint<K, VM, NO>(a, st, t, p0, lane, kKindVar, vb_var, 0u, a2);
            break;
          case kPatVC:
            leaf_adjoint<K, VM, NO>(a, st, t, p0, lane, kKindVar, va_var, 0u, a1);
            leaf_adjoint<K, VM, NO>(a, st, t, p0, lane, kKindConst, 0, node_b, a2);
            break;
          case kPatCV:
            leaf_adjoint<K, VM, NO>(a, st, t, p0, lane, kKindConst, 0, node_a, a1);
            leaf_adjoint<K, VM, NO>(a, st, t, p0, lane, kKindVar, vb_var, 0u, a2);
            break;
          case kPatCC:
            leaf_adjoint<K, VM, NO>(a, st, t, p0, lane, kKindConst, 0, node_a, a1);
            leaf_adjoint<K, VM, NO>(a, st, t, p0, lane, kKindConst, 0, node_b, a2);
            break;
          case kPatH: follow(a1); break;
          case kPatV: leaf_adjoint<K, VM, NO>(a, st, t, p0, lane, kKindVar, va_var, 0u, a1); break;
          default: leaf_adjoint<K, VM, NO>(a, st, t, p0, lane, kKindConst, 0, node_a, a1); break;  // kPatC
        }
        if (eop) {
          if (psp == 0) break;  // the tree's last path
          --psp;
          const float* sadj = vals + (CAP - 1 - psp) * (K * kWave);
#pragma unroll
          for (int j = 0; j < K; ++j) cur[j] = sadj[j * kWave];
          const uint32_t info = (uint32_t)__builtin_amdgcn_readfirstlane(pinfo[psp]);
          rs = info & 0xfffu;
          rl = (info >> 12) & 0xfffu;
          rlev = (int)((info >> 24) & 15u);
          run_next = true;
          break;
        }
      }
      if (!run_next) break;
    }
  }

  // ---- grad_X: one atomic per (lane, point, variable) for the whole run ----
  if (a.grad_X && swept) {
#pragma unroll
    for (int v = 0; v < VM; ++v) {
      if (v < a.V) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const int64_t p = p0 + j * kWave;
          if (p < a.D) atomicAdd(&a.grad_X[(int64_t)v * a.ldx + p], st.gx[v][j]);
        }
      }
    }
  }
}

// Both sweeps: heavy-path trees, then the trees whose sweep would not fit the
// heavy-path kernel's LDS budget (each kernel skips the other's trees).
template <int K, int VM, int NO>
hipError_t launch_adjoint_kvo(const AdjArgs& a, int block_waves, int64_t grid, hipStream_t s) {
  if (a.cap > 0) {
    const size_t lds_p = (size_t)block_waves * (a.cap * K * kWave * sizeof(float) + a.cap * sizeof(int));
    adjoint_path_kernel<K, VM, NO><<<dim3((unsigned)grid), dim3(block_waves * kWave), lds_p, s>>>(a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const size_t lds = (size_t)block_waves * (kMaxSlots - kRegSlots + a.pend_slots) * K * kWave * sizeof(float);
  adjoint_kernel<K, VM, NO><<<dim3((unsigned)grid), dim3(block_waves * kWave), lds, s>>>(a);
  return hipGetLastError();
}

// Single-output populations carry one output accumulator and adjoint; multi-output ones
// (2 to 4 outputs) carry four.
template <int K, int VM>
hipError_t launch_adjoint_kv(const AdjArgs& a, int block_waves, int64_t grid, hipStream_t s) {
  return a.n_out == 1 ? launch_adjoint_kvo<K, VM, 1>(a, block_waves, grid, s)
                      : launch_adjoint_kvo<K, VM, kMaxOutGrad>(a, block_waves, grid, s);
}

}  // namespace tgp
