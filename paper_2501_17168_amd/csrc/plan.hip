// Plan kernel: validate every tree of the population and compile it into a
// program for the wave-uniform interpreter (see tgp_isa.h).
//
// One 64-lane wave per tree, lanes over nodes. Validation follows the
// encoding of §III-A (NaN padding after len = size[0]; subtree sizes give
// child positions c1 = i+1, c2 = c1 + size[c1]). The integer figures are
// the length, the maximum stack depth of the reversed-prefix evaluation of
// §III-C, the constant and Modi node counts and the length bucket.
//
// Code generation runs in three data-parallel passes over the node array
// held in LDS: a bottom-up pass (spill need and code size of each subtree,
// iterated to a fixed point within each 64-node chunk, last chunk first),
// a top-down pass (code start and spill base of each subtree, first chunk
// first), and an emission pass in which every function node writes its
// own instructions at positions known from the two passes.
#include <hip/hip_runtime.h>
#include <math.h>

#include "tgp_kernels.h"

namespace tgp {

namespace {

constexpr int kWave = 64;

// node record bits in LDS
//  0..1 kind (0 var, 1 const, 2 func), 2..3 arity, 4..7 op, 8..11 modi out + 1 (0 = plain), 12..16 var index
__device__ __forceinline__ int rec_kind(int r) { return r & 3; }
__device__ __forceinline__ int rec_arity(int r) { return (r >> 2) & 3; }
__device__ __forceinline__ int rec_op(int r) { return (r >> 4) & 15; }
__device__ __forceinline__ int rec_modi(int r) { return ((r >> 8) & 15) - 1; }
__device__ __forceinline__ int rec_var(int r) { return (r >> 12) & 31; }

__device__ __forceinline__ bool is_intf(float x) { return isfinite(x) && x == floorf(x); }

__device__ __forceinline__ bool fused_op(int op) {
  return op == kOpAdd || op == kOpSub || op == kOpMul || op == kOpMax || op == kOpMin;
}

// number of instructions a function node emits for its own operation
__device__ __forceinline__ int own_code(int r) {
  const int a = rec_arity(r);
  if (rec_modi(r) >= 0) return a == 2 ? 3 : 2;  // [TLD] MB/MU ACC
  if (a == 2) return fused_op(rec_op(r)) ? 1 : 2;
  return 1;
}

__device__ __forceinline__ int wave_min(int v) {
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, kWave));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, kWave));
  return v;
}
__device__ __forceinline__ int wave_sum(int v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// source operand of a leaf for instruction encoding
__device__ __forceinline__ void leaf_src(int r, const float* vals, int i, int& src, float& pay) {
  if (rec_kind(r) == kTypeConst) {
    src = kSrcC;
    pay = vals[i];
  } else {
    src = kSrcX0 + rec_var(r);
    pay = 0.0f;
  }
}

__device__ __forceinline__ void put(uint2* __restrict__ prog, int64_t cap, int pos, uint32_t w, float pay) {
  if (pos >= 0 && pos < cap) prog[pos] = make_uint2(w, __float_as_uint(pay));
}

__device__ __forceinline__ int src_slot(int slot, int& aux) {
  if (slot < kRegSlots) {
    aux = 0;
    return kSrcR0 + slot;
  }
  aux = slot;
  return kSrcRM;
}

__device__ __forceinline__ int fused_case(int op, bool a_first, int src) {
  switch (op) {
    case kOpAdd: return kADD + src;
    case kOpMul: return kMUL + src;
    case kOpMax: return kMAX + src;
    case kOpMin: return kMIN + src;
    default: return (a_first ? kSUBA : kSUBR) + src;  // kOpSub
  }
}

}  // namespace

constexpr int kMaxChunks = kMaxLmax / kWave;

// LDS per tree: rec, need|code size, start|base, constant value, adjoint
// order (int/float, Lpad each) and subtree size (short, Lpad); Lpad = Lmax
// rounded up to 64.
__host__ __device__ constexpr size_t plan_lds_bytes(int Lmax) {
  return (size_t)((Lmax + kWave - 1) / kWave * kWave) * (5 * sizeof(int) + sizeof(short));
}

__global__ __launch_bounds__(64) void plan_kernel(PlanArgs a) {
  extern __shared__ int s_plan[];
  const int Lpad = (a.Lmax + kWave - 1) / kWave * kWave;
  int* s_rec = s_plan;
  int* s_nc = s_rec + Lpad;  // need << 16 | code size; -1 = unknown
  int* s_sb = s_nc + Lpad;   // start | base << 16; -1 = unknown
  float* s_val = (float*)(s_sb + Lpad);
  int* s_ai = (int*)(s_val + Lpad);  // internal-node count, then record position | pop << 16
  short* s_sz = (short*)(s_ai + Lpad);

  const int lane = threadIdx.x;
  const int64_t t = blockIdx.x;
  if (t >= a.P) return;
  const float* trow = a.type + t * a.row_stride;
  const float* vrow = a.value + t * a.row_stride;
  const float* srow = a.size + t * a.row_stride;
  int32_t* info = a.info + t * kInfoStride;
  uint2* prog = a.prog + t * a.pstride;
  const int Lmax = a.Lmax;

  // Issue every global load of the row at once (the padding check reads all
  // Lmax entries, so their count is known before len is).
  float tv[kMaxChunks], vv[kMaxChunks], sv[kMaxChunks];
  const int nch_all = (Lmax + kWave - 1) / kWave;
  int nch_loaded = a.check_tail ? nch_all : 0;
#pragma unroll
  for (int ch = 0; ch < kMaxChunks; ++ch) {
    const int i = ch * kWave + lane;
    tv[ch] = vv[ch] = sv[ch] = __builtin_nanf("");
    if (ch < nch_loaded && i < Lmax) {
      tv[ch] = trow[i];
      vv[ch] = vrow[i];
      sv[ch] = srow[i];
    }
  }
  const float s0 = a.check_tail ? __shfl(sv[0], 0, kWave) : srow[0];

  int status = 0;
  int len = 0;
  if (!(is_intf(s0) && s0 >= 1.0f && s0 <= (float)Lmax)) status = 1;
  else len = (int)s0;

  int n_const = 0, n_modi = 0, max_stack = 0, need0 = 0, prog_len = 0, n_int = 0;

  if (status == 0) {
    const int scan_end = a.check_tail ? Lmax : len;
    if (!a.check_tail) {
      nch_loaded = (len + kWave - 1) / kWave;
#pragma unroll
      for (int ch = 0; ch < kMaxChunks; ++ch) {
        const int i = ch * kWave + lane;
        if (ch < nch_loaded && i < len) {
          tv[ch] = trow[i];
          vv[ch] = vrow[i];
          sv[ch] = srow[i];
        }
      }
    }
    // ---- pass 1: decode, NaN / padding / code checks ----
    int err = 1 << 20;
    int size_bad = 0;
#pragma unroll
    for (int ch = 0; ch < kMaxChunks; ++ch) {
      const int i = ch * kWave + lane;
      if (ch >= nch_loaded || i >= scan_end) continue;
      const float tq = tv[ch], vq = vv[ch], sq = sv[ch];
      if (i >= len) {
        if (!(isnan(tq) && isnan(vq) && isnan(sq))) err = min(err, 3);
        continue;
      }
      s_nc[i] = 0;
      s_sb[i] = -1;
      s_val[i] = vq;
      if (isnan(tq) || isnan(vq) || isnan(sq)) {
        err = min(err, 2);
        s_rec[i] = 0;
        s_sz[i] = -1;
        continue;
      }
      int rec = 0;
      if (!(is_intf(tq) && tq >= 0.0f && tq < (float)(kTypeModi0 + a.n_out))) {
        err = min(err, 4);
      } else {
        const int ti = (int)tq;
        if (ti == kTypeConst) {
          rec = kTypeConst;
          ++n_const;
        } else if (ti == kTypeVar) {
          if (!(is_intf(vq) && vq >= 0.0f && vq < (float)a.V)) err = min(err, 6);
          else rec = kTypeVar | ((int)vq << 12);
        } else {
          if (!(is_intf(vq) && vq >= 0.0f && vq < (float)kNumOps)) {
            err = min(err, 5);
          } else {
            const int op = (int)vq;
            const int mo = ti >= kTypeModi0 ? ti - kTypeModi0 : -1;
            rec = kTypeFunc | (op_arity(op) << 2) | (op << 4) | ((mo + 1) << 8);
            if (mo >= 0) ++n_modi;
          }
        }
      }
      s_rec[i] = rec;
      if (is_intf(sq) && sq >= 1.0f && sq <= (float)len) s_sz[i] = (short)(int)sq;
      else { s_sz[i] = -1; size_bad = 1; }
      // leaves are complete for the bottom-up pass; function nodes unknown
      s_nc[i] = (rec_kind(rec) == kTypeFunc) ? -1 : 0;
    }
    err = wave_min(err);
    n_const = wave_sum(n_const);
    n_modi = wave_sum(n_modi);
    size_bad = wave_max(size_bad);
    __syncthreads();
    if (err < (1 << 20)) status = err;
    else if (size_bad) status = 7;

    // ---- pass 2: subtree-size invariant ----
    if (status == 0) {
      int bad = 0;
      for (int base = 0; base < len; base += kWave) {
        const int i = base + lane;
        if (i >= len) continue;
        const int r = s_rec[i];
        const int ar = rec_arity(r);
        int want = 1, c = i + 1;
        for (int k = 0; k < ar; ++k) {
          if (c >= len) { bad = 1; break; }
          const int sc = s_sz[c];
          if (sc < 1) { bad = 1; break; }
          want += sc;
          c += sc;
        }
        if (!bad && (s_sz[i] != want || i + s_sz[i] > len)) bad = 1;
      }
      if (wave_max(bad)) status = 7;
    }
  }

  if (status == 0) {
    // ---- pass 3: max stack depth, suffix sums of (1 - arity) ----
    int carry = 0, best = 0;
    const int nch = (len + kWave - 1) / kWave;
    for (int ch = nch - 1; ch >= 0; --ch) {
      const int i = ch * kWave + lane;
      int x = (i < len) ? 1 - rec_arity(s_rec[i]) : 0;
      for (int off = 1; off < kWave; off <<= 1) {
        const int y = __shfl_down(x, off, kWave);
        if (lane + off < kWave) x += y;
      }
      if (i < len) best = max(best, x + carry);
      carry += __shfl(x, 0, kWave);
    }
    max_stack = wave_max(best);

    // ---- pass 4: bottom-up spill need and code size ----
    for (int ch = nch - 1; ch >= 0; --ch) {
      const int i = ch * kWave + lane;
      bool done = !(i < len && rec_kind(s_rec[i]) == kTypeFunc);
      for (int it = 0; it <= kWave; ++it) {
        if (!done) {
          const int r = s_rec[i];
          const int c1 = i + 1;
          const int nc1 = s_nc[c1];
          const bool l1 = rec_kind(s_rec[c1]) != kTypeFunc;
          const int oc = own_code(r);
          if (rec_arity(r) == 1) {
            if (nc1 >= 0) {
              const int need = l1 ? 0 : (nc1 >> 16);
              const int cs = (l1 ? 1 : (nc1 & 0xffff)) + oc;
              s_nc[i] = (need << 16) | cs;
              done = true;
            }
          } else {
            const int c2 = c1 + s_sz[c1];
            const int nc2 = s_nc[c2];
            const bool l2 = rec_kind(s_rec[c2]) != kTypeFunc;
            if (nc1 >= 0 && nc2 >= 0) {
              int need, cs;
              if (l1 && l2) { need = 0; cs = 1 + oc; }
              else if (l1) { need = nc2 >> 16; cs = (nc2 & 0xffff) + oc; }
              else if (l2) { need = nc1 >> 16; cs = (nc1 & 0xffff) + oc; }
              else {
                const int n1 = nc1 >> 16, n2 = nc2 >> 16;
                need = (n1 == n2) ? n1 + 1 : max(n1, n2);
                cs = (nc1 & 0xffff) + (nc2 & 0xffff) + 1 + oc;
              }
              s_nc[i] = (need << 16) | cs;
              done = true;
            }
          }
        }
        __syncthreads();
        if (__all(done)) break;
      }
    }
    const int root = s_rec[0];
    if (rec_kind(root) == kTypeFunc) {
      need0 = s_nc[0] >> 16;
      prog_len = (s_nc[0] & 0xffff) + 1;
    } else {
      need0 = 0;
      prog_len = 2;
    }

    // ---- pass 5: top-down code start and spill base ----
    if (lane == 0) s_sb[0] = 0;
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
      const int i = ch * kWave + lane;
      bool done = !(i < len && rec_kind(s_rec[i]) == kTypeFunc);
      for (int it = 0; it <= kWave; ++it) {
        if (!done) {
          const int sb = s_sb[i];
          if (sb >= 0) {
            const int st = sb & 0xffff, bs = sb >> 16;
            const int r = s_rec[i];
            const int c1 = i + 1;
            const bool l1 = rec_kind(s_rec[c1]) != kTypeFunc;
            if (rec_arity(r) == 1) {
              if (!l1) s_sb[c1] = sb;
            } else {
              const int c2 = c1 + s_sz[c1];
              const bool l2 = rec_kind(s_rec[c2]) != kTypeFunc;
              if (l1 && !l2) s_sb[c2] = sb;
              else if (!l1 && l2) s_sb[c1] = sb;
              else if (!l1 && !l2) {
                const int nc1 = s_nc[c1], nc2 = s_nc[c2];
                const bool f1 = (nc1 >> 16) >= (nc2 >> 16);
                const int F = f1 ? c1 : c2, S = f1 ? c2 : c1;
                const int csF = (f1 ? nc1 : nc2) & 0xffff;
                s_sb[F] = sb;
                s_sb[S] = (st + csF + 1) | ((bs + 1) << 16);
              }
            }
            done = true;
          }
        }
        __syncthreads();
        if (__all(done)) break;
      }
    }

    // ---- pass 6: emission ----
    if (rec_kind(root) != kTypeFunc) {
      if (lane == 0) {
        int src; float pay;
        leaf_src(root, s_val, 0, src, pay);
        put(prog, a.pstride, 0, mkword(kLD + src), pay);
      }
    }
    for (int base = 0; base < len; base += kWave) {
      const int i = base + lane;
      if (i >= len) continue;
      const int r = s_rec[i];
      if (rec_kind(r) != kTypeFunc) continue;
      const int sb = s_sb[i];
      const int st = sb & 0xffff, bs = sb >> 16;
      const int cs = s_nc[i] & 0xffff;
      const int oc = own_code(r);
      int pos = st + cs - oc;  // first own instruction
      const int op = rec_op(r);
      const int mo = rec_modi(r);
      const int c1 = i + 1;
      const int r1 = s_rec[c1];
      const bool l1 = rec_kind(r1) != kTypeFunc;
      if (rec_arity(r) == 1) {
        if (l1) {
          int src; float pay;
          leaf_src(r1, s_val, c1, src, pay);
          put(prog, a.pstride, st, mkword(kLD + src), pay);
        }
        if (mo < 0) {
          put(prog, a.pstride, pos, mkword(kUN + un_index(op)), 0.0f);
        } else {
          put(prog, a.pstride, pos, mkword(kMU + un_index(op)), 0.0f);
          put(prog, a.pstride, pos + 1, mkword(kACC, mo), 0.0f);
        }
        continue;
      }
      const int c2 = c1 + s_sz[c1];
      const int r2 = s_rec[c2];
      const bool l2 = rec_kind(r2) != kTypeFunc;
      int src, aux = 0;
      float pay = 0.0f;
      bool a_first;  // A holds the first operand and src the second
      if (l1 && l2) {
        int s1; float p1;
        leaf_src(r1, s_val, c1, s1, p1);
        put(prog, a.pstride, st, mkword(kLD + s1), p1);
        leaf_src(r2, s_val, c2, src, pay);
        a_first = true;
      } else if (l1) {
        leaf_src(r1, s_val, c1, src, pay);
        a_first = false;
      } else if (l2) {
        leaf_src(r2, s_val, c2, src, pay);
        a_first = true;
      } else {
        const int nc1 = s_nc[c1], nc2 = s_nc[c2];
        const bool f1 = (nc1 >> 16) >= (nc2 >> 16);
        const int csF = (f1 ? nc1 : nc2) & 0xffff;
        int saux;
        if (bs < kRegSlots) put(prog, a.pstride, st + csF, mkword(kSPL + bs), 0.0f);
        else put(prog, a.pstride, st + csF, mkword(kSPLM, bs), 0.0f);
        src = src_slot(bs, saux);
        aux = saux;
        a_first = !f1;  // first-evaluated child is in the slot
      }
      if (mo >= 0) {
        put(prog, a.pstride, pos, mkword(kTLD + src, aux), pay);
        put(prog, a.pstride, pos + 1, mkword(kMB + 2 * bin_index(op) + (a_first ? 0 : 1)), 0.0f);
        put(prog, a.pstride, pos + 2, mkword(kACC, mo), 0.0f);
      } else if (fused_op(op)) {
        put(prog, a.pstride, pos, mkword(fused_case(op, a_first, src), aux), pay);
      } else {
        put(prog, a.pstride, pos, mkword(kTLD + src, aux), pay);
        put(prog, a.pstride, pos + 1, mkword(kBT + 2 * bin_index(op) + (a_first ? 0 : 1)), 0.0f);
      }
    }
    if (lane == 0) {
      put(prog, a.pstride, prog_len - 1, mkword(kEND), 0.0f);
      put(prog, a.pstride, prog_len, mkword(kEND), 0.0f);  // read by the interpreter's one-word lookahead
    }

    // ---- pass 7: adjoint records (gradient calls only) ----
    if (a.adj) {
      // bottom-up: number of function nodes in each subtree
      for (int base = 0; base < len; base += kWave) {
        const int i = base + lane;
        if (i < len) s_ai[i] = rec_kind(s_rec[i]) == kTypeFunc ? -1 : 0;
      }
      __syncthreads();
      for (int ch = nch - 1; ch >= 0; --ch) {
        const int i = ch * kWave + lane;
        bool done = !(i < len && rec_kind(s_rec[i]) == kTypeFunc);
        for (int it = 0; it <= kWave; ++it) {
          if (!done) {
            const int c1 = i + 1;
            const int a1 = s_ai[c1];
            int a2 = 0;
            if (rec_arity(s_rec[i]) == 2) a2 = s_ai[c1 + s_sz[c1]];
            if (a1 >= 0 && a2 >= 0) {
              s_ai[i] = 1 + a1 + a2;
              done = true;
            }
          }
          __syncthreads();
          if (__all(done)) break;
        }
      }
      n_int = rec_kind(root) == kTypeFunc ? s_ai[0] : 0;
      __syncthreads();
      // top-down: record position and pending flag (smaller child first)
      if (lane == 0 && rec_kind(root) == kTypeFunc) s_ai[0] = 0 | (1 << 30);
      __syncthreads();
      for (int ch = 0; ch < nch; ++ch) {
        const int i = ch * kWave + lane;
        bool done = !(i < len && rec_kind(s_rec[i]) == kTypeFunc);
        for (int it = 0; it <= kWave; ++it) {
          if (!done) {
            const int qi = s_ai[i];
            if (qi & (1 << 30)) {
              const int q = qi & 0xffff;
              const int c1 = i + 1;
              const bool f1 = rec_kind(s_rec[c1]) == kTypeFunc;
              if (rec_arity(s_rec[i]) == 1) {
                if (f1) s_ai[c1] = (q + 1) | (1 << 30);
              } else {
                const int c2 = c1 + s_sz[c1];
                const bool f2 = rec_kind(s_rec[c2]) == kTypeFunc;
                const bool c2first = s_sz[c2] < s_sz[c1];
                const int F = c2first ? c2 : c1, S = c2first ? c1 : c2;
                const bool fF = c2first ? f2 : f1, fS = c2first ? f1 : f2;
                const int nF = fF ? s_ai[F] : 0;
                if (fF) s_ai[F] = (q + 1) | (1 << 30);
                if (fS) s_ai[S] = (q + 1 + nF) | (1 << 30) | (fF ? (1 << 16) : 0);
              }
              done = true;
            }
          }
          __syncthreads();
          if (__all(done)) break;
        }
      }
      // emission
      uint32_t* recs = a.adj + t * (int64_t)Lmax * kAdjWords;
      for (int base = 0; base < len; base += kWave) {
        const int i = base + lane;
        if (i >= len) continue;
        const int r = s_rec[i];
        if (rec_kind(r) != kTypeFunc) continue;
        const int qi = s_ai[i];
        const int q = qi & 0xffff;
        if (q >= Lmax) continue;
        const int pop = (qi >> 16) & 1;
        const int ar = rec_arity(r);
        const int c1 = i + 1;
        const int c2 = ar == 2 ? c1 + s_sz[c1] : -1;
        uint32_t wv[kAdjWords] = {0, 0, 0, 0, 0, 0, 0, 0};
        int kinds[2] = {kKindNone, kKindNone}, vars[2] = {0, 0};
        const int ch2[2] = {c1, c2};
        bool both_func = ar == 2;
        for (int k = 0; k < ar; ++k) {
          const int c = ch2[k];
          const int rc = s_rec[c];
          if (rec_kind(rc) == kTypeFunc) {
            kinds[k] = kKindFunc;
            wv[1 + 2 * k] = (uint32_t)(s_sb[c] & 0xffff);
            wv[2 + 2 * k] = (uint32_t)(s_nc[c] & 0xffff);
          } else if (rec_kind(rc) == kTypeVar) {
            kinds[k] = kKindVar;
            vars[k] = rec_var(rc);
            both_func = false;
          } else {
            kinds[k] = kKindConst;
            wv[1 + 2 * k] = (uint32_t)c;
            wv[2 + 2 * k] = __float_as_uint(s_val[c]);
            both_func = false;
          }
        }
        const int c2first = (ar == 2 && s_sz[c2] < s_sz[c1]) ? 1 : 0;
        wv[0] = (uint32_t)(rec_op(r) | (ar << 4) | ((rec_modi(r) >= 0 ? 1 : 0) << 6) | (c2first << 7) |
                           (pop << 8) | ((both_func ? 1 : 0) << 9) | (kinds[0] << 10) | (kinds[1] << 12) |
                           (vars[0] << 14) | (vars[1] << 18));
        uint4* dst = (uint4*)(recs + (int64_t)q * kAdjWords);
        dst[0] = make_uint4(wv[0], wv[1], wv[2], wv[3]);
        dst[1] = make_uint4(wv[4], 0u, 0u, 0u);
      }
    }
  }

  if (status != 0) {
    len = 0; n_const = 0; n_modi = 0; max_stack = 0; need0 = 0; prog_len = 0; n_int = 0;
  }
  if (lane == 0) {
    const int bucket = len <= 1 ? 0 : 32 - __clz(len - 1);
    info[kInfoStatus] = status;
    info[kInfoLen] = len;
    info[kInfoMaxStack] = max_stack;
    info[kInfoNConst] = n_const;
    info[kInfoNModi] = n_modi;
    info[kInfoBucket] = bucket;
    info[kInfoProgLen] = prog_len;
    info[kInfoNeed] = need0;
    info[kInfoNInternal] = n_int;
    a.acc[t] = 0.0;
    if (a.hist && status == 0) atomicAdd(&a.hist[bucket], 1);
    if (a.out_status) a.out_status[t] = status;
    if (a.out_info) {
      int32_t* o = a.out_info + t * 6;
      o[0] = status; o[1] = len; o[2] = max_stack; o[3] = n_const; o[4] = n_modi; o[5] = bucket;
    }
  }
}

__global__ void prep_kernel(int32_t* c, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) c[i] = 0;
}

// Counting sort of the trees by length bucket, longest bucket first, invalid trees last.
__global__ void order_kernel(OrderArgs a) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.P) return;
  const int32_t* inf = a.info + t * kInfoStride;
  int pos;
  if (inf[kInfoStatus] != 0) {
    // invalid trees go after every valid one (the evaluators skip them)
    int nvalid = 0;
    for (int k = 0; k < 16; ++k) nvalid += a.hist[k];
    pos = nvalid + atomicAdd(&a.cursor[16], 1);
  } else {
    const int b = inf[kInfoBucket];
    int off = 0;
    for (int k = 15; k > b; --k) off += a.hist[k];
    pos = off + atomicAdd(&a.cursor[b], 1);
  }
  a.order[pos] = (int32_t)t;
}

hipError_t launch_prep(int32_t* counters, int n, hipStream_t s) {
  prep_kernel<<<(n + 255) / 256, 256, 0, s>>>(counters, n);
  return hipGetLastError();
}

hipError_t launch_plan(const PlanArgs& a, hipStream_t s) {
  if (a.P <= 0) return hipSuccess;
  plan_kernel<<<dim3((unsigned)a.P), dim3(64), plan_lds_bytes(a.Lmax), s>>>(a);
  return hipGetLastError();
}

hipError_t launch_order(const OrderArgs& a, hipStream_t s) {
  if (a.P <= 0) return hipSuccess;
  order_kernel<<<(unsigned)((a.P + 255) / 256), 256, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace tgp
