// Plan kernel: validate every tree of the population and compile it into a
// program for the wave-uniform interpreter (see tgp_isa.h).
//
// One 64-lane wave per tree, lanes over nodes. Validation follows the
// encoding of §III-A (NaN padding after len = size[0]; subtree sizes give
// child positions c1 = i+1, c2 = c1 + size[c1]). The integer figures are
// the length, the maximum stack depth of the reversed-prefix evaluation of
// §III-C, the constant and Modi node counts and the length bucket.
//
// Code generation takes the child with the larger subtree first at every
// node whose two children are both function nodes, and spills its value
// while the smaller child runs. A value is held only while descending into
// a subtree of at most half the size, so a tree of at most 1024 nodes needs
// at most 8 spill slots. With that rule every figure the emitter needs is a
// sum over a contiguous node range or over the ancestors of a node, and
// subtrees are contiguous ranges in the prefix encoding (§III-A):
//   * the code size of a subtree and its count of function nodes are range
//     sums of per-node contributions (one prefix scan);
//   * the code start, the spill base and the adjoint-record position of a
//     node are sums of terms that its ancestors attach to the range of one
//     of their children (a difference array: each ancestor adds its term at
//     the first index of the range and subtracts it after the last; one
//     prefix scan gives, at every node, the sum over its ancestors).
// Every pass is a fixed number of chunk-wide scans: no per-tree iteration
// to a fixed point and no dependence on the tree's height.

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
// set on the later-visited child of a node whose children are both function nodes (adjoint order)
constexpr int kRecPop = 1 << 20;
// set on the light child of a node whose children are both function nodes: the smaller one, which
// the code evaluates second (ties: the second child)
constexpr int kRecLight = 1 << 21;
// forward programs: set on a unary node that takes the second action of the word carrying its
// child's function (pass 3b)
constexpr int kRecSecond = 1 << 22;

__device__ __forceinline__ bool is_intf(float x) { return isfinite(x) && x == floorf(x); }

__device__ __forceinline__ bool fused_op(int op) {
  return op == kOpAdd || op == kOpSub || op == kOpMul || op == kOpDiv || op == kOpMax || op == kOpMin;
}

// number of instructions a function node emits for its own operation (a
// unary node over a leaf emits its load with the function in the action
// bits, which is the same count)
__device__ __forceinline__ int own_code(int r) {
  const int a = rec_arity(r);
  if (rec_modi(r) >= 0) return a == 2 ? 3 : 2;  // TLD MB ACC | (LD or NOP) + action, ACC
  return 1;                                     // fused binary op | (LD or NOP) + action
}

// Forward programs: a unary node whose child is a binary function node puts
// its function in the action bits of that child's last word (the fused op
// word, or the ACC of a Modi child), which never carries an action of its
// own, instead of a NOP word; it then emits nothing, or only its ACC when it
// is a Modi node. Gradient programs keep the NOP: there the child's last word
// captures the child's value for the adjoint sweep.
__device__ __forceinline__ bool folds_into_child(int r, int rc1, bool adj) {
  return !adj && rec_kind(r) == kTypeFunc && rec_arity(r) == 1 && rec_kind(rc1) == kTypeFunc &&
         rec_arity(rc1) == 2;
}

// action bits of a unary node: its function, for the Modi register if Modi
__device__ __forceinline__ int unary_act(int op, int mo) {
  return kActUn | un_index(op) | (mo >= 0 ? kActModi : 0);
}

// Wave-wide integer reductions and scans with DPP row shifts and row
// broadcasts (VALU only; no LDS round trips). All 64 lanes must be active.
constexpr int kRowShr = 0x110, kRowBcast15 = 0x142, kRowBcast31 = 0x143;

template <int CTRL, int ROW_MASK, bool KEEP>
__device__ __forceinline__ int dpp(int v) {
  // KEEP: lanes without a source keep v; otherwise they read 0
  return __builtin_amdgcn_update_dpp(KEEP ? v : 0, v, CTRL, ROW_MASK, 0xf, !KEEP);
}

// inclusive prefix sum over the 64 lanes
__device__ __forceinline__ int wave_incl_scan(int x) {
  x += dpp<kRowShr + 1, 0xf, false>(x);
  x += dpp<kRowShr + 2, 0xf, false>(x);
  x += dpp<kRowShr + 4, 0xf, false>(x);
  x += dpp<kRowShr + 8, 0xf, false>(x);
  x += dpp<kRowBcast15, 0xa, false>(x);
  x += dpp<kRowBcast31, 0xc, false>(x);
  return x;
}

__device__ __forceinline__ int lane63(int v) { return __builtin_amdgcn_readlane(v, 63); }

__device__ __forceinline__ int wave_sum(int v) { return lane63(wave_incl_scan(v)); }

template <bool MAX>
__device__ __forceinline__ int wave_ext(int v) {
  auto f = [](int a, int b) { return MAX ? max(a, b) : min(a, b); };
  v = f(v, dpp<kRowShr + 1, 0xf, true>(v));
  v = f(v, dpp<kRowShr + 2, 0xf, true>(v));
  v = f(v, dpp<kRowShr + 4, 0xf, true>(v));
  v = f(v, dpp<kRowShr + 8, 0xf, true>(v));
  v = f(v, dpp<kRowBcast15, 0xa, true>(v));
  v = f(v, dpp<kRowBcast31, 0xc, true>(v));
  return lane63(v);
}
__device__ __forceinline__ int wave_max(int v) { return wave_ext<true>(v); }
__device__ __forceinline__ int wave_min(int v) { return wave_ext<false>(v); }

// source operand of a leaf for instruction encoding
__device__ __forceinline__ void leaf_src(int r, float value, int& src, float& pay) {
  if (rec_kind(r) == kTypeConst) {
    src = kSrcC;
    pay = value;
  } else {
    src = kSrcX0 + rec_var(r);
    pay = 0.0f;
  }
}

// a binary non-Modi node over two leaves, one of them a variable, is one
// word: the variable is pre-loaded into A and the case takes the other leaf
__device__ __forceinline__ bool preload_fusable(int r, int r1, int r2) {
  return rec_modi(r) < 0 && (rec_kind(r1) == kTypeVar || rec_kind(r2) == kTypeVar);
}

// a load of leaf source `src`, with action bits, spilling A first when the
// spill map says so (pre = slot + 1)
__device__ __forceinline__ uint32_t load_word(int src, int act, int pre) {
  const uint32_t w = mkword(kLD + src, 0, act);
  return pre ? with_spill(w, pre - 1) : w;
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
    case kOpDiv: return (a_first ? kDIVA : kDIVR) + src;
    default: return (a_first ? kSUBA : kSUBR) + src;  // kOpSub
  }
}

}  // namespace


// packed fields of the prefix sums E: code size (bits 0..15), function nodes (16..31)
// and of the ancestor sums D: code start (0..11), spill base (12..15), record shift (16..)
constexpr int kStartBits = 12;

// Heavy child of function node h (its larger function child, the one its code
// evaluates first, ties: the first child; or its only function child), or -1;
// `light` receives the other function child of a node with two, or -1.
__device__ int heavy_child(const int* s_rec, const short* s_sz, int h, int& light) {
  light = -1;
  const int c1 = h + 1;
  const bool f1 = rec_kind(s_rec[c1]) == kTypeFunc;
  if (rec_arity(s_rec[h]) == 1) return f1 ? c1 : -1;
  const int c2 = c1 + s_sz[c1];
  const bool f2 = rec_kind(s_rec[c2]) == kTypeFunc;
  if (f1 && f2) {
    if (s_sz[c1] >= s_sz[c2]) {
      light = c2;
      return c1;
    }
    light = c1;
    return c2;
  }
  return f1 ? c1 : (f2 ? c2 : -1);
}

// Values (each K points of a lane) the heavy-path sweep holds at once: at the
// start of each path, the captures of the path's function children plus the
// adjoint of every waiting light child. Along a path the count only falls (a
// record pops its children's captures before it parks its light child), so
// the path starts give the maximum. Sequential; one lane.
__device__ int path_need(const int* s_rec, const short* s_sz, int* stk) {
  int sp = 0, need = 0;
  stk[sp++] = 0;
  while (sp > 0) {
    const int F = stk[--sp];
    int caps = 0, lt;
    for (int h = F; h >= 0;) {
      const int hv = heavy_child(s_rec, s_sz, h, lt);
      caps += (hv >= 0) + (lt >= 0);
      h = hv;
    }
    need = max(need, sp + caps);
    for (int h = F; h >= 0;) {
      const int hv = heavy_child(s_rec, s_sz, h, lt);
      if (lt >= 0) stk[sp++] = lt;
      h = hv;
    }
    need = max(need, sp);
  }
  return need;
}

// Heavy-path adjoint records in processing order (tgp_isa.h). Sequential; one lane.
__device__ void emit_path_records(const int* s_rec, const short* s_sz, const int* s_D, const int* s_E,
                                  const float* vrow, int* stk, uint32_t* recs) {
  int sp = 0, q = 0;
  stk[sp++] = 0;
  while (sp > 0) {
    const int F = stk[--sp];
    int lt;
    for (int h = F; h >= 0;) {
      const int hv = heavy_child(s_rec, s_sz, h, lt);
      const int r = s_rec[h];
      const int ar = rec_arity(r);
      const int c1 = h + 1;
      const int ch[2] = {c1, ar == 2 ? c1 + s_sz[c1] : -1};
      uint32_t pay[2] = {0, 0}, node[2] = {0, 0};
      int kinds[2] = {kKindConst, kKindConst}, vars[2] = {0, 0};
      for (int k = 0; k < ar; ++k) {
        const int c = ch[k];
        const int rc = s_rec[c];
        if (c == hv) {
          kinds[k] = kPathHeavy;
        } else if (c == lt) {
          kinds[k] = kPathLight;
          const int start = s_D[c] & ((1 << kStartBits) - 1);
          const int clen = (s_E[c + s_sz[c]] - s_E[c]) & 0xffff;
          const int ld = (s_D[c] >> kStartBits) & 15;
          pay[k] = (uint32_t)(start | (clen << 12) | (ld << 24));
        } else if (rec_kind(rc) == kTypeVar) {
          kinds[k] = kKindVar;
          vars[k] = rec_var(rc);
        } else {
          kinds[k] = kKindConst;
          pay[k] = __float_as_uint(vrow[c]);
          node[k] = (uint32_t)c;
        }
      }
      const uint32_t w0 = (uint32_t)(rec_op(r) | (ar << 4) | ((rec_modi(r) >= 0 ? 1 : 0) << 6) |
                                     (path_pattern(ar, kinds[0], kinds[1]) << 7) | (vars[0] << 11) | (vars[1] << 15) |
                                     ((hv < 0 ? 1 : 0) << 19) | ((lt >= 0 ? 1 : 0) << 20) |
                                     ((hv >= 0 ? 1 : 0) << 21)) |
                          (node[0] << 22);
      const uint32_t mo = (uint32_t)max(rec_modi(r), 0);
      *(uint4*)(recs + (int64_t)q * kPathWords) = make_uint4(w0, pay[0], pay[1], node[1] | (mo << 16));
      ++q;
      h = hv;
    }
    // light children wait in path order, so the deepest one is taken first
    for (int h = F; h >= 0;) {
      const int hv = heavy_child(s_rec, s_sz, h, lt);
      if (lt >= 0) stk[sp++] = lt;
      h = hv;
    }
  }
}

// LDS per tree: node record (int), prefix sums E and difference array D
// (int, Lmax + 1 entries each, rounded up), subtree size (short), one byte
// per program word and, for gradient calls, a stack of nodes for the
// heavy-path walk (int).
__host__ __device__ constexpr int plan_lpad(int Lmax) { return (Lmax + kWave) / kWave * kWave; }
__host__ __device__ constexpr size_t plan_lds_bytes(int Lmax, bool adj) {
  // + one byte per program word: spill slot + 1 to set on the load at that word, or 0
  return (size_t)plan_lpad(Lmax) * (3 * sizeof(int) + sizeof(short)) + (size_t)(prog_stride(Lmax) + 3) / 4 * 4 +
         (adj ? (size_t)plan_lpad(Lmax) * sizeof(int) : 0);
}


// NCH = node chunks of 64 held in registers while the row is decoded (Lmax <= 64 NCH)
template <int NCH>
__global__ __launch_bounds__(64) void plan_kernel(PlanArgs a) {
  extern __shared__ int s_plan[];
  const int Lp = plan_lpad(a.Lmax);
  int* s_rec = s_plan;
  int* s_E = s_rec + Lp;  // s_E[i] = sum over nodes < i (code size | function count << 16)
  int* s_D = s_E + Lp;    // difference array, then ancestor sums (start | base << 12 | shift << 16)
  short* s_sz = (short*)(s_D + Lp);
  unsigned char* s_pre = (unsigned char*)(s_sz + Lp);  // per program word: spill slot + 1, or 0
  int* s_stk = (int*)(s_pre + (prog_stride(a.Lmax) + 3) / 4 * 4);  // heavy-path walk: stack of path heads

  const int lane = threadIdx.x;
  const int64_t t = blockIdx.x;
  if (t >= a.P) return;
  // the ordering and queue counters of this call: 64 per wave, read only by later kernels
  for (int64_t z = t * kWave + lane; z < a.n_zero; z += a.P * kWave) a.zero[z] = 0;
  const float* trow = a.type + t * a.row_stride;
  const float* vrow = a.value + t * a.row_stride;
  const float* srow = a.size + t * a.row_stride;
  int32_t* info = a.info + t * kInfoStride;
  uint2* prog = a.prog + t * a.pstride;
  const int Lmax = a.Lmax;

  // Issue every global load of the row at once (the padding check reads all
  // Lmax entries, so their count is known before len is).
  float tv[NCH], vv[NCH], sv[NCH];
  const int nch_all = (Lmax + kWave - 1) / kWave;
  int nch_loaded = a.check_tail ? nch_all : 0;
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    const int i = ch * kWave + lane;
    tv[ch] = vv[ch] = sv[ch] = __builtin_nanf("");
    if (ch < nch_loaded && i < Lmax) {
      tv[ch] = trow[i];
      vv[ch] = vrow[i];
      sv[ch] = srow[i];
    }
  }
  const float s0 = a.check_tail ? __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(sv[0]))) : srow[0];

  int status = 0;
  int len = 0;
  if (!(is_intf(s0) && s0 >= 1.0f && s0 <= (float)Lmax)) status = 1;
  else len = (int)s0;

  int n_const = 0, n_modi = 0, max_stack = 0, need0 = 0, prog_len = 0, n_int = 0, adj_fmt = kAdjFmtRecompute;

  if (status == 0) {
    const int scan_end = a.check_tail ? Lmax : len;
    if (!a.check_tail) {
      nch_loaded = (len + kWave - 1) / kWave;
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
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
    for (int ch = 0; ch < NCH; ++ch) {
      const int i = ch * kWave + lane;
      if (ch >= nch_loaded || i >= scan_end) continue;
      const float tq = tv[ch], vq = vv[ch], sq = sv[ch];
      if (i >= len) {
        if (!(isnan(tq) && isnan(vq) && isnan(sq))) err = min(err, 3);
        continue;
      }
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
      const int x = (i < len) ? 1 - rec_arity(s_rec[i]) : 0;
      // suffix sum within the chunk: chunk total - inclusive prefix + own term
      const int incl = wave_incl_scan(x);
      const int tot = lane63(incl);
      const int suf = tot - incl + x;
      if (i < len) best = max(best, suf + carry);
      carry += tot;
    }
    max_stack = wave_max(best);

    // ---- pass 3b (forward programs): second actions along unary chains ----
    // A unary node whose child is a non-Modi unary node is linked to it. The
    // bottom of a run of linked nodes puts its function on a load, on its
    // binary child's last word or on a NOP of its own, as that word's first
    // action; the node above it takes the same word's second action, the one
    // above that emits a NOP, and so on: node i takes a second action when
    // d(i), the number of linked nodes from i down the run, is odd. Runs are
    // contiguous in prefix order, so d comes from a ballot of the unlinked
    // nodes per chunk, chunks taken last to first.
    if (!a.adj) {
      int carry = 0;  // d of the first node of the chunk after this one
      for (int ch = nch - 1; ch >= 0; --ch) {
        const int i = ch * kWave + lane;
        bool link = false;
        if (i < len) {
          const int r = s_rec[i];
          if (rec_kind(r) == kTypeFunc && rec_arity(r) == 1) {
            const int rc = s_rec[i + 1];
            link = rec_kind(rc) == kTypeFunc && rec_arity(rc) == 1 && rec_modi(rc) < 0;
          }
        }
        const unsigned long long stop = __builtin_amdgcn_ballot_w64(!link);
        const unsigned long long ahead = stop >> lane;  // unlinked nodes at or after node i
        const int d = ahead ? __builtin_ctzll(ahead) : (kWave - lane) + carry;
        if (link && (d & 1)) s_rec[i] |= kRecSecond;
        carry = stop ? __builtin_ctzll(stop) : kWave + carry;
      }
    }

    // ---- pass 4: code size and function count of every subtree ----
    // E[i] = sum over nodes j < i of (code words node j emits | 1 << 16 if j is a function)
    {
      int acc = 0;
      for (int ch = 0; ch < nch; ++ch) {
        const int i = ch * kWave + lane;
        int x = 0;
        if (i < len) {
          const int r = s_rec[i];
          if (rec_kind(r) == kTypeFunc) {
            const int c1 = i + 1;
            const bool l1 = rec_kind(s_rec[c1]) != kTypeFunc;
            const bool folded = folds_into_child(r, s_rec[c1], a.adj) || (r & kRecSecond);
            int cc = own_code(r) - (folded ? 1 : 0);
            if (rec_arity(r) == 2) {
              const int r2 = s_rec[c1 + s_sz[c1]];
              const bool l2 = rec_kind(r2) != kTypeFunc;
              // LD of the first leaf, unless a variable operand rides on the op word
              if (l1 && l2 && !preload_fusable(r, s_rec[c1], r2)) cc += 1;
            }
            x = cc | (1 << 16);
          }
        }
        const int incl = wave_incl_scan(x);
        if (i < len) s_E[i + 1] = acc + incl;
        acc += lane63(incl);
      }
      if (lane == 0) s_E[0] = 0;
    }
    for (int ch = 0; ch * kWave <= len; ++ch) {
      const int i = ch * kWave + lane;
      if (i <= len) s_D[i] = 0;
    }
    __syncthreads();

    // ---- pass 5: ancestor terms on child ranges ----
    // For a node whose two children are both function nodes:
    //   forward code: the larger child F runs first (ties: first child), then
    //   its value is spilled to slot base, then the smaller child S runs with
    //   base + 1; every node in S's range starts (code size of F) + 1 words
    //   later and one spill slot higher;
    //   adjoint records: the smaller child's records come first (ties: first
    //   child); when that is the second child, records in its range move back
    //   by the first child's function count and records in the first child's
    //   range move forward by the second child's.
    int max_base = -1;
    for (int ch = 0; ch < nch; ++ch) {
      const int i = ch * kWave + lane;
      if (i >= len) continue;
      const int r = s_rec[i];
      if (rec_kind(r) != kTypeFunc || rec_arity(r) != 2) continue;
      const int c1 = i + 1, z1 = s_sz[c1], c2 = c1 + z1, z2 = s_sz[c2];
      if (rec_kind(s_rec[c1]) != kTypeFunc || rec_kind(s_rec[c2]) != kTypeFunc) continue;
      const bool f1 = z1 >= z2;
      const int F = f1 ? c1 : c2, zF = f1 ? z1 : z2;
      const int S = f1 ? c2 : c1, zS = f1 ? z2 : z1;
      const int csF = (s_E[F + zF] - s_E[F]) & 0xffff;
      const int v = csF + (1 << kStartBits);
      atomicAdd(&s_D[S], v);
      atomicAdd(&s_D[S + zS], -v);
      if (a.adj) atomicOr(&s_rec[S], kRecLight);
      if (a.adj && z2 < z1) {
        const int n1 = (s_E[c2] - s_E[c1]) >> 16, n2 = (s_E[c2 + z2] - s_E[c2]) >> 16;
        atomicAdd(&s_D[c2], -(n1 << 16));
        atomicAdd(&s_D[c2 + z2], n1 << 16);
        atomicAdd(&s_D[c1], n2 << 16);
        atomicAdd(&s_D[c2], -(n2 << 16));
      }
    }
    __syncthreads();
    // inclusive scan of D: at every node, the sum of its ancestors' terms
    {
      int acc = 0;
      for (int ch = 0; ch < nch; ++ch) {
        const int i = ch * kWave + lane;
        const int x = i < len ? s_D[i] : 0;
        const int incl = wave_incl_scan(x);
        if (i < len) {
          const int d = acc + incl;
          s_D[i] = d;
          if (rec_kind(s_rec[i]) == kTypeFunc && rec_arity(s_rec[i]) == 2) {
            // a node that spills uses slot base
            const int c1 = i + 1, c2 = c1 + s_sz[c1];
            if (rec_kind(s_rec[c1]) == kTypeFunc && rec_kind(s_rec[c2]) == kTypeFunc)
              max_base = max(max_base, (d >> kStartBits) & 15);
          }
        }
        acc += lane63(incl);
      }
    }
    __syncthreads();
    const int root = s_rec[0];
    need0 = wave_max(max_base) + 1;
    prog_len = rec_kind(root) == kTypeFunc ? (s_E[len] & 0xffff) + 1 : 2;
    n_int = s_E[len] >> 16;

    // spill map: the first word of every second-evaluated subtree (always a
    // load) first stores A, the first-evaluated sibling's value, to the
    // parent's spill slot
    for (int k = lane; k <= prog_len; k += kWave) s_pre[k] = 0;
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
      const int i = ch * kWave + lane;
      if (i >= len) continue;
      const int r = s_rec[i];
      if (rec_kind(r) != kTypeFunc || rec_arity(r) != 2) continue;
      const int c1 = i + 1, z1 = s_sz[c1], c2 = c1 + z1;
      if (rec_kind(s_rec[c1]) != kTypeFunc || rec_kind(s_rec[c2]) != kTypeFunc) continue;
      const int S = z1 >= s_sz[c2] ? c2 : c1;
      const int stS = s_D[S] & ((1 << kStartBits) - 1);
      if (stS <= prog_len) s_pre[stS] = (unsigned char)(((s_D[i] >> kStartBits) & 15) + 1);
    }
    __syncthreads();

    // ---- pass 6: emission ----
    // the program's last word (the root's, or a folded unary root's child's) also stops the run,
    // so no END word is dispatched
    const int last = prog_len - 2;
    auto emit = [&](int q, uint32_t w, float pay) {
      put(prog, a.pstride, q, q == last ? w | ((uint32_t)kActStop << kActShift) : w, pay);
    };
    if (rec_kind(root) != kTypeFunc) {
      if (lane == 0) {
        int src; float pay;
        leaf_src(root, vrow[0], src, pay);
        emit(0, mkword(kLD + src), pay);  // a leaf root has no spill
      }
    }
    for (int ch = 0; ch < nch; ++ch) {
      const int i = ch * kWave + lane;
      if (i >= len) continue;
      const int r = s_rec[i];
      if (rec_kind(r) != kTypeFunc) continue;
      const int sb = s_D[i];
      const int st = sb & ((1 << kStartBits) - 1), bs = (sb >> kStartBits) & 15;
      // gradient calls: the node's last word captures its value for its parent's path (the
      // parent's light depth: this node's, less one when this node is a light child)
      const int capl = (a.adj && i > 0) ? bs - ((r & kRecLight) ? 1 : 0) : -1;
      auto cap = [capl](uint32_t w) { return capl >= 0 ? with_capture(w, capl) : w; };
      const int cs = (s_E[i + s_sz[i]] - s_E[i]) & 0xffff;
      const int op = rec_op(r);
      const int mo = rec_modi(r);
      const int c1 = i + 1;
      const int r1 = s_rec[c1];
      const bool l1 = rec_kind(r1) != kTypeFunc;
      const bool folded = folds_into_child(r, r1, a.adj) || (r & kRecSecond);
      const int oc = own_code(r) - (folded ? 1 : 0);
      const int pos = st + cs - oc;  // first own instruction
      if (folded) {
        if (mo >= 0) emit(pos, mkword(kACC), __uint_as_float((uint32_t)mo));
        continue;
      }
      if (rec_arity(r) == 1) {
        // over a leaf: its load carries the function; otherwise a NOP does
        uint32_t wd = mkword(kNOP, 0, unary_act(op, mo));
        float pay = 0.0f;
        if (l1) {
          int src;
          leaf_src(r1, vrow[c1], src, pay);
          wd = load_word(src, unary_act(op, mo), s_pre[pos]);
        }
        // the function of a unary parent (node i - 1) that takes the second action
        if (i > 0 && (s_rec[i - 1] & kRecSecond)) {
          const int rp = s_rec[i - 1];
          wd = with_act2(wd, unary_act(rec_op(rp), rec_modi(rp)));
        }
        emit(pos, mo >= 0 ? wd : cap(wd), pay);
        if (mo >= 0) emit(pos + 1, cap(mkword(kACC)), __uint_as_float((uint32_t)mo));
        continue;
      }
      const int z1 = s_sz[c1];
      const int c2 = c1 + z1;
      const int r2 = s_rec[c2];
      const bool l2 = rec_kind(r2) != kTypeFunc;
      // the function of a unary parent folded into this node's last word (node i - 1 is the
      // parent exactly when it is a unary function node)
      const int rp = i > 0 ? s_rec[i - 1] : 0;
      uint32_t pact =
          (i > 0 && folds_into_child(rp, r, a.adj)) ? (uint32_t)unary_act(rec_op(rp), rec_modi(rp)) << kActShift : 0u;
      // and the function of a unary grandparent (node i - 2, over the unary parent) that takes the
      // second action
      if (i > 1 && (s_rec[i - 2] & kRecSecond)) {
        const int rg = s_rec[i - 2];
        pact = with_act2(pact, unary_act(rec_op(rg), rec_modi(rg)));
      }
      int src, aux = 0;
      float pay = 0.0f;
      bool a_first;  // A holds the first operand and src the second
      if (l1 && l2 && preload_fusable(r, r1, r2)) {
        // one word: pre-load the variable operand, the case takes the other leaf
        const bool v1 = rec_kind(r1) == kTypeVar;
        const int pv = v1 ? rec_var(r1) : rec_var(r2);
        leaf_src(v1 ? r2 : r1, vrow[v1 ? c2 : c1], src, pay);
        a_first = v1;
        uint32_t wd = with_preload(mkword(fused_case(op, a_first, src), aux), pv) | pact;
        if (s_pre[pos]) wd = with_spill(wd, s_pre[pos] - 1);
        emit(pos, cap(wd), pay);
        continue;
      } else if (l1 && l2) {
        int s1; float p1;
        leaf_src(r1, vrow[c1], s1, p1);
        emit(st, load_word(s1, 0, s_pre[st]), p1);
        leaf_src(r2, vrow[c2], src, pay);
        a_first = true;
      } else if (l1) {
        leaf_src(r1, vrow[c1], src, pay);
        a_first = false;
      } else if (l2) {
        leaf_src(r2, vrow[c2], src, pay);
        a_first = true;
      } else {
        const bool f1 = z1 >= s_sz[c2];
        int saux;
        src = src_slot(bs, saux);  // the spill happens on the second subtree's first load
        aux = saux;
        a_first = !f1;  // the first-evaluated child is in the slot
      }
      if (mo >= 0) {
        emit(pos, mkword(kTLD + src, aux), pay);
        emit(pos + 1, mkword(kMB + 2 * bin_index(op) + (a_first ? 0 : 1)), 0.0f);
        emit(pos + 2, cap(mkword(kACC) | pact), __uint_as_float((uint32_t)mo));
      } else {
        emit(pos, cap(mkword(fused_case(op, a_first, src), aux) | pact), pay);
      }
    }
    if (lane == 0) {
      // END words: a guard after the last word, and the word the interpreter's one-word lookahead
      // reads
      put(prog, a.pstride, prog_len - 1, mkword(kEND), 0.0f);
      put(prog, a.pstride, prog_len, mkword(kEND), 0.0f);
    }

    // ---- pass 7: adjoint records (gradient calls only) ----
    // Heavy-path format when the sweep's live values fit the adjoint kernel's
    // budget (adj_cap), else the recompute format.
    // Recompute format: record q of a function node is its position in a
    // pre-order walk that visits the smaller child first = (function nodes
    // before it in the array) + (its ancestors' shifts). A record whose node
    // is the later-visited child of a node with two function children takes
    // its adjoint from the pending stack ("pop"); that parent pushes it.
    uint32_t* recs = a.adj ? a.adj + t * (int64_t)Lmax * kAdjWords : nullptr;
    if (a.adj && a.adj_cap > 0) {
      int need = 0;
      if (lane == 0 && rec_kind(root) == kTypeFunc) need = path_need(s_rec, s_sz, s_stk);
      need = __shfl(need, 0, kWave);
      // spill slots beyond the registers' four sit between the captures and the pending
      // adjoints during every run
      if (need + max(need0 - kRegSlots, 0) <= a.adj_cap) adj_fmt = kAdjFmtPath;
    }
    if (adj_fmt == kAdjFmtPath) {
      // a single-leaf tree has no records
      if (lane == 0 && rec_kind(root) == kTypeFunc) emit_path_records(s_rec, s_sz, s_D, s_E, vrow, s_stk, recs);
    } else if (a.adj) {
      for (int ch = 0; ch < nch; ++ch) {
        const int i = ch * kWave + lane;
        if (i >= len) continue;
        const int r = s_rec[i];
        if (rec_kind(r) != kTypeFunc || rec_arity(r) != 2) continue;
        const int c1 = i + 1, z1 = s_sz[c1], c2 = c1 + z1;
        if (rec_kind(s_rec[c1]) != kTypeFunc || rec_kind(s_rec[c2]) != kTypeFunc) continue;
        atomicOr(&s_rec[s_sz[c2] < z1 ? c1 : c2], kRecPop);
      }
      __syncthreads();
      for (int ch = 0; ch < nch; ++ch) {
        const int i = ch * kWave + lane;
        if (i >= len) continue;
        const int r = s_rec[i];
        if (rec_kind(r) != kTypeFunc) continue;
        const int q = (s_D[i] >> 16) + (s_E[i] >> 16);
        if (q < 0 || q >= Lmax) continue;
        const int ar = rec_arity(r);
        const int c1 = i + 1;
        const int c2 = ar == 2 ? c1 + s_sz[c1] : -1;
        uint32_t wv[5] = {0, 0, 0, 0, 0};
        int kinds[2] = {kKindNone, kKindNone}, vars[2] = {0, 0};
        const int ch2[2] = {c1, c2};
        bool both_func = ar == 2;
        for (int k = 0; k < ar; ++k) {
          const int c = ch2[k];
          const int rc = s_rec[c];
          if (rec_kind(rc) == kTypeFunc) {
            kinds[k] = kKindFunc;
            wv[1 + 2 * k] = (uint32_t)(s_D[c] & ((1 << kStartBits) - 1));
            wv[2 + 2 * k] = (uint32_t)((s_E[c + s_sz[c]] - s_E[c]) & 0xffff);
          } else if (rec_kind(rc) == kTypeVar) {
            kinds[k] = kKindVar;
            vars[k] = rec_var(rc);
            both_func = false;
          } else {
            kinds[k] = kKindConst;
            wv[1 + 2 * k] = (uint32_t)c;
            wv[2 + 2 * k] = __float_as_uint(vrow[c]);
            both_func = false;
          }
        }
        const int c2first = (ar == 2 && s_sz[c2] < s_sz[c1]) ? 1 : 0;
        const int pop = (r & kRecPop) ? 1 : 0;
        wv[0] = (uint32_t)(rec_op(r) | (ar << 4) | ((rec_modi(r) >= 0 ? 1 : 0) << 6) | (c2first << 7) |
                           (pop << 8) | ((both_func ? 1 : 0) << 9) | (kinds[0] << 10) | (kinds[1] << 12) |
                           (vars[0] << 14) | (vars[1] << 18) | (max(rec_modi(r), 0) << 22));
        uint4* dst = (uint4*)(recs + (int64_t)q * kAdjWords);
        dst[0] = make_uint4(wv[0], wv[1], wv[2], wv[3]);
        dst[1] = make_uint4(wv[4], 0u, 0u, 0u);
      }
    }
  }

  if (status != 0) {
    len = 0; n_const = 0; n_modi = 0; max_stack = 0; need0 = 0; prog_len = 0; n_int = 0;
    adj_fmt = kAdjFmtRecompute;
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
    info[kInfoAdjFmt] = adj_fmt;
    info[kInfoHdr] = (int32_t)((uint32_t)t | (status != 0 ? kHdrInvalid : 0u) | (n_modi > 0 ? kHdrModi : 0u));
    if (a.out_status) a.out_status[t] = status;
    if (a.out_info) {
      int32_t* o = a.out_info + t * 6;
      o[0] = status; o[1] = len; o[2] = max_stack; o[3] = n_const; o[4] = n_modi; o[5] = bucket;
    }
  }
}

// Counting sort of the trees by length bucket, longest bucket first,
// invalid trees last. Two kernels of 256 trees per workgroup; each
// workgroup aggregates its counts in LDS and issues one global atomic per
// bucket it holds (one cache line of counters would otherwise take one
// atomic per tree).
constexpr int kOrderBlock = 256;
constexpr int kKeys = 17;  // 16 length buckets + invalid trees

__device__ __forceinline__ int order_key(const int32_t* info, int64_t t) {
  const int32_t* inf = info + t * kInfoStride;
  return inf[kInfoStatus] != 0 ? 16 : inf[kInfoBucket];
}

__global__ __launch_bounds__(kOrderBlock) void hist_kernel(OrderArgs a) {
  __shared__ int cnt[kKeys];
  if (threadIdx.x < kKeys) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * kOrderBlock + threadIdx.x;
  if (t < a.P) {
    const int k = order_key(a.info, t);
    if (k < 16) atomicAdd(&cnt[k], 1);
  }
  __syncthreads();
  if (threadIdx.x < 16 && cnt[threadIdx.x] > 0) atomicAdd(&a.hist[threadIdx.x], cnt[threadIdx.x]);
}

__global__ __launch_bounds__(kOrderBlock) void order_kernel(OrderArgs a) {
  __shared__ int cnt[kKeys], base[kKeys];
  if (threadIdx.x < kKeys) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * kOrderBlock + threadIdx.x;
  int k = -1, rank = 0;
  if (t < a.P) {
    k = order_key(a.info, t);
    rank = atomicAdd(&cnt[k], 1);
  }
  __syncthreads();
  if (threadIdx.x < kKeys) {
    const int key = threadIdx.x;
    // first slot of this key: buckets longer than it, or every valid tree for invalid ones
    int off = 0;
    for (int b = 15; b >= 0; --b)
      if (b > key || key == 16) off += a.hist[b];
    base[key] = cnt[key] > 0 ? off + atomicAdd(&a.cursor[key], cnt[key]) : 0;
  }
  __syncthreads();
  if (k >= 0) a.order[base[k] + rank] = a.info[t * kInfoStride + kInfoHdr];
}

hipError_t launch_plan(const PlanArgs& a, hipStream_t s) {
  if (a.P <= 0) return hipSuccess;
  const dim3 grid((unsigned)a.P), block(64);
  const size_t lds = plan_lds_bytes(a.Lmax, a.adj != nullptr);
  if (a.Lmax <= 64) plan_kernel<1><<<grid, block, lds, s>>>(a);
  else if (a.Lmax <= 128) plan_kernel<2><<<grid, block, lds, s>>>(a);
  else if (a.Lmax <= 256) plan_kernel<4><<<grid, block, lds, s>>>(a);
  else if (a.Lmax <= 512) plan_kernel<8><<<grid, block, lds, s>>>(a);
  else plan_kernel<kMaxLmax / kWave><<<grid, block, lds, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_order(const OrderArgs& a, hipStream_t s) {
  if (a.P <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((a.P + kOrderBlock - 1) / kOrderBlock);
  hist_kernel<<<grid, kOrderBlock, 0, s>>>(a);
  order_kernel<<<grid, kOrderBlock, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace tgp
