// Subtree exchange on the padded prefix encoding (§III-B).
//
// exchange(T_old, k, T_new): with s = k and e = s + size_old[k], every row of
// the result is old[0, s) ++ new ++ old[e, len_old), and in the size row the
// ancestors of k gain dn = size_new[root] - size_old[k]. The result is
// refused (T_old returned) when len_old + dn exceeds the length limit.
//
// One wave builds one output tree. Its header (rows, nodes, segment bounds,
// status) is wave-uniform and comes from a handful of scalar loads; the
// lanes then write the output row column by column, each column's source
// chosen by three comparisons:
//   p <  s             old[p]; in the size row an ancestor test
//                      (p < k < p + size_old[p]) adds dn;
//   s <= p < s + nn    donor[j + p - s]   (the inserted subtree, sizes kept);
//   s + nn <= p < len  old[p - dn]        (the old suffix from e on);
//   p >= len           NaN padding.
// Refused and invalid exchanges run the same loop with s = len = len_old
// (or a verbatim copy of the row, or an all-NaN row), dn = 0, nn = 0.
// The work is a copy: each column is loaded once and stored once, so the
// kernel is bound by HBM bandwidth; loads and stores are coalesced across
// the lanes of a wave and the loop is unrolled for memory-level parallelism.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "tgp.h"
#include "tgp_exchange.h"

namespace tgp {
namespace {

constexpr int kXchgWaves = 4;  // waves (output trees) per workgroup

__device__ inline bool int_in(float x, int lo, int hi) {
  // an integer in [lo, hi]; false for NaN and infinities
  return x == floorf(x) && x >= (float)lo && x <= (float)hi;
}

// Node floor(u * n) (float32 product), clamped to n - 1; -1 when u is not in [0, 1).
__device__ inline int pick_node(float u, int n) {
  if (!(u >= 0.0f && u < 1.0f)) return -1;
  const float prod = u * (float)n;
  return min((int)floorf(prod), n - 1);
}

__device__ inline int uniform_i(int x) { return __builtin_amdgcn_readfirstlane(x); }

__global__ __launch_bounds__(64 * kXchgWaves) void exchange_kernel(XchgArgs a) {
  const int wave = uniform_i(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t b = (int64_t)blockIdx.x * kXchgWaves + wave;
  if (b >= a.B) return;

  // ---- wave-uniform header: which rows, which segments, which outcome
  int st = TGP_XCHG_OK;
  int s = 0, nn = 0, len = 0, dn = 0;
  const int orow = a.old_row ? a.old_row[b] : (int)b;
  int64_t obase = 0, nbase = 0;
  if (orow < 0 || (int64_t)orow >= a.old_P) {
    st = TGP_XCHG_BAD_OLD;  // no tree to return: all-NaN row
  } else {
    obase = (int64_t)orow * a.old_ld;
    const float* osz = a.os + obase;
    const float l0 = osz[0];
    if (!int_in(l0, 1, a.Lo)) {
      st = TGP_XCHG_BAD_OLD;  // unreadable length: verbatim copy of the row
      s = len = a.Lo;
    } else {
      const int n_old = (int)l0;
      s = len = n_old;  // the old tree, unless every check below passes
      const int k = (a.flags & TGP_XCHG_OLD_UNIFORM) ? pick_node(((const float*)a.old_node)[b], n_old)
                                                     : ((const int32_t*)a.old_node)[b];
      if (k < 0 || k >= n_old || !int_in(osz[k], 1, n_old - k)) {
        st = TGP_XCHG_BAD_OLD;
      } else {
        const int nrow = a.new_row ? a.new_row[b] : (int)b;
        int j = -1;
        if (nrow >= 0 && (int64_t)nrow < a.new_P) {
          nbase = (int64_t)nrow * a.new_ld;
          const float* nsz = a.ns + nbase;
          if (a.flags & TGP_XCHG_NEW_UNIFORM) {
            const float d0 = nsz[0];
            if (int_in(d0, 1, a.Ln)) j = pick_node(((const float*)a.new_node)[b], (int)d0);
          } else {
            j = a.new_node ? ((const int32_t*)a.new_node)[b] : 0;
          }
          if (j >= 0 && j < a.Ln && !int_in(nsz[j], 1, a.Ln - j)) j = -1;
          if (j >= a.Ln) j = -1;
        }
        if (j < 0) {
          st = TGP_XCHG_BAD_DONOR;
        } else {
          const int nk = (int)osz[k];
          const int nsub = (int)a.ns[nbase + j];
          if (n_old - nk + nsub > a.max_len) {
            st = TGP_XCHG_TOO_LONG;
          } else {
            s = k;
            nn = nsub;
            dn = nsub - nk;
            len = n_old + dn;
            nbase += j;
          }
        }
      }
    }
  }
  s = uniform_i(s);
  nn = uniform_i(nn);
  len = uniform_i(len);
  dn = uniform_i(dn);
  if (a.status && lane == 0) a.status[b] = st;

  // ---- the output row
  const float nan = __builtin_nanf("");
  float* __restrict__ out_t = a.out_t + b * a.out_ld;
  float* __restrict__ out_v = a.out_v + b * a.out_ld;
  float* __restrict__ out_s = a.out_s + b * a.out_ld;
  const float fdn = (float)dn;
  const int donor_end = s + nn;
  const int64_t nshift = nbase - s;  // donor element of output column p: nshift + p
#pragma unroll 4
  for (int p = lane; p < a.Lo; p += 64) {
    float t = nan, v = nan, z = nan;
    if (p < len) {
      const bool from_donor = p >= s && p < donor_end;
      const int64_t q = from_donor ? nshift + p : obase + (p < s ? p : p - dn);
      t = (from_donor ? a.nt : a.ot)[q];
      v = (from_donor ? a.nv : a.ov)[q];
      z = (from_donor ? a.ns : a.os)[q];
      // ancestor of k: starts before it and its subtree reaches past it
      if (p < s && dn != 0 && z > (float)(s - p)) z += fdn;
    }
    out_t[p] = t;
    out_v[p] = v;
    out_s[p] = z;
  }
}

}  // namespace

hipError_t launch_exchange(const XchgArgs& a, hipStream_t s) {
  if (a.B <= 0) return hipSuccess;
  const int64_t grid = (a.B + kXchgWaves - 1) / kXchgWaves;
  hipLaunchKernelGGL(exchange_kernel, dim3((unsigned)grid), dim3(64 * kXchgWaves), 0, s, a);
  return hipGetLastError();
}

}  // namespace tgp
