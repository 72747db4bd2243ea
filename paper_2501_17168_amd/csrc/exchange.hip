// Subtree exchange on the padded prefix encoding (§III-B).
//
// exchange(T_old, k, T_new): with s = k and e = s + size_old[k], every row of
// the result is old[0, s) ++ new ++ old[e, len_old), and in the size row the
// ancestors of k gain dn = size_new[root] - size_old[k]. The result is
// refused (T_old returned) when len_old + dn exceeds the length limit.
//
// A wave owns G consecutive output trees. Lane l first works out the header
// of tree l (rows, node choice, checks, segment bounds, status): the
// dependent loads of G headers are in flight together. The wave then writes
// the rows, reading each header back from its lane, with output column p of
// the row taken from
//   p <  s             old[p]; in the size row an ancestor test
//                      (p < k < p + size_old[p]) adds dn;
//   s <= p < s + nn    donor[j + p - s]   (the inserted subtree, sizes kept);
//   s + nn <= p < len  old[p - dn]        (the old suffix from e on);
//   p >= len           NaN padding.
// Refused and invalid exchanges use the same mapping with s = len = len_old
// (or a verbatim copy of the row, or an all-NaN row), dn = 0, nn = 0.
//
// The work is a copy, bound by HBM bandwidth. Accesses are coalesced across
// the lanes; trees go in groups of U whose loads are issued together, and
// the loads of the next group are issued before the stores of the current
// one, so the wait for a group's data overlaps the previous group's stores
// (the memory counters of a wave retire in issue order). Most written bytes
// are NaN padding, which needs no load; with TGP_XCHG_OUT_PADDED the output
// rows already hold padded trees and only the columns below the larger of
// the new and the current length are written.
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
__device__ inline int lane_i(int x, int l) { return __builtin_amdgcn_readlane(x, l); }
__device__ inline int64_t lane_i64(int64_t x, int l) {
  const uint32_t lo = (uint32_t)lane_i((int)(uint32_t)x, l);
  const uint32_t hi = (uint32_t)lane_i((int)(uint32_t)((uint64_t)x >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Where output tree b comes from: the outcome, the segment bounds, and how
// many columns of its row to write.
struct Hdr {
  int st, s, nn, len, dn, wlen;
  int64_t obase;   // first element of the old row
  int64_t nshift;  // donor element of output column p is nshift + p
};

// The loads come in three passes, each issued before anything waits on it:
// the per-output arguments (rows, node arguments), then the two trees'
// lengths, then the sizes at the two chosen nodes. The checks run after.
__device__ Hdr header(const XchgArgs& a, int64_t b) {
  const float nan = __builtin_nanf("");
  // loads, first pass: the per-output arguments
  const int orow = a.old_row ? a.old_row[b] : (int)b;
  const int nrow = a.new_row ? a.new_row[b] : (int)b;
  const int32_t kraw = ((const int32_t*)a.old_node)[b];
  const int32_t jraw = a.new_node ? ((const int32_t*)a.new_node)[b] : 0;
  const bool padded = a.flags & TGP_XCHG_OUT_PADDED;
  const float prev = padded ? a.out_s[b * a.out_ld] : nan;  // current length of a padded output row
  // loads, second pass: the two trees' lengths
  const bool orow_ok = orow >= 0 && (int64_t)orow < a.old_P;
  const bool nrow_ok = nrow >= 0 && (int64_t)nrow < a.new_P;
  const int64_t obase = orow_ok ? (int64_t)orow * a.old_ld : 0;
  const int64_t nbase = nrow_ok ? (int64_t)nrow * a.new_ld : 0;
  const float l0 = orow_ok ? a.os[obase] : nan;
  const float d0 = nrow_ok ? a.ns[nbase] : nan;
  // node choice
  const bool len_ok = int_in(l0, 1, a.Lo);
  const int n_old = len_ok ? (int)l0 : 0;
  int k = -1;
  if (len_ok) k = (a.flags & TGP_XCHG_OLD_UNIFORM) ? pick_node(__int_as_float(kraw), n_old) : kraw;
  const bool k_in = k >= 0 && k < n_old;
  int j = -1;
  if (nrow_ok) {
    if (a.flags & TGP_XCHG_NEW_UNIFORM) {
      if (int_in(d0, 1, a.Ln)) j = pick_node(__int_as_float(jraw), (int)d0);
    } else {
      j = jraw;
    }
  }
  const bool j_in = j >= 0 && j < a.Ln;
  // loads, third pass: the sizes at the two chosen nodes
  const float szk = k_in ? a.os[obase + k] : nan;
  const float szj = j_in ? a.ns[nbase + j] : nan;

  Hdr h{TGP_XCHG_OK, 0, 0, 0, 0, a.Lo, obase, 0};
  if (!orow_ok) {
    h.st = TGP_XCHG_BAD_OLD;  // no tree to return: all-NaN row
  } else if (!len_ok) {
    h.st = TGP_XCHG_BAD_OLD;  // unreadable length: verbatim copy of the row
    h.s = h.len = a.Lo;
  } else {
    h.s = h.len = n_old;  // the old tree, unless every check below passes
    if (!k_in || !int_in(szk, 1, n_old - k)) {
      h.st = TGP_XCHG_BAD_OLD;
    } else if (!j_in || !int_in(szj, 1, a.Ln - j)) {
      h.st = TGP_XCHG_BAD_DONOR;
    } else {
      const int nk = (int)szk, nsub = (int)szj;
      if (n_old - nk + nsub > a.max_len) {
        h.st = TGP_XCHG_TOO_LONG;
      } else {
        h.s = k;
        h.nn = nsub;
        h.dn = nsub - nk;
        h.len = n_old + h.dn;
        h.nshift = nbase + j - k;
      }
    }
  }
  // with padded output rows, only the first max(new, current) columns change; a row whose
  // current length is unreadable is written whole
  if (padded && int_in(prev, 1, a.Lo)) h.wlen = max(h.len, (int)prev);
  return h;
}

// Registers of U trees' loaded columns.
template <int CH, int U>
struct Group {
  float t[U][CH], v[U][CH], z[U][CH];
  int s[U], len[U], dn[U], wlen[U];
};

template <int CH, int U>
__device__ __forceinline__ void load_group(const XchgArgs& a, const Hdr& h, int t0, int ntrees, int lane,
                                           Group<CH, U>& r) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int t = t0 + u;
    r.s[u] = r.len[u] = r.dn[u] = r.wlen[u] = 0;
    if (t < ntrees) {
      const int s = lane_i(h.s, t), nn = lane_i(h.nn, t), len = lane_i(h.len, t), dn = lane_i(h.dn, t);
      const int64_t obase = lane_i64(h.obase, t), nshift = lane_i64(h.nshift, t);
      r.s[u] = s;
      r.len[u] = len;
      r.dn[u] = dn;
      r.wlen[u] = lane_i(h.wlen, t);
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int p = c * 64 + lane;
        if (c * 64 < len && p < len) {
          const bool from_donor = p >= s && p < s + nn;
          const int64_t q = from_donor ? nshift + p : obase + (p < s ? p : p - dn);
          r.t[u][c] = (from_donor ? a.nt : a.ot)[q];
          r.v[u][c] = (from_donor ? a.nv : a.ov)[q];
          r.z[u][c] = (from_donor ? a.ns : a.os)[q];
        }
      }
    }
  }
}

template <int CH, int U>
__device__ __forceinline__ void store_group(const XchgArgs& a, int64_t b0, int t0, int ntrees, int lane,
                                            const Group<CH, U>& r) {
  const float nan = __builtin_nanf("");
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int t = t0 + u;
    if (t < ntrees) {
      float* __restrict__ out_t = a.out_t + (b0 + t) * a.out_ld;
      float* __restrict__ out_v = a.out_v + (b0 + t) * a.out_ld;
      float* __restrict__ out_s = a.out_s + (b0 + t) * a.out_ld;
      const int s = r.s[u], len = r.len[u], dn = r.dn[u], wlen = r.wlen[u];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int p = c * 64 + lane;
        if (c * 64 < wlen && p < wlen) {
          float tt = nan, vv = nan, zz = nan;
          if (p < len) {
            tt = r.t[u][c];
            vv = r.v[u][c];
            zz = r.z[u][c];
            // ancestor of k: starts before it and its subtree reaches past it
            if (p < s && dn != 0 && zz > (float)(s - p)) zz += (float)dn;
          }
          out_t[p] = tt;
          out_v[p] = vv;
          out_s[p] = zz;
        }
      }
    }
  }
}

// CH: 64-column chunks per row (Lo <= 64 * CH); U: trees per load group; G: trees per wave.
template <int CH, int U, int G>
__global__ __launch_bounds__(64 * kXchgWaves) void exchange_kernel(XchgArgs a) {
  static_assert(G <= 64 && G % (2 * U) == 0, "G trees per wave in pairs of groups");
  const int wave = uniform_i(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t b0 = ((int64_t)blockIdx.x * kXchgWaves + wave) * G;
  if (b0 >= a.B) return;
  const int64_t b = b0 + lane;
  Hdr h{TGP_XCHG_BAD_OLD, 0, 0, 0, 0, 0, 0, 0};
  if (lane < G && b < a.B) {
    h = header(a, b);
    if (a.status) a.status[b] = h.st;
  }
  const int ntrees = (int)min<int64_t>(G, a.B - b0);
  Group<CH, U> r0, r1;
  load_group<CH, U>(a, h, 0, ntrees, lane, r0);
  for (int t0 = 0; t0 < ntrees; t0 += 2 * U) {
    if (t0 + U < ntrees) load_group<CH, U>(a, h, t0 + U, ntrees, lane, r1);
    store_group<CH, U>(a, b0, t0, ntrees, lane, r0);
    if (t0 + U >= ntrees) break;
    if (t0 + 2 * U < ntrees) load_group<CH, U>(a, h, t0 + 2 * U, ntrees, lane, r0);
    store_group<CH, U>(a, b0, t0 + U, ntrees, lane, r1);
  }
}

template <int CH, int U, int G>
hipError_t launch(const XchgArgs& a, hipStream_t s) {
  const int64_t per_block = (int64_t)G * kXchgWaves;
  const int64_t grid = (a.B + per_block - 1) / per_block;
  hipLaunchKernelGGL((exchange_kernel<CH, U, G>), dim3((unsigned)grid), dim3(64 * kXchgWaves), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_exchange(const XchgArgs& a, hipStream_t s) {
  if (a.B <= 0) return hipSuccess;
  // Writing whole rows is bound by bandwidth: wide load groups. Writing only the changed
  // columns of padded rows is bound by latency: lean groups, more waves resident.
  const bool padded = a.flags & TGP_XCHG_OUT_PADDED;
  if (a.Lo <= 64) return padded ? launch<1, 1, 16>(a, s) : launch<1, 8, 32>(a, s);
  if (a.Lo <= 128) return padded ? launch<2, 1, 16>(a, s) : launch<2, 8, 32>(a, s);
  if (a.Lo <= 256) return padded ? launch<4, 1, 16>(a, s) : launch<4, 8, 32>(a, s);
  if (a.Lo <= 512) return launch<8, 2, 16>(a, s);
  if (a.Lo <= 1024) return launch<16, 2, 16>(a, s);
  return hipErrorInvalidValue;
}

}  // namespace tgp
