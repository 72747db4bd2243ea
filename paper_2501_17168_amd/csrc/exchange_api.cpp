// C-ABI entry of the subtree exchange (§III-B): host-side checks, then one
// kernel launch on the caller's stream.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "tgp.h"
#include "tgp_exchange.h"

using namespace tgp;

namespace {

constexpr int32_t kMaxRowLen = 1024;   // the library-wide Lmax limit
constexpr int64_t kMaxRows = INT32_MAX;

tgp_status check_side(const tgp_pop* p) {
  if (!p) return TGP_E_ARG;
  if (p->P < 0) return TGP_E_SHAPE;
  if (p->P > 0 && (!p->type || !p->value || !p->size)) return TGP_E_ARG;
  if (p->Lmax < 1 || p->row_stride < p->Lmax) return TGP_E_SHAPE;
  if (p->Lmax > kMaxRowLen || p->P > kMaxRows) return TGP_E_UNSUPPORTED;
  return TGP_OK;
}

// Byte range [lo, hi) of rows x stride floats, the last row holding `cols`.
struct Range {
  uintptr_t lo, hi;
};

Range range_of(const void* p, int64_t rows, int64_t stride, int64_t cols) {
  const uintptr_t lo = (uintptr_t)p;
  if (!p || rows <= 0) return {lo, lo};
  return {lo, lo + (uintptr_t)(((rows - 1) * stride + cols) * (int64_t)sizeof(float))};
}

bool overlap(Range a, Range b) { return a.lo < a.hi && b.lo < b.hi && a.lo < b.hi && b.lo < a.hi; }

}  // namespace

extern "C" {

__attribute__((visibility("default"))) tgp_status tgp_subtree_exchange(
    const tgp_pop* old, const tgp_pop* donor, const tgp_exchange* x, float* out_type, float* out_value,
    float* out_size, int64_t out_stride, int32_t* xstatus, hipStream_t stream) {
  tgp_status st = check_side(old);
  if (st) return st;
  st = check_side(donor);
  if (st) return st;
  if (!x) return TGP_E_ARG;
  if (x->B < 0) return TGP_E_SHAPE;
  if (x->B > kMaxRows) return TGP_E_UNSUPPORTED;
  if (x->flags & ~(TGP_XCHG_OLD_UNIFORM | TGP_XCHG_NEW_UNIFORM | TGP_XCHG_OUT_PADDED)) return TGP_E_ARG;
  if (x->max_len < 1 || x->max_len > old->Lmax) return TGP_E_SHAPE;
  if (x->B == 0) return TGP_OK;
  if (!x->old_node || !out_type || !out_value || !out_size) return TGP_E_ARG;
  if ((x->flags & TGP_XCHG_NEW_UNIFORM) && !x->new_node) return TGP_E_ARG;
  if (out_stride < old->Lmax) return TGP_E_SHAPE;

  // outputs are written while other waves read the inputs: no overlap allowed
  const Range outs[3] = {range_of(out_type, x->B, out_stride, old->Lmax),
                         range_of(out_value, x->B, out_stride, old->Lmax),
                         range_of(out_size, x->B, out_stride, old->Lmax)};
  const Range ins[6] = {range_of(old->type, old->P, old->row_stride, old->Lmax),
                        range_of(old->value, old->P, old->row_stride, old->Lmax),
                        range_of(old->size, old->P, old->row_stride, old->Lmax),
                        range_of(donor->type, donor->P, donor->row_stride, donor->Lmax),
                        range_of(donor->value, donor->P, donor->row_stride, donor->Lmax),
                        range_of(donor->size, donor->P, donor->row_stride, donor->Lmax)};
  for (int i = 0; i < 3; ++i) {
    for (int j = i + 1; j < 3; ++j)
      if (overlap(outs[i], outs[j])) return TGP_E_ARG;
    for (const Range& r : ins)
      if (overlap(outs[i], r)) return TGP_E_ARG;
  }

  XchgArgs a{};
  a.ot = old->type;
  a.ov = old->value;
  a.os = old->size;
  a.old_P = old->P;
  a.Lo = old->Lmax;
  a.old_ld = old->row_stride;
  a.nt = donor->type;
  a.nv = donor->value;
  a.ns = donor->size;
  a.new_P = donor->P;
  a.Ln = donor->Lmax;
  a.new_ld = donor->row_stride;
  a.old_row = x->old_row;
  a.new_row = x->new_row;
  a.old_node = x->old_node;
  a.new_node = x->new_node;
  a.B = x->B;
  a.max_len = x->max_len;
  a.flags = x->flags;
  a.out_t = out_type;
  a.out_v = out_value;
  a.out_s = out_size;
  a.out_ld = out_stride;
  a.status = xstatus;
  return launch_exchange(a, stream) == hipSuccess ? TGP_OK : TGP_E_HIP;
}

}  // extern "C"
