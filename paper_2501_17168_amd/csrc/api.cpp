// C-ABI entry points: argument checks, workspace layout, launch selection.
//
// Every evaluation call enqueues, on the caller's stream and without any
// allocation or synchronisation:
//   plan (validate, plan figures, compile programs and, for the persistent
//         schedule, zero the bucket counters and work queues)
//   -> [order trees by length bucket, persistent mode only]
//   -> evaluation kernel -> finalize (fitness and per-tree status).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "tgp.h"
#include "tgp_autotune.h"
#include "tgp_kernels.h"

using namespace tgp;

namespace {

constexpr size_t kAlign = 256;
constexpr int kCounters = 64 + kMaxTileQueues * kQueueStride;  // hist[16] | cursor[17] @16 | tile queues @64

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t info, part, order, counters, prog, gwork, total;
};

// part_tiles: point tiles the fitness partials [tiles][P] must hold (0 for plan-only calls)
Layout layout(int64_t P, int Lmax, int64_t part_tiles, int64_t grad_bytes) {
  Layout L{};
  size_t off = 0;
  L.info = off; off = align_up(off + (size_t)P * kInfoStride * sizeof(int32_t));
  L.part = off; off = align_up(off + (size_t)P * part_tiles * sizeof(double));
  L.order = off; off = align_up(off + (size_t)P * sizeof(int32_t));
  L.counters = off; off = align_up(off + kCounters * sizeof(int32_t));
  L.prog = off; off = align_up(off + (size_t)P * prog_stride(Lmax) * sizeof(uint2));
  L.gwork = off; off = align_up(off + (size_t)grad_bytes);
  L.total = off;
  return L;
}

tgp_status check_pop(const tgp_pop* pop) {
  if (!pop) return TGP_E_ARG;
  if (pop->P < 0) return TGP_E_SHAPE;
  if (pop->P > 0 && (!pop->type || !pop->value || !pop->size)) return TGP_E_ARG;
  if (pop->Lmax < 1) return TGP_E_SHAPE;
  if (pop->Lmax > kMaxLmax) return TGP_E_UNSUPPORTED;
  if (pop->row_stride < pop->Lmax) return TGP_E_SHAPE;
  if (pop->P > (int64_t)kHdrTree) return TGP_E_UNSUPPORTED;  // tree index in a 30-bit header field
  return TGP_OK;
}

tgp_status check_data(const tgp_data* d, bool need_y) {
  if (!d) return TGP_E_ARG;
  if (!d->X) return TGP_E_ARG;
  if (d->V < 1 || d->D < 1) return TGP_E_SHAPE;
  if (d->V > kMaxV) return TGP_E_UNSUPPORTED;
  if (d->ldx < d->D) return TGP_E_SHAPE;
  if (d->n_out < 1) return TGP_E_SHAPE;
  if (d->n_out > kMaxOut) return TGP_E_UNSUPPORTED;
  if (need_y && !d->Y) return TGP_E_ARG;
  if (d->Y && d->ldy < d->D) return TGP_E_SHAPE;
  return TGP_OK;
}

tgp_status check_ws(void* ws, size_t ws_bytes, size_t need) {
  if (!ws) return TGP_E_WORKSPACE;
  if (((uintptr_t)ws) % kAlign) return TGP_E_WORKSPACE;
  if (ws_bytes < need) return TGP_E_WORKSPACE;
  return TGP_OK;
}

int vm_for(int V) { return V <= 2 ? 2 : V <= 4 ? 4 : V <= 8 ? 8 : 16; }

// Point tiles of the smallest tile a call may use: 64 lanes x 4 points for the
// forward kernels, x 2 points for the adjoint.
int64_t part_tiles(const tgp_data* d, bool grad) {
  const int64_t tile = grad ? 128 : 256;
  return (d->D + tile - 1) / tile;
}

// Finalize segments per tree: about 32 tiles per thread, at most 16 threads per tree.
int fin_segs(int64_t ntiles) {
  int s = 1;
  while (s < 16 && (int64_t)s * 32 < ntiles) s *= 2;
  return s;
}

// adjoint records: one 32-byte record per function node, Lmax slots per tree
int64_t grad_work_bytes(const tgp_pop* pop, const tgp_data* d) {
  (void)d;
  return (int64_t)pop->P * pop->Lmax * kAdjWords * (int64_t)sizeof(uint32_t);
}

// Pending-stack slots of the adjoint sweep: the sweep descends into the
// smaller child of a node with two function children and parks the larger,
// so the k-th parked entry sits at a node of at least 5 nodes inside a
// subtree of at most len / 2^(k-1): k <= floor(log2 len) <= floor(log2 Lmax).
int pend_slots_for(int Lmax) {
  int lg = 0;
  while ((1 << (lg + 1)) <= Lmax) ++lg;
  return std::max(1, lg);
}

// Values per wave the heavy-path adjoint sweep holds in LDS (captures, waiting light
// children and spill slots beyond the four in registers), by points per lane: 16 at 2
// points (8 KB per wave; it covers every tree of the depth-8 ramped populations) and at 3
// (12 KB per wave: the twelve waves per CU the registers allow fit), 12 at 4 (12 KB per
// wave; 96% of depth-8 ramped trees; 16 at 4 measured slower, its ten waves per CU
// costing more than the recompute sweep of the other 4%). Trees whose sweep needs more go
// to the recompute sweep.
int adj_path_cap(int K) { return K <= 3 ? 16 : 12; }

int device_cus() {
  static int cus = -1;
  static std::mutex m;
  std::lock_guard<std::mutex> g(m);
  if (cus < 0) {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
      cus = p.multiProcessorCount;
    else
      cus = 256;
  }
  return cus;
}


// Schedule named by the environment variable TGP_FORCE_MODE ("tree-major" or 1,
// "point-major" or 2, "persistent" or 3), or TGP_MODE_AUTO when it is unset or
// names none of them.
int forced_mode() {
  const char* e = getenv("TGP_FORCE_MODE");
  if (!e) return TGP_MODE_AUTO;
  if (!strcmp(e, "1") || !strcmp(e, "tree-major")) return TGP_MODE_TREE_MAJOR;
  if (!strcmp(e, "2") || !strcmp(e, "point-major")) return TGP_MODE_POINT_MAJOR;
  if (!strcmp(e, "3") || !strcmp(e, "persistent")) return TGP_MODE_PERSISTENT;
  return TGP_MODE_AUTO;
}

// Fill unset fields of a launch configuration (for a forward call with these
// outputs and prediction flag). TGP_FORCE_MODE overrides the schedule of the
// given, cached or default configuration.
tgp_cfg resolve(const tgp_cfg* in, const tgp_pop* pop, const tgp_data* d, int n_out, bool grad, bool pred) {
  tgp_cfg c{};
  if (in) c = *in;
  if (!in || c.mode == TGP_MODE_AUTO) {
    tgp_cfg cached{};
    if (autotune_lookup(pop, d, n_out, grad, &cached)) {
      const int flags = c.flags;
      c = cached;
      c.flags |= flags;
    }
  }
  if (const int fm = forced_mode()) {
    if (fm != c.mode) c.trees_per_unit = 0;  // trees per unit means something else per schedule
    c.mode = fm;
  }
  // K = 16 exists for up to 2 variables, K = 8 for up to 8, K = 4 for all (and for more than
  // kMaxOutNarrow outputs)
  const int kmax = n_out > kMaxOutNarrow ? 4 : (d->V <= 2 ? 16 : (d->V <= 8 ? 8 : 4));
  if (c.points_per_lane != 4 && c.points_per_lane != 8 && c.points_per_lane != 16) c.points_per_lane = std::min(8, kmax);
  c.points_per_lane = std::min(c.points_per_lane, kmax);
  const int64_t tile = 64LL * c.points_per_lane;
  const int64_t ntiles = (d->D + tile - 1) / tile;
  if (c.mode < TGP_MODE_TREE_MAJOR || c.mode > TGP_MODE_PERSISTENT)
    c.mode = d->D > 16384 ? TGP_MODE_POINT_MAJOR : TGP_MODE_TREE_MAJOR;
  // persistent waves are bound to tiles, one queue per tile
  if (c.mode == TGP_MODE_PERSISTENT && ntiles > kMaxTileQueues) c.mode = TGP_MODE_POINT_MAJOR;
  if (c.block_waves != 1 && c.block_waves != 2 && c.block_waves != 4)
    c.block_waves = (int)std::min<int64_t>(4, std::max<int64_t>(1, ntiles));
  if (c.trees_per_unit < 1) {
    if (c.mode == TGP_MODE_POINT_MAJOR) {
      const int64_t ngroups = (ntiles + c.block_waves - 1) / c.block_waves;
      c.trees_per_unit = (int)std::max<int64_t>(1, (pop->P * ngroups + 8191) / 8192);
    } else {
      // persistent: group trees only when the chunks still fill every resident wave slot;
      // a short queue of long chunks leaves lone waves exposed to program-fetch latency
      const int64_t slots = (int64_t)device_cus() *
                            eval_resident_waves(c.points_per_lane, vm_for(d->V), n_out, pred, c.block_waves);
      c.trees_per_unit = (int)std::min<int64_t>(8, std::max<int64_t>(1, pop->P * ntiles / slots));
    }
  }
  return c;
}


// Enqueue plan (+ order). The plan kernel zeroes the ordering and queue
// counters when the order is wanted; nothing else reads them.
tgp_status enqueue_plan(const tgp_pop* pop, int V, int n_out, const tgp_cfg& c, char* ws,
                        const Layout& L, int32_t* out_info, int32_t* out_status, bool want_order,
                        hipStream_t s, bool want_adj = false, int64_t n_queues = 0, int adj_cap = 0) {
  int32_t* counters = (int32_t*)(ws + L.counters);
  PlanArgs pa{};
  pa.type = pop->type;
  pa.value = pop->value;
  pa.size = pop->size;
  pa.P = pop->P;
  pa.Lmax = pop->Lmax;
  pa.row_stride = pop->row_stride;
  pa.V = V;
  pa.n_out = n_out;
  pa.check_tail = (c.flags & TGP_FLAG_NO_TAIL_CHECK) ? 0 : 1;
  pa.info = (int32_t*)(ws + L.info);
  pa.prog = (uint2*)(ws + L.prog);
  pa.pstride = prog_stride(pop->Lmax);
  pa.adj = want_adj ? (uint32_t*)(ws + L.gwork) : nullptr;
  pa.adj_cap = want_adj ? adj_cap : 0;
  pa.out_info = out_info;
  pa.out_status = out_status;
  pa.zero = want_order ? counters : nullptr;
  pa.n_zero = want_order ? 64 + n_queues * kQueueStride : 0;
  if (launch_plan(pa, s) != hipSuccess) return TGP_E_HIP;
  if (want_order) {
    OrderArgs oa{};
    oa.info = pa.info;
    oa.P = pop->P;
    oa.hist = counters;
    oa.cursor = counters + 16;
    oa.order = (int32_t*)(ws + L.order);
    if (launch_order(oa, s) != hipSuccess) return TGP_E_HIP;
  }
  return TGP_OK;
}

tgp_status forward(const tgp_pop* pop, const tgp_data* d, const tgp_cfg* cfg, int n_out, float* mse,
                   float* pred, int64_t ldp, int32_t* tree_status, void* ws, size_t ws_bytes,
                   hipStream_t s, int loss = kLossSquared) {
  tgp_status st = check_pop(pop);
  if (st) return st;
  st = check_data(d, mse != nullptr);
  if (st) return st;
  if (pred && ldp < d->D) return TGP_E_SHAPE;
  const Layout L = layout(pop->P, pop->Lmax, part_tiles(d, false), 0);
  st = check_ws(ws, ws_bytes, L.total);
  if (st) return st;
  if (pop->P == 0) return TGP_OK;
  const tgp_cfg c = resolve(cfg, pop, d, n_out, false, pred != nullptr);
  char* w = (char*)ws;
  const int K = c.points_per_lane;
  const int64_t tile = 64LL * K;
  const int64_t ntiles = (d->D + tile - 1) / tile;
  const bool persistent = c.mode == TGP_MODE_PERSISTENT;
  st = enqueue_plan(pop, d->V, n_out, c, w, L, nullptr, nullptr, persistent, s, false,
                    (persistent && !(c.flags & TGP_FLAG_STATIC_ORDER)) ? kMaxTileQueues : 0);
  if (st) return st;

  const int bw = c.block_waves;
  EvalArgs ea{};
  ea.X = d->X;
  ea.ldx = d->ldx;
  ea.V = d->V;
  ea.D = d->D;
  ea.Y = mse ? d->Y : nullptr;
  ea.ldy = d->ldy;
  ea.n_out = n_out;
  ea.ny = loss == kLossAccuracy ? 1 : n_out;
  ea.loss = loss;
  ea.info = (const int32_t*)(w + L.info);
  ea.prog = (const uint2*)(w + L.prog);
  ea.pstride = prog_stride(pop->Lmax);
  ea.part = (double*)(w + L.part);
  ea.pred = pred;
  ea.ldp = ldp;
  ea.P = pop->P;
  ea.order = (const int32_t*)(w + L.order);
  ea.mode = c.mode;
  ea.ntiles = (int32_t)ntiles;
  ea.ngroups = (int32_t)((ntiles + bw - 1) / bw);
  ea.tpu = c.mode == TGP_MODE_TREE_MAJOR ? 1 : c.trees_per_unit;
  ea.queue = (int32_t*)(w + L.counters) + 64;
  int64_t grid;
  if (c.mode == TGP_MODE_TREE_MAJOR) {
    grid = pop->P * ea.ngroups;
  } else if (c.mode == TGP_MODE_POINT_MAJOR) {
    grid = ((pop->P + ea.tpu - 1) / ea.tpu) * ea.ngroups;
  } else {
    // persistent waves: as many as the chip holds at once for this instantiation
    const int64_t cap = (int64_t)device_cus() * eval_resident_waves(K, vm_for(d->V), n_out, pred != nullptr, bw);
    const int64_t chunks = (pop->P + ea.tpu - 1) / ea.tpu;
    ea.wpt = (int32_t)std::max<int64_t>(1, std::min<int64_t>(cap / ntiles, chunks));
    ea.dynamic = (c.flags & TGP_FLAG_STATIC_ORDER) ? 0 : 1;
    // up to 8 sub-queues per tile, each served by at least one wave
    ea.nsub = (int32_t)std::max<int64_t>(1, std::min<int64_t>({8, kMaxTileQueues / ntiles, (int64_t)ea.wpt}));
    grid = (ntiles * ea.wpt + bw - 1) / bw;
  }
  const int NO = n_out;
  void* tok = nullptr;
  profile_before(s, &tok);
  const hipError_t le = launch_eval(ea, K, vm_for(d->V), NO, pred != nullptr, bw, grid, s);
  profile_after(s, tok);
  if (le != hipSuccess) return TGP_E_HIP;
  FinalArgs fa{};
  fa.info = ea.info;
  fa.part = ea.part;
  fa.ntiles = (int32_t)ntiles;
  fa.segs = fin_segs(ntiles);
  fa.P = pop->P;
  fa.inv_D = 1.0 / (double)d->D;
  fa.mse = mse;
  fa.tree_status = tree_status;
  if ((mse || tree_status) && launch_finalize(fa, s) != hipSuccess) return TGP_E_HIP;
  return TGP_OK;
}

}  // namespace

extern "C" {

__attribute__((visibility("default"))) size_t tgp_workspace_bytes(const tgp_pop* pop, const tgp_data* data,
                                                                   int32_t n_out, int32_t want_grad) {
  if (check_pop(pop) != TGP_OK) return 0;
  if (data && check_data(data, false) != TGP_OK) return 0;
  if (n_out < 1 || n_out > kMaxOut) return 0;
  int64_t gb = 0;
  if (want_grad && data) gb = grad_work_bytes(pop, data);
  return layout(pop->P, pop->Lmax, data ? part_tiles(data, want_grad != 0) : 0, gb).total;
}

__attribute__((visibility("default"))) tgp_status tgp_plan(const tgp_pop* pop, int32_t V, int32_t n_out,
                                                           const tgp_cfg* cfg, int32_t* info,
                                                           int32_t* tree_status, void* ws, size_t ws_bytes,
                                                           hipStream_t stream) {
  tgp_status st = check_pop(pop);
  if (st) return st;
  if (V < 1 || n_out < 1) return TGP_E_SHAPE;
  if (V > kMaxV || n_out > kMaxOut) return TGP_E_UNSUPPORTED;
  const Layout L = layout(pop->P, pop->Lmax, 0, 0);
  st = check_ws(ws, ws_bytes, L.total);
  if (st) return st;
  if (pop->P == 0) return TGP_OK;
  tgp_cfg c{};
  if (cfg) c = *cfg;
  return enqueue_plan(pop, V, n_out, c, (char*)ws, L, info, tree_status, false, stream);
}

__attribute__((visibility("default"))) tgp_status tgp_eval_mse(const tgp_pop* pop, const tgp_data* data,
                                                               const tgp_cfg* cfg, float* mse,
                                                               int32_t* tree_status, void* ws,
                                                               size_t ws_bytes, hipStream_t stream) {
  if (!mse) return TGP_E_ARG;
  if (!data) return TGP_E_ARG;
  if (data->n_out != 1) return TGP_E_SHAPE;
  return forward(pop, data, cfg, 1, mse, nullptr, 0, tree_status, ws, ws_bytes, stream);
}

__attribute__((visibility("default"))) tgp_status tgp_eval_accuracy(const tgp_pop* pop, const tgp_data* data,
                                                                    const tgp_cfg* cfg, float* accuracy,
                                                                    int32_t* tree_status, void* ws,
                                                                    size_t ws_bytes, hipStream_t stream) {
  if (!accuracy || !data || !data->Y) return TGP_E_ARG;
  if (data->n_out < 2) return TGP_E_SHAPE;
  return forward(pop, data, cfg, data->n_out, accuracy, nullptr, 0, tree_status, ws, ws_bytes, stream,
                 kLossAccuracy);
}

__attribute__((visibility("default"))) tgp_status tgp_eval_multi_output(
    const tgp_pop* pop, const tgp_data* data, const tgp_cfg* cfg, float* mse, float* pred, int64_t ldp,
    int32_t* tree_status, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!mse && !pred) return TGP_E_ARG;
  if (!data) return TGP_E_ARG;
  return forward(pop, data, cfg, data->n_out, mse, pred, ldp, tree_status, ws, ws_bytes, stream);
}

__attribute__((visibility("default"))) tgp_status tgp_eval_mse_grad(
    const tgp_pop* pop, const tgp_data* data, const tgp_cfg* cfg, const float* grad_mse, float* mse,
    float* grad_value, float* grad_X, int32_t* tree_status, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!mse) return TGP_E_ARG;
  tgp_status st = check_pop(pop);
  if (st) return st;
  st = check_data(data, true);
  if (st) return st;
  const int n_out = data->n_out;
  if (n_out > kMaxOutGrad) return TGP_E_UNSUPPORTED;
  const Layout L = layout(pop->P, pop->Lmax, part_tiles(data, true), grad_work_bytes(pop, data));
  st = check_ws(ws, ws_bytes, L.total);
  if (st) return st;
  if (pop->P == 0) return TGP_OK;
  tgp_cfg c{};
  if (cfg) c = *cfg;
  if (!cfg || c.mode == TGP_MODE_AUTO) {
    tgp_cfg cached{};
    if (autotune_lookup(pop, data, n_out, true, &cached)) {
      const int flags = c.flags;
      c = cached;
      c.flags |= flags;
    }
  }
  c.mode = TGP_MODE_POINT_MAJOR;
  // 2 to 4 points per lane: fewer points per lane give more waves per CU, more give less scalar
  // dispatch per point; 3 measured fastest for one output (three waves per SIMD), and
  // multi-output populations (four output accumulators and adjoints) default to 2
  if (c.points_per_lane < 2 || c.points_per_lane > 4) c.points_per_lane = n_out == 1 ? 3 : 2;
  // one wave per workgroup by default: the adjoint's LDS (spill slots and pending stack) bounds
  // residency, and small workgroups pack it best
  if (c.block_waves != 1 && c.block_waves != 2 && c.block_waves != 4) c.block_waves = 1;
  char* w = (char*)ws;
  const int cap = (c.flags & TGP_FLAG_ADJ_RECOMPUTE) ? 0 : adj_path_cap(c.points_per_lane);
  st = enqueue_plan(pop, data->V, n_out, c, w, L, nullptr, nullptr, false, stream, true, 0, cap);
  if (st) return st;
  if (launch_zero_f32(grad_value, pop->P, pop->row_stride, pop->row_stride, stream) != hipSuccess) return TGP_E_HIP;
  if (launch_zero_f32(grad_X, data->V, data->D, data->ldx, stream) != hipSuccess) return TGP_E_HIP;

  const int K = c.points_per_lane;
  const int bw = c.block_waves;
  const int64_t tile = 64LL * K;
  const int64_t ntiles = (data->D + tile - 1) / tile;
  const int64_t ngroups = (ntiles + bw - 1) / bw;
  // trees per unit: enough units for about 64 resident waves per CU, at most 64 trees per unit
  int64_t tpu = c.trees_per_unit;
  if (tpu < 1) tpu = std::min<int64_t>(64, std::max<int64_t>(1, pop->P * ntiles / ((int64_t)device_cus() * 64)));
  AdjArgs aa{};
  aa.X = data->X;
  aa.ldx = data->ldx;
  aa.V = data->V;
  aa.D = data->D;
  aa.Y = data->Y;
  aa.ldy = data->ldy;
  aa.n_out = n_out;
  aa.inv_D = (float)(1.0 / (double)data->D);
  aa.info = (const int32_t*)(w + L.info);
  aa.prog = (const uint2*)(w + L.prog);
  aa.pstride = prog_stride(pop->Lmax);
  aa.adj = (const uint32_t*)(w + L.gwork);
  aa.Lmax = pop->Lmax;
  aa.part = (double*)(w + L.part);
  aa.grad_mse = grad_mse;
  aa.grad_value = grad_value;
  aa.gv_stride = pop->row_stride;
  aa.grad_X = grad_X;
  aa.P = pop->P;
  aa.ntiles = (int32_t)ntiles;
  aa.ngroups = (int32_t)ngroups;
  aa.tpu = (int32_t)tpu;
  aa.pend_slots = pend_slots_for(pop->Lmax);
  aa.cap = cap;
  const int64_t grid = ((pop->P + tpu - 1) / tpu) * ngroups;
  void* tok = nullptr;
  profile_before(stream, &tok);
  const hipError_t le = launch_adjoint(aa, K, vm_for(data->V), bw, grid, stream);
  profile_after(stream, tok);
  if (le != hipSuccess) return TGP_E_HIP;
  FinalArgs fa{};
  fa.info = aa.info;
  fa.part = aa.part;
  fa.ntiles = (int32_t)ntiles;
  fa.segs = fin_segs(ntiles);
  fa.P = pop->P;
  fa.inv_D = 1.0 / (double)data->D;
  fa.mse = mse;
  fa.tree_status = tree_status;
  if (launch_finalize(fa, stream) != hipSuccess) return TGP_E_HIP;
  return TGP_OK;
}

__attribute__((visibility("default"))) tgp_status tgp_autotune(const tgp_pop* pop, const tgp_data* data,
                                                               int32_t n_out, int32_t want_grad, tgp_cfg* out,
                                                               void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!out) return TGP_E_ARG;
  tgp_status st = check_pop(pop);
  if (st) return st;
  st = check_data(data, true);
  if (st) return st;
  const Layout L = layout(pop->P, pop->Lmax, part_tiles(data, want_grad != 0),
                          want_grad ? grad_work_bytes(pop, data) : 0);
  st = check_ws(ws, ws_bytes, L.total);
  if (st) return st;
  return autotune_run(pop, data, n_out, want_grad != 0, out, ws, ws_bytes, stream);
}

__attribute__((visibility("default"))) tgp_status tgp_autotune_cached(const tgp_pop* pop, const tgp_data* data,
                                                                      int32_t n_out, int32_t want_grad,
                                                                      tgp_cfg* out, int32_t* found) {
  if (!out || !found) return TGP_E_ARG;
  tgp_status st = check_pop(pop);
  if (st) return st;
  st = check_data(data, true);
  if (st) return st;
  if (n_out < 1 || n_out > (want_grad ? kMaxOutGrad : kMaxOut)) return TGP_E_UNSUPPORTED;
  *found = autotune_lookup(pop, data, n_out, want_grad != 0, out) ? 1 : 0;
  return TGP_OK;
}

__attribute__((visibility("default"))) const char* tgp_status_str(tgp_status s) {
  switch (s) {
    case TGP_OK: return "ok";
    case TGP_E_ARG: return "invalid argument (null pointer or bad scalar)";
    case TGP_E_SHAPE: return "inconsistent sizes or strides";
    case TGP_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case TGP_E_UNSUPPORTED: return "unsupported size (Lmax > 1024, V > 16, n_out > 12, or n_out > 4 for gradients)";
    case TGP_E_HIP: return "HIP runtime error";
    case TGP_E_TOO_LARGE: return "the call needs more scratch than the static buffer of tgp_eval_mse_noalloc holds";
    case TGP_E_IO: return "autotune cache file cannot be opened or written";
    default: return "unknown status";
  }
}

}  // extern "C"

// forward entry used by the autotuner (same checks as the public calls)
tgp_status tgp_internal_forward(const tgp_pop* pop, const tgp_data* d, const tgp_cfg* cfg, int n_out, float* mse,
                                void* ws, size_t ws_bytes, hipStream_t s) {
  return forward(pop, d, cfg, n_out, mse, nullptr, 0, nullptr, ws, ws_bytes, s);
}
