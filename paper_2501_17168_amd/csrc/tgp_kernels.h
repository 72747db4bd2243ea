// Kernel argument blocks and launch helpers shared by the library's HIP sources.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tgp.h"
#include "tgp_isa.h"

namespace tgp {

struct PlanArgs {
  const float* type;
  const float* value;
  const float* size;
  int64_t P;
  int32_t Lmax;
  int64_t row_stride;
  int32_t V;
  int32_t n_out;
  int32_t check_tail;
  int32_t* info;        // [P][kInfoStride]
  uint2* prog;          // [P][prog_stride(Lmax)]
  int64_t pstride;
  uint32_t* adj;        // optional [P][Lmax][kAdjWords] adjoint records
  int32_t adj_cap;      // values the heavy-path sweep may hold per wave (0: recompute format only)
  int32_t* out_info;    // optional [P][6]
  int32_t* out_status;  // optional [P]
  int32_t* zero;        // optional counters the plan zeroes (their readers run after it)
  int64_t n_zero;
};

// persistent work queues: one counter per point tile, each in its own
// 64-byte line (waves bound to one tile share its counter)
constexpr int kMaxTileQueues = 1024;  // counters for all tiles' sub-queues
constexpr int kQueueStride = 16;

struct OrderArgs {
  const int32_t* info;
  int64_t P;
  int32_t* hist;        // [16] valid trees per length bucket, zero on entry
  int32_t* cursor;      // [17], zero on entry (16 buckets + invalid trees)
  int32_t* order;       // [P] tree headers (index | kHdr* flags), longest length bucket first
};

// Per-point fitness terms: squared error summed over the outputs, or 1 when
// the argmax of the outputs equals the point's class label.
constexpr int kLossSquared = 0, kLossAccuracy = 1;

struct EvalArgs {
  const float* X;
  int64_t ldx;
  int32_t V;
  int64_t D;
  const float* Y;       // null in prediction-only mode
  int64_t ldy;
  int32_t n_out;
  int32_t ny;           // rows of Y read: n_out (squared error) or 1 (class labels)
  int32_t loss;         // kLossSquared or kLossAccuracy
  const int32_t* info;
  const uint2* prog;
  int64_t pstride;
  double* part;         // fitness partials [ntiles][P]: part[tile * P + t], one per (tree, tile)
  float* pred;          // optional [P][n_out][ldp]
  int64_t ldp;
  int64_t P;
  const int32_t* order; // optional tree order (persistent mode)
  int32_t mode;         // 1 tree-major, 2 point-major, 3 persistent
  int32_t ntiles;       // point tiles of 64*K points
  int32_t ngroups;      // tile groups of block_waves tiles (tree-major / point-major)
  int32_t tpu;          // trees per unit
  int32_t* queue;       // persistent: ntiles chunk counters kQueueStride ints apart, zero on entry
  int32_t wpt;          // persistent: waves bound to each tile
  int32_t dynamic;      // persistent: chunks from the tile counters (else round-robin)
  int32_t nsub;         // persistent dynamic: sub-queues (counters) per tile
};

struct AdjArgs {
  const float* X;
  int64_t ldx;
  int32_t V;
  int64_t D;
  const float* Y;       // Y[o * ldy + p], o < n_out
  int64_t ldy;
  int32_t n_out;        // 1..4; Modi outputs of multi-output trees
  float inv_D;
  const int32_t* info;
  const uint2* prog;
  int64_t pstride;
  const uint32_t* adj;  // adjoint records [P][Lmax][kAdjWords]
  int32_t Lmax;
  double* part;         // fitness partials [ntiles][P], as for the forward kernel
  const float* grad_mse;  // optional [P]
  float* grad_value;    // optional [P][gv_stride], zeroed beforehand
  int64_t gv_stride;
  float* grad_X;        // optional [V][ldx], zeroed beforehand
  int64_t P;
  int32_t ntiles;
  int32_t ngroups;
  int32_t tpu;
  int32_t pend_slots;   // pending-adjoint stack entries per wave (recompute sweep)
  int32_t cap;          // LDS values per wave of the heavy-path sweep (0: not launched)
};

// Fitness from the per-(tree, tile) partials, summed in a fixed order (tiles
// split into `segs` interleaved segments summed in order, segments added in
// order), so repeated calls give bitwise identical results.
struct FinalArgs {
  const int32_t* info;
  const double* part;   // [ntiles][P]; read only when mse is requested
  int32_t ntiles;
  int32_t segs;         // 1..16 segments per tree (a power of two)
  int64_t P;
  double inv_D;
  float* mse;
  int32_t* tree_status;
};

// launchers (defined in plan.hip / eval.hip)
hipError_t launch_plan(const PlanArgs& a, hipStream_t s);
hipError_t launch_order(const OrderArgs& a, hipStream_t s);
hipError_t launch_eval(const EvalArgs& a, int K, int VM, int NO, bool pred, int block_waves,
                       int64_t grid, hipStream_t s);
// waves of this evaluation-kernel instantiation resident on one CU at once
int eval_resident_waves(int K, int VM, int NO, bool pred, int block_waves);
hipError_t launch_finalize(const FinalArgs& a, hipStream_t s);
hipError_t launch_adjoint(const AdjArgs& a, int K, int VM, int block_waves, int64_t grid, hipStream_t s);
hipError_t launch_zero_f32(float* p, int64_t rows, int64_t cols, int64_t ld, hipStream_t s);

// optional event pair around the evaluation kernel (measure.hip)
void profile_before(hipStream_t s, void** token);
void profile_after(hipStream_t s, void* token);

}  // namespace tgp
