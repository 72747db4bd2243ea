// Launch-configuration autotuner: measured choice among the evaluation
// schedules, cached per problem shape for the life of the process.
#pragma once
#include "tgp.h"

namespace tgp {

// Cached configuration for this shape, if any.
bool autotune_lookup(const tgp_pop* pop, const tgp_data* d, int n_out, bool grad, tgp_cfg* out);

// Time the candidates on the caller's data (synchronises `s`), cache and return the fastest:
// forward schedules, or with `grad` the gradient call's points per lane, workgroup shape and trees
// per unit.
tgp_status autotune_run(const tgp_pop* pop, const tgp_data* d, int n_out, bool grad, tgp_cfg* out, void* ws,
                        size_t ws_bytes, hipStream_t s);

}  // namespace tgp

// Forward evaluation with explicit configuration (defined with the C entry points).
tgp_status tgp_internal_forward(const tgp_pop* pop, const tgp_data* d, const tgp_cfg* cfg, int n_out,
                                float* mse, void* ws, size_t ws_bytes, hipStream_t s);
