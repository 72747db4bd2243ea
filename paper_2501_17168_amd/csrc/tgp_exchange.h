// Argument block and launcher of the subtree-exchange kernel (exchange.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tgp {

// Output tree b is built from old tree old_row[b] (node from old_node) and the
// donor subtree of tree new_row[b] (node from new_node).
struct XchgArgs {
  const float* ot;
  const float* ov;
  const float* os;
  int64_t old_P;
  int32_t Lo;
  int64_t old_ld;
  const float* nt;
  const float* nv;
  const float* ns;
  int64_t new_P;
  int32_t Ln;
  int64_t new_ld;
  const int32_t* old_row;
  const int32_t* new_row;
  const void* old_node;
  const void* new_node;
  int64_t B;
  int32_t max_len;
  int32_t flags;
  float* out_t;
  float* out_v;
  float* out_s;
  int64_t out_ld;
  int32_t* status;
};

hipError_t launch_exchange(const XchgArgs& a, hipStream_t s);

}  // namespace tgp
