// Argument block and launcher of the tree-generation kernel (generate.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tgp {

constexpr int kMaxGenDepth = 30;  // bounds the per-thread slot and open-node stacks

struct GenArgs {
  int64_t P;           // rows to write
  int64_t first_tree;  // tree index of row 0 (the first counter word)
  int32_t Lmax;
  int32_t V;
  int32_t method;      // TGP_GEN_*
  int32_t d_min, d_max;
  int32_t n_funcs;
  int32_t funcs[16];   // op ids
  float lo, hi;        // constant range [lo, hi)
  float p_func, p_const;
  int32_t attempts_per_depth;
  uint32_t key0, key1;
  float* out_t;
  float* out_v;
  float* out_s;
  int64_t out_ld;
  int32_t* attempts;   // optional [P]
};

hipError_t launch_generate(const GenArgs& a, hipStream_t s);

}  // namespace tgp
