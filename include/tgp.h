/* tgp.h -- symbolic-regression fitness evaluation for tensorized tree GP on gfx950.
 *
 * The problem (paper: "Enabling Population-Level Parallelism in Tree-Based
 * Genetic Programming for GPU Acceleration"):
 *   - a population of P expression trees in the tensorized prefix encoding of
 *     §III-A: three row-major [P][row_stride] float32 tensors holding, per
 *     tree, node types, node values and subtree sizes of the prefix node
 *     sequence in the first len entries and NaN after them (len = size[0]);
 *   - a data set of D points with V input variables and n_out targets;
 *   - one fitness per tree: the squared error of the tree's prediction
 *     against the targets, averaged over the D points and summed over
 *     outputs (§III-C first paragraph; Alg. 1 maximises its negation).
 *   Multi-output trees use Modi nodes (§IV-C): a Modi node adds its function
 *   value to its output and hands its rightmost child's value to its parent.
 *
 * Node encoding used by this library (the paper fixes no codes):
 *   type 0 = variable (value = input index in [0,V)), 1 = constant,
 *   2 = function (value = op id), 3+o = Modi node for output o (value = op id).
 *   op ids: 0 add, 1 sub, 2 mul, 3 protected div (|b| < 1e-6f gives 1),
 *   4 sin, 5 cos, 6 tanh, 7 exp with the argument clamped to [-20,20],
 *   8 protected log log(|a| + 1e-6f), 9 max, 10 min (NaN operand ignored),
 *   11 tan. A binary node computes f(first child, second child); the first
 *   child sits at index i+1, the second at i+1+size[i+1].
 *   A tree with no Modi node predicts out[0] = root value and 0 for other
 *   outputs; a tree with Modi nodes predicts out[o] = sum of its Modi(o)
 *   contributions (0 if none).
 *
 * Conventions for every call below:
 *   - Pointers inside tgp_pop / tgp_data and all output pointers are DEVICE
 *     pointers owned by the caller. The library never frees or retains them.
 *   - Work is enqueued asynchronously on `stream`; evaluation calls allocate
 *     nothing and never synchronise, so they can be captured in a hipGraph.
 *   - Errors detectable on the host (null pointers, bad sizes, a workspace
 *     that is too small, unsupported sizes) return a negative status at once
 *     and enqueue nothing. Errors in a tree's encoding are found on the
 *     device: that tree gets a non-zero tree_status and a NaN fitness, and
 *     the call still returns TGP_OK.
 *   - `ws` is a caller-owned device workspace of at least
 *     tgp_workspace_bytes(...) bytes, 256-byte aligned. Its contents are
 *     scratch between calls; concurrent calls must not share one workspace.
 *   - Limits: 1 <= Lmax <= 1024, 1 <= V <= 16, 1 <= n_out <= 12 (<= 4 for
 *     gradients; populations of more than 4 outputs run at 4 points per lane),
 *     D >= 1.
 */
#ifndef TGP_H
#define TGP_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tgp_status;
enum {
  TGP_OK = 0,
  TGP_E_ARG = -1,          /* null pointer or invalid scalar argument            */
  TGP_E_SHAPE = -2,        /* inconsistent sizes or strides                       */
  TGP_E_WORKSPACE = -4,    /* workspace null, misaligned or smaller than needed   */
  TGP_E_UNSUPPORTED = -5,  /* sizes beyond the limits listed above                */
  TGP_E_HIP = -6,          /* a HIP runtime call or kernel launch failed          */
  TGP_E_TOO_LARGE = -7,    /* tgp_eval_mse_noalloc: the call needs more scratch than
                              the static buffer holds                             */
  TGP_E_IO = -8            /* autotune cache file: cannot be opened or written     */
};

/* Per-tree status codes written to tree_status[t] (the smallest applicable):
 * 0 ok; 1 size[0] not an integer in [1,Lmax]; 2 NaN inside the first len
 * entries; 3 non-NaN entry at or after len; 4 unknown type code (or Modi
 * output >= n_out); 5 bad op id; 6 bad variable index; 7 subtree sizes
 * inconsistent with the prefix sequence. */
enum { TGP_TREE_OK = 0, TGP_TREE_LEN = 1, TGP_TREE_NAN = 2, TGP_TREE_TAIL = 3,
       TGP_TREE_TYPE = 4, TGP_TREE_OP = 5, TGP_TREE_VAR = 6, TGP_TREE_SIZE = 7 };

/* Population: row-major [P][row_stride] float32 tensors, first Lmax columns used. */
typedef struct tgp_pop {
  const float* type;
  const float* value;
  const float* size;
  int64_t P;
  int32_t Lmax;
  int64_t row_stride;      /* >= Lmax, in elements */
} tgp_pop;

/* Data: X[v*ldx + p] (variable-major), Y[o*ldy + p]; p in [0,D). */
typedef struct tgp_data {
  const float* X;
  int32_t V;
  int64_t D;
  int64_t ldx;             /* >= D */
  const float* Y;          /* may be NULL for prediction-only calls */
  int32_t n_out;
  int64_t ldy;             /* >= D when Y is given */
} tgp_data;

/* Launch configuration. Zero fields mean "default"; a NULL cfg means
 * "autotuned choice for this shape if tgp_autotune has cached one, else
 * the built-in default". The environment variable TGP_FORCE_MODE
 * ("tree-major" or 1, "point-major" or 2, "persistent" or 3) overrides the
 * schedule of every forward evaluation call, whatever the cfg says (the
 * trees per unit then take their default unless the schedule is unchanged);
 * it is read at each call. */
enum { TGP_MODE_AUTO = 0, TGP_MODE_TREE_MAJOR = 1, TGP_MODE_POINT_MAJOR = 2,
       TGP_MODE_PERSISTENT = 3 };
/* Persistent mode: trees are ordered longest length bucket first; the waves
 * bound to each point tile take that order in chunks of trees_per_unit,
 * pulled from the tile's queue (one atomic per chunk, on up to 8 counters
 * per tile) or, with TGP_FLAG_STATIC_ORDER, dealt round-robin in snake
 * order without atomics. */
enum { TGP_FLAG_NO_TAIL_CHECK = 1,     /* skip reading the NaN padding after len */
       TGP_FLAG_STATIC_ORDER = 2,
       TGP_FLAG_ADJ_RECOMPUTE = 4 };   /* gradient calls: recompute sweep for every tree */
typedef struct tgp_cfg {
  int32_t mode;             /* TGP_MODE_*                                           */
  int32_t block_waves;      /* waves per workgroup: 1, 2 or 4                       */
  int32_t points_per_lane;  /* data points per lane: 4, 8 (V <= 8) or 16 (V <= 2)  */
  int32_t trees_per_unit;   /* trees handled per work unit (point-major, persistent) */
  int32_t flags;            /* TGP_FLAG_*                                           */
} tgp_cfg;

/* Bytes of workspace needed by any call on these shapes (n_out outputs;
 * want_grad != 0 adds room for tgp_eval_mse_grad). data may be NULL only to
 * size a tgp_plan call: evaluation calls keep one float64 fitness partial
 * per (tree, tile of 256 points; 128 for gradient calls), which the
 * finalize step adds in a fixed order, so a call's fitness values are
 * bitwise reproducible whatever order its waves ran in. Returns 0 for shapes
 * the library rejects. */
size_t tgp_workspace_bytes(const tgp_pop* pop, const tgp_data* data, int32_t n_out,
                           int32_t want_grad);

/* Validate and plan every tree (§III-A encoding, §III-C evaluation order).
 * info: optional device int32 [P][6] receiving, per tree,
 *   (status, len, max stack depth of the reversed-prefix evaluation,
 *    number of constant nodes, number of Modi nodes, length bucket
 *    = 0 for len 1 else ceil(log2(len))); all zero except status for an
 *   invalid tree.
 * tree_status: optional device int32 [P]. V and n_out bound variable
 * indices and Modi outputs. */
tgp_status tgp_plan(const tgp_pop* pop, int32_t V, int32_t n_out, const tgp_cfg* cfg,
                    int32_t* info, int32_t* tree_status, void* ws, size_t ws_bytes,
                    hipStream_t stream);

/* Fitness of every tree: mse[t] = (1/D) sum_p (out_0(x_p) - Y[p])^2 (n_out = 1).
 * data->n_out must be 1 and data->Y non-null. mse: device float32 [P].
 * tree_status: optional device int32 [P]. */
tgp_status tgp_eval_mse(const tgp_pop* pop, const tgp_data* data, const tgp_cfg* cfg,
                        float* mse, int32_t* tree_status, void* ws, size_t ws_bytes,
                        hipStream_t stream);

/* tgp_eval_mse for callers that cannot allocate device memory (code under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, results and launches as tgp_eval_mse, but no workspace:
 * the scratch comes from a static device array of TGP_NOALLOC_SCRATCH_BYTES
 * (32 MiB) that each device running the library holds until the process
 * ends. The call allocates nothing (its first call on a device looks up the
 * array's address once); the caller still passes the inputs and outputs.
 * A call whose workspace would exceed the array returns TGP_E_TOO_LARGE and
 * enqueues nothing: tgp_workspace_bytes(pop, data, 1, 0) must be at most
 * TGP_NOALLOC_SCRATCH_BYTES (for example up to 5,298 trees of Lmax 256 on
 * 2,000 points; 2,000 such trees need 12.7 MB). All calls on one device share its array, which
 * keeps the last call's contents (nothing in it needs to start at zero:
 * every call writes what it reads), so calls that overlap in time on one
 * device, on any streams, race and must not be issued. */
#define TGP_NOALLOC_SCRATCH_BYTES (32u << 20)
tgp_status tgp_eval_mse_noalloc(const tgp_pop* pop, const tgp_data* data, const tgp_cfg* cfg,
                                float* mse, int32_t* tree_status, hipStream_t stream);

/* Multi-output evaluation (§IV-C). With data->Y: mse[t] = sum over the
 * n_out outputs of the mean squared error (mse may be NULL to skip).
 * pred (optional, device float32): pred[(t*n_out + o)*ldp + p] receives
 * out_o of tree t at point p (ldp >= D); invalid trees get NaN.
 * At least one of mse / pred must be non-null. */
tgp_status tgp_eval_multi_output(const tgp_pop* pop, const tgp_data* data, const tgp_cfg* cfg,
                                 float* mse, float* pred, int64_t ldp, int32_t* tree_status,
                                 void* ws, size_t ws_bytes, hipStream_t stream);

/* Classification fitness (the classification domain of §V-D; multi-output
 * trees of §IV-C): data->n_out = C classes (2..12), and row 0 of data->Y
 * holds each point's class label (a float32 integer in [0, C); other values
 * never match). Tree t predicts class c(x) = the first index of the largest
 * of its C outputs, a NaN output counting below every number, and
 * accuracy[t] = (1/D) * #{p : c(x_p) == label_p}; NaN for an invalid tree.
 * The argmax is taken on the float32 outputs. accuracy: device float32 [P].
 * tree_status: optional device int32 [P]. */
tgp_status tgp_eval_accuracy(const tgp_pop* pop, const tgp_data* data, const tgp_cfg* cfg, float* accuracy,
                             int32_t* tree_status, void* ws, size_t ws_bytes, hipStream_t stream);

/* Fitness and its gradient (not in the paper; reverse-mode sweep over the
 * prefix tree with subtree values recomputed, nothing stored per point).
 * The sweep walks each tree by heavy paths: one run of the program gives the
 * fitness and the values along the root's path of larger children, and every
 * smaller child's subtree is run once more for its own path. A tree whose
 * sweep would hold more values per lane at once than the sweep's LDS budget
 * (16 at 2 or 3 points per lane, 12 at 4; deep trees) is swept
 * instead node by node, re-running each function child's subtree;
 * TGP_FLAG_ADJ_RECOMPUTE in cfg->flags sends every tree that way. Both give
 * the same gradient up to the order of float32 sums.
 * grad_mse: optional device float32 [P], upstream dL/dmse_t (NULL = all ones).
 * grad_value: optional device float32 [P][row_stride], overwritten with
 *   dL/dvalue (non-zero only at constant nodes; zero elsewhere and for
 *   invalid trees).
 * grad_X: optional device float32 [V][ldx], overwritten with
 *   sum_t dL/dmse_t * dmse_t/dX.
 * data->n_out outputs (1..4), as in tgp_eval_multi_output: mse[t] sums the
 * outputs' mean squared errors, a Modi node for output o passes
 * dL/dout_o * df/dchild to its children (§IV-C), and Y must hold n_out rows.
 * mse: device float32 [P]. cfg: mode is ignored (the sweep is point-major);
 * points_per_lane 2, 3 or 4 (anything else: 3 for one output, 2 for several),
 * block_waves and trees_per_unit as for the forward calls. */
tgp_status tgp_eval_mse_grad(const tgp_pop* pop, const tgp_data* data, const tgp_cfg* cfg,
                             const float* grad_mse, float* mse, float* grad_value,
                             float* grad_X, int32_t* tree_status, void* ws, size_t ws_bytes,
                             hipStream_t stream);

/* Time the candidate launch configurations on this population and data,
 * keep the fastest in a process-wide cache keyed by the shape, and return
 * it in *out. Synchronises the stream; not capturable. With want_grad the
 * gradient call is tuned instead (its points per lane, 2 to 4, workgroup
 * shape and trees per unit;
 * the workspace sized with want_grad), and later
 * tgp_eval_mse_grad calls on this shape with a NULL or AUTO cfg use it.
 * Allocates and frees temporary device buffers. */
tgp_status tgp_autotune(const tgp_pop* pop, const tgp_data* data, int32_t n_out,
                        int32_t want_grad, tgp_cfg* out, void* ws, size_t ws_bytes,
                        hipStream_t stream);

/* Persistent autotune cache (not in the paper). The cache key is the device's
 * architecture name and compute-unit count, P, Lmax, V, D, n_out and the
 * gradient flag. A cache file holds one JSON object per line:
 *   {"arch":"gfx950","cus":256,"P":..,"Lmax":..,"V":..,"D":..,"n_out":..,
 *    "grad":0|1,"mode":..,"block_waves":..,"points_per_lane":..,
 *    "trees_per_unit":..,"flags":..}
 * in exactly that key order. If the environment variable TGP_AUTOTUNE_CACHE
 * names a file, the library reads it on its first cache lookup or tuning run
 * and appends every new tgp_autotune result to it.
 * tgp_autotune_cache_load: read a cache file into the process's cache (later
 *   entries for a key replace earlier ones). A line that does not parse
 *   exactly, or holds a value outside the limits (an unknown mode or flag, a
 *   points-per-lane or workgroup size the call does not run, sizes beyond the
 *   limits above), is skipped and counted in *n_rejected; such shapes keep
 *   their default or tuned configuration. Both counts are optional.
 *   TGP_E_IO if the file cannot be opened. Needs no device.
 * tgp_autotune_cache_save: write every cached entry to path (through a
 *   temporary file renamed over it). TGP_E_IO if it cannot be written. */
tgp_status tgp_autotune_cache_load(const char* path, int32_t* n_loaded, int32_t* n_rejected);
/* The configuration a call without one would take from the cache for this
 * population, data, output count and gradient flag on the current device:
 * *found = 1 and *out filled, or *found = 0. Reads the TGP_AUTOTUNE_CACHE file
 * first if this process has not yet. Argument errors as tgp_autotune. */
tgp_status tgp_autotune_cached(const tgp_pop* pop, const tgp_data* data, int32_t n_out,
                               int32_t want_grad, tgp_cfg* out, int32_t* found);
tgp_status tgp_autotune_cache_save(const char* path);

/* ---- subtree exchange (§III-B) ----
 * exchange(T_old, k, T_new) replaces the subtree rooted at node k of T_old
 * by T_new: with s = k and e = s + size_old[k], each row of the result is
 * old[0, s), then T_new's row, then old[e, len_old); in the size row every
 * ancestor of k first gains dn = size_new[root] - size_old[k]. When
 * len_old + dn exceeds the length limit the exchange is refused and T_old
 * is returned. One-point crossover inserts a subtree of another parent,
 * subtree mutation a freshly generated tree, hoist mutation a subtree of
 * T_old itself.
 *
 * Batch form: output tree b is exchange(old tree old_row[b], node k_b,
 * subtree of donor tree new_row[b] rooted at node j_b). Node arguments are
 * int32 indices, or, for a side whose TGP_XCHG_*_UNIFORM flag is set,
 * float32 u in [0, 1) mapped to node floor(u * len) (product rounded to
 * float32, clamped to len - 1; len = size[0] of that tree), so a random node
 * of each tree is drawn on the device from caller-supplied uniforms.
 *
 * Per-output status (first failing check wins), and the row written:
 *   TGP_XCHG_BAD_OLD   old_row[b] outside [0, old->P): all-NaN row;
 *                      size_old[0] not an integer in [1, old->Lmax]: the
 *                      old row copied verbatim;
 *                      k outside [0, len_old) (or u not in [0, 1)), or
 *                      size_old[k] not an integer in [1, len_old - k]: T_old;
 *   TGP_XCHG_BAD_DONOR new_row[b] outside [0, donor->P); with the uniform
 *                      flag, size_new[0] not an integer in [1, donor->Lmax]
 *                      or u not in [0, 1); j outside [0, donor->Lmax), or
 *                      size_new[j] not an integer in [1, donor->Lmax - j]:
 *                      T_old;
 *   TGP_XCHG_TOO_LONG  len_old + dn > max_len: T_old;
 *   TGP_XCHG_OK        the exchanged tree.
 * "T_old" is the old row's first len_old entries followed by NaN (for a
 * valid tree, the row itself). The exchanged tree is what the definition
 * gives for valid old and donor trees (tgp_plan status 0); for others only
 * the checks above are made. */
enum { TGP_XCHG_OK = 0, TGP_XCHG_TOO_LONG = 1, TGP_XCHG_BAD_OLD = 2, TGP_XCHG_BAD_DONOR = 3 };
/* TGP_XCHG_OUT_PADDED: the output rows already hold valid padded trees (for
 * example the population of two generations back, when two buffers take
 * turns); only the first max(new length, current length) columns of each
 * row are written, which gives the same rows as a full write. A row whose
 * current size[0] is not an integer in [1, old->Lmax] is written whole. */
enum { TGP_XCHG_OLD_UNIFORM = 1, TGP_XCHG_NEW_UNIFORM = 2, TGP_XCHG_OUT_PADDED = 4 };

typedef struct tgp_exchange {
  const int32_t* old_row;  /* device [B]; NULL: output b uses old tree b             */
  const void* old_node;    /* device [B]; int32 k, or float32 u with OLD_UNIFORM     */
  const int32_t* new_row;  /* device [B]; NULL: donor tree b                         */
  const void* new_node;    /* device [B]; int32 j, or float32 u with NEW_UNIFORM;
                              NULL (index mode only): node 0, the whole donor tree  */
  int64_t B;               /* number of output trees, 0 <= B <= 2^31 - 1             */
  int32_t max_len;         /* length limit, 1 <= max_len <= old->Lmax                */
  int32_t flags;           /* TGP_XCHG_OLD_UNIFORM | _NEW_UNIFORM | _OUT_PADDED      */
} tgp_exchange;

/* Enqueue B subtree exchanges on `stream` (no allocation, no synchronisation;
 * capturable). old and donor are populations as above (they may be the same
 * population). Output: device float32 rows out_type/out_value/out_size
 * [B][out_stride], out_stride >= old->Lmax, of which the first old->Lmax
 * columns are written; they must not overlap any input. xstatus: optional
 * device int32 [B] receiving the TGP_XCHG_* code of each output. Host-side
 * argument errors return a negative status and enqueue nothing. */
tgp_status tgp_subtree_exchange(const tgp_pop* old, const tgp_pop* donor, const tgp_exchange* x,
                                float* out_type, float* out_value, float* out_size, int64_t out_stride,
                                int32_t* xstatus, hipStream_t stream);

/* ---- random tree generation ----
 * Grow, full and ramped half-and-half initialisation, one tree per thread
 * (the paper initialises one individual per GPU thread), written as padded
 * rows (§III-A). Random numbers are Philox4x32-10 (Salmon et al., SC 2011)
 * with counter (tree, attempt, position, 0) and key (seed low 32 bits,
 * seed high 32 bits); the four words of one call serve one node, mapped to
 * [0, 1) as (w >> 8) * 2^-24. Tree index = first_tree + row.
 *
 * Per tree: depth limit d and method are d_max and the configured method,
 * or, for RAMPED, d_min + (tree / 2) mod (d_max - d_min + 1), full for even
 * trees and grow for odd ones. Slots are filled in prefix order; a slot at
 * depth h holds a function when h < d and (full, or h == 0, or u0 < p_func),
 * else a terminal. A function's op is funcs[floor(u1 * n_funcs)]; a
 * terminal is a constant lo + (hi - lo) * u2 (float32, separately rounded)
 * when u1 < p_const, else variable floor(u2 * V). Products are float32 and
 * indices are clamped to the last entry. A tree that outgrows Lmax is
 * drawn again with the next attempt number; after attempts_per_depth
 * failures at one depth limit the limit drops by one (depth 0 is a single
 * terminal, which always fits). */
enum { TGP_GEN_GROW = 0, TGP_GEN_FULL = 1, TGP_GEN_RAMPED = 2 };

typedef struct tgp_gen_cfg {
  int32_t method;              /* TGP_GEN_*                                            */
  int32_t depth_min;           /* ramped only; 0 <= depth_min <= depth_max             */
  int32_t depth_max;           /* <= 30                                                */
  int32_t V;                   /* input variables, 1..16                               */
  const int32_t* funcs;        /* HOST array of n_funcs distinct op ids (0..11)        */
  int32_t n_funcs;             /* 1..12                                                */
  float const_lo, const_hi;    /* constants drawn from [const_lo, const_hi), finite    */
  float p_func;                /* < 0: default n_funcs / (n_funcs + V + 1) (float32)   */
  float p_const;               /* < 0: default 1 / (V + 1) (float32)                   */
  int32_t attempts_per_depth;  /* >= 1                                                 */
  uint64_t seed;
  int64_t first_tree;          /* >= 0, first_tree + P <= 2^32                         */
} tgp_gen_cfg;

/* Enqueue the generation of P trees on `stream` (no allocation, no
 * synchronisation). out_type/out_value/out_size: device float32 rows
 * [P][out_stride], first Lmax columns written (1 <= Lmax <= 1024,
 * out_stride >= Lmax). attempts: optional device int32 [P], the number of
 * attempts each tree took. Host-side argument errors return a negative
 * status and enqueue nothing. */
tgp_status tgp_generate(const tgp_gen_cfg* g, int64_t P, int32_t Lmax, float* out_type, float* out_value,
                        float* out_size, int64_t out_stride, int32_t* attempts, hipStream_t stream);

/* Static description of a status code. */
const char* tgp_status_str(tgp_status s);

/* ---- measurement helpers (not part of the evaluated method) ----
 * tgp_op_cost: cost of op id `op` (0..11) in vector-ALU issue slots per
 *   application and lane, measured on the current device: a straight-line
 *   compiled loop applies the operator to 8 independent streams of spread
 *   inputs per lane (fresh values each step, x in [-8, 8), [-20, 20) for
 *   exp, so lanes take data-dependent branches as on real data); its time
 *   above the same loop without the operator, divided by the time of one
 *   issue slot (from the same loop with 32 dependent FMAs added), is the
 *   cost. Synchronous; it allocates and frees a small
 *   device buffer. Returns TGP_E_ARG for a bad op or null output.
 * tgp_profile(enable): while enabled, every forward and gradient call
 *   records a HIP event pair around its evaluation- or sweep-kernel launch
 *   on the caller's stream (pairs are created once and reused after each
 *   read; disabling releases the unused ones).
 * tgp_profile_read: waits for the recorded events, returns the summed
 *   kernel time in ms and the number of launches, and clears the record. */
/* tgp_op_apply: y[i] = unary operator `op` (sin, cos, tanh, exp, log or
 *   tan: op ids 4-8 and 11, with the protection of exp and log) applied to
 *   x[i] exactly as the evaluation kernels apply it; x and y are device
 *   float32 [n]. Enqueued on `stream`; TGP_E_ARG for another op, a negative
 *   n or a null array. For checking the operators' accuracy. */
tgp_status tgp_op_cost(int32_t op, double* slots);
tgp_status tgp_op_apply(int32_t op, const float* x, float* y, int64_t n, hipStream_t stream);
tgp_status tgp_profile(int32_t enable);
tgp_status tgp_profile_read(double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* TGP_H */
