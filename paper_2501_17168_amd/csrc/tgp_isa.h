// Internal instruction set of the wave-uniform tree interpreter.
//
// The plan kernel compiles every valid tree into a short program for an
// accumulator machine; the evaluation kernels run it with one wave per
// (tree, point tile), every lane holding K data points. Registers per lane:
//   A      accumulator (K values)
//   T      second-operand register (K)
//   R0..R3 spill slots in registers (K each); slots 4..7 live in LDS ("RM")
//   X0..   the tile of input variables (K per variable)
//   r      Modi contribution register (K), O[o] output accumulators (K each)
// A program evaluates the tree bottom-up in post-order, taking the child
// that needs more spill slots first (Sethi-Ullman order), so a tree of at
// most 1024 nodes never needs more than 8 slots. Leaves are not
// instructions of their own: they are source operands of their parent.
//
// Each instruction is 8 bytes: word = case | aux << 16, then a float
// payload (the constant of a C source). aux holds an LDS slot (0..7) or a
// Modi output index. Programs are straight-line and end with END, so the
// interpreter's program counter only moves forward and always reaches END.
#pragma once
#include <stdint.h>

namespace tgp {

// ---- node encoding (tensor level) ----
constexpr int kTypeVar = 0, kTypeConst = 1, kTypeFunc = 2, kTypeModi0 = 3;
constexpr int kOpAdd = 0, kOpSub = 1, kOpMul = 2, kOpDiv = 3, kOpSin = 4, kOpCos = 5, kOpTanh = 6,
              kOpExp = 7, kOpLog = 8, kOpMax = 9, kOpMin = 10, kOpTan = 11, kNumOps = 12;
__host__ __device__ constexpr int op_arity(int op) {
  return (op == kOpAdd || op == kOpSub || op == kOpMul || op == kOpDiv || op == kOpMax || op == kOpMin) ? 2 : 1;
}
// index among binary ops (add sub mul div max min) and unary ops (sin cos tanh exp log tan)
__host__ __device__ constexpr int bin_index(int op) { return op <= kOpDiv ? op : op - 5; }
__host__ __device__ constexpr int un_index(int op) { return op == kOpTan ? 5 : op - 4; }

constexpr float kDivTau = 1e-6f;   // protected division threshold
constexpr float kLogEps = 1e-6f;   // protected log offset
constexpr float kExpClamp = 20.0f; // exp argument clamp

// ---- limits ----
constexpr int kMaxLmax = 1024;
constexpr int kMaxV = 16;
constexpr int kMaxOut = 12;        // outputs (Modi output index in 4 bits of the node record)
constexpr int kMaxOutNarrow = 4;   // outputs with exact-count accumulator instantiations, any K
constexpr int kMaxOutGrad = 4;     // outputs of gradient calls
constexpr int kRegSlots = 4;       // spill slots held in registers
constexpr int kMaxSlots = 8;       // spill slots in total (need <= 8 for len <= 1024)

// ---- source operands ----
// 0: constant payload; 1..4: R0..R3; 5: LDS slot in aux; 6..21: X0..X15
// (variables last, so the cases a kernel instantiated for fewer variables
// cannot reach form one contiguous range per group)
constexpr int kSrcC = 0, kSrcR0 = 1, kSrcRM = 5, kSrcX0 = 6, kNumSrc = 22;

// ---- instruction word ----
// A program is a sequence of 8-byte words: 32 bits of code, then a float
// payload (the constant of a constant source). Code bits:
//    0..8   case (below): the data movement or arithmetic on A
//    9..11  spill slot, 12 spill flag: before the case, store A to that
//           slot (the value of a first-evaluated subtree, saved while its
//           sibling is computed; always carried by the sibling's first word)
//   16..21  action after the case: kActUn | unary index applies a unary
//           function to A (to the Modi register r instead with kActModi);
//           kActStop ends the program
//   22..24  aux: LDS slot of a kSrcRM source (kACC carries its output
//           index in the payload instead)
//   25      pre-load flag, 26..29 variable: after the spill and before the
//           case, A = x[variable] (a binary node over two leaves is then
//           one word)
//   13      capture flag, with a 4-bit level in bits 14..15 (low) and
//           30..31 (high): set on the last word of every non-root function
//           node (after it, A holds the value the node hands to its parent);
//           the level is the light depth of the node's parent (below). Only
//           the adjoint's interpreter reads these bits: a run at level l
//           pushes A on the capture stack after every word whose level is l.
//           Forward programs (never captured) use the same bits for a second
//           action: bit 13 set, the 4-bit field holding a unary index
//           (bits 0..2) and kActModi; it applies after the first action (a
//           unary node over a unary node whose function rides on a load or
//           on a binary node's last word).
constexpr int kLD = 0;                    // A = src
constexpr int kTLD = kLD + kNumSrc;       // T = src
constexpr int kADD = kTLD + kNumSrc;      // A = A + src
constexpr int kMUL = kADD + kNumSrc;      // A = A * src
constexpr int kMAX = kMUL + kNumSrc;      // A = max(A, src)
constexpr int kMIN = kMAX + kNumSrc;      // A = min(A, src)
constexpr int kSUBA = kMIN + kNumSrc;     // A = A - src
constexpr int kSUBR = kSUBA + kNumSrc;    // A = src - A
constexpr int kDIVA = kSUBR + kNumSrc;    // A = A / src (protected)
constexpr int kDIVR = kDIVA + kNumSrc;    // A = src / A (protected)
constexpr int kMB = kDIVR + kNumSrc;      // Modi binary: r = op(A,T) (ord 0) or op(T,A) (ord 1),
                                          // A = the second operand's value: kMB + 2*bin_index + ord
constexpr int kACC = kMB + 12;            // O[o] += r, o in the payload word
constexpr int kNOP = kACC + 1;            // nothing (the action bits do the work)
constexpr int kEND = kNOP + 1;            // stop
constexpr int kNumCases = kEND + 1;

constexpr int kCaseBits = 9, kSpillShift = 9, kSpillFlag = 1 << 12, kActShift = 16, kAuxShift = 22;
constexpr int kAuxMask = 7, kPreLoadFlag = 1 << 25, kPreLoadShift = 26;
constexpr uint32_t kCapFlag = 1u << 13;
// actions (bits 16..21 of a word)
constexpr int kActModi = 8, kActUn = 16, kActStop = 32;

__host__ __device__ constexpr uint32_t mkword(int c, int aux = 0, int act = 0) {
  return (uint32_t)c | ((uint32_t)act << kActShift) | ((uint32_t)aux << kAuxShift);
}
__host__ __device__ constexpr uint32_t with_spill(uint32_t w, int slot) {
  return w | (uint32_t)kSpillFlag | ((uint32_t)slot << kSpillShift);
}
__host__ __device__ constexpr int word_case(uint32_t w) { return (int)(w & ((1u << kCaseBits) - 1)); }
__host__ __device__ constexpr uint32_t with_preload(uint32_t w, int var) {
  return w | (uint32_t)kPreLoadFlag | ((uint32_t)var << kPreLoadShift);
}
__host__ __device__ constexpr uint32_t with_capture(uint32_t w, int level) {
  return w | kCapFlag | ((uint32_t)(level & 3) << 14) | ((uint32_t)(level >> 2) << 30);
}
__host__ __device__ constexpr int capture_level(uint32_t w) { return (int)(((w >> 14) & 3u) | ((w >> 28) & 12u)); }
// the second action of a forward-program word (act = kActUn | index, with kActModi for a Modi node)
constexpr uint32_t kAct2Flag = kCapFlag;
__host__ __device__ constexpr uint32_t with_act2(uint32_t w, int act) { return with_capture(w, act & 15); }
__host__ __device__ constexpr int act2_of(uint32_t w) { return kActUn | capture_level(w); }

// ---- per-tree plan record (int32 fields) ----
// info[t*kInfoStride + k]
// kInfoAdjFmt: the adjoint-record format written for the tree (gradient calls):
// kAdjFmtRecompute or kAdjFmtPath, below.
constexpr int kInfoStatus = 0, kInfoLen = 1, kInfoMaxStack = 2, kInfoNConst = 3, kInfoNModi = 4,
              kInfoBucket = 5, kInfoProgLen = 6, kInfoNeed = 7, kInfoNInternal = 8, kInfoHdr = 9,
              kInfoAdjFmt = 10, kInfoStride = 11;

// tree header word (info[kInfoHdr]) and persistent order entries: tree index in the low 30 bits
constexpr uint32_t kHdrInvalid = 1u << 31, kHdrModi = 1u << 30, kHdrTree = (1u << 30) - 1;

// ---- adjoint records ----
// One record (8 x uint32) per function node, in pre-order with the smaller
// child visited first, so that at most log2(len) adjoints wait on the
// pending stack. Children are either leaves (a variable or a constant) or
// function nodes, whose value is recomputed by re-running their contiguous
// code range [start, start + len) of the forward program.
//   w0 = op | arity << 4 | modi << 6 | c2_first << 7 | pop << 8 | push << 9
//        | kind1 << 10 | kind2 << 12 | var1 << 14 | var2 << 18 | Modi output << 22
//   w1, w2 = child 1: code start, code length (function) or node index,
//            constant bits (constant)
//   w3, w4 = child 2, likewise; w5..w7 = 0
// kind: 0 function, 1 variable, 2 constant, 3 absent (unary node).
// pop: the node's adjoint comes from the pending stack (it is the second
// visited function child of its parent); otherwise it is the "current"
// adjoint left by the previous record. push: the node's second-visited
// child's adjoint goes to the pending stack.
constexpr int kAdjWords = 8;
constexpr int kKindFunc = 0, kKindVar = 1, kKindConst = 2, kKindNone = 3;

// ---- adjoint records, heavy-path format ----
// The heavy child of a function node is its larger function child (the one
// its code evaluates first; ties: the first child), or its only function
// child; the other function child of a node with two is light. A node's
// light depth counts the light edges from the root to it. Following heavy
// children from a node F (F = the root or a light child) gives F's path.
// Running F's code once at level light_depth(F) captures, in code order, the
// values of the function children of every node on F's path: deepest first,
// the heavy child before the light one, so the node at the top of the path
// finds its children's values at the top of the capture stack.
// Records, one per function node, come in processing order: F's path top
// down; then, deepest light child first, each light child's own path and
// what hangs below it (the light children wait on a pending stack).
// A record is 4 words (kPathWords; the records of a tree are kPathWords apart):
//   w0 = op | arity << 4 | modi << 6 | pattern << 7 | var_a << 11
//        | var_b << 15 | end_of_path << 19 | has_light << 20 | has_heavy << 21
//        | (node index of a constant child a) << 22
//   w1 = child a's payload: a constant's bits, or for a light child
//        code start | code length << 12 | light depth << 24
//   w2 = child b's payload, likewise
//   w3 = node index of a constant child b | Modi output << 16
// pattern: the kinds of the children (heavy, light, variable, constant), one
// of kPat*: for a binary node (child a, child b), for a unary node child a.
constexpr int kPathHeavy = 0, kPathLight = 3, kPathWords = 4;
enum : int { kPatHL = 0, kPatLH, kPatHV, kPatVH, kPatHC, kPatCH, kPatVV, kPatVC, kPatCV, kPatCC,
             kPatH, kPatV, kPatC, kNumPat };
__host__ __device__ constexpr int path_pattern(int arity, int kind_a, int kind_b) {
  // kinds: kPathHeavy, kKindVar, kKindConst, kPathLight
  return arity == 1 ? (kind_a == kPathHeavy ? kPatH : kind_a == kKindVar ? kPatV : kPatC)
       : kind_a == kPathHeavy ? (kind_b == kPathLight ? kPatHL : kind_b == kKindVar ? kPatHV : kPatHC)
       : kind_a == kPathLight ? kPatLH
       : kind_a == kKindVar ? (kind_b == kPathHeavy ? kPatVH : kind_b == kKindVar ? kPatVV : kPatVC)
       : (kind_b == kPathHeavy ? kPatCH : kind_b == kKindVar ? kPatCV : kPatCC);
}
// per-tree record format
constexpr int kAdjFmtRecompute = 0, kAdjFmtPath = 1;

// program capacity per tree, in instructions (bound: 2*len + #unary nodes + 2 <= 3*Lmax + 2)
__host__ __device__ constexpr int64_t prog_stride(int Lmax) { return ((3 * (int64_t)Lmax + 2) + 7) / 8 * 8; }

}  // namespace tgp
