// Internal definitions shared by the kfb HIP translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/kfb.h"

namespace kfb {

typedef __hip_bfloat16 bf16;

// ---------------------------------------------------------------------------
// Per-problem records.  Every stage kernel of a (possibly grouped) call gets a
// device array of Rec, one per independent problem, and resolves its operand
// pointers as rec.p[slot] + byte offset.  Shapes and offsets are shared by
// all problems of one launch and travel by value in the kernel arguments.
// ---------------------------------------------------------------------------
constexpr int REC_SLOTS = 10;
struct Rec {
  void* p[REC_SLOTS];
  double s[4];
  int64_t z[4];  // per-problem sizes of the cross-shape grouped update (width d, ld of U, ld of M)
};

// Slots used by the Brand update.
enum UpdSlot { U_FRONT = 0, U_BACK = 1, M_IN = 2, WS = 3, D_FRONT = 4, D_BACK = 5, STATUS = 6 };
// Slots used by the preconditioner.
// (the factored form also reads A_k from P_AK; G_k comes in P_G)
enum PreSlot { PU_G = 0, PD_G = 1, PU_A = 2, PD_A = 3, P_G = 4, P_S = 5, PWS = 6, P_AK = 7 };

// Slots of the B-R-KFAC calls (with the update's slots): the dense EA factor
// and the Gaussian sketch of the randomized SVD.
enum DenseSlot { B_X = 7, B_OMEGA = 8 };
// Slots of the cross-shape grouped update (with the update's slots, which then
// point at zero-padded copies in the workspace): the state's own front U, the
// caller's batch, the state's own back U.
enum CrossSlot { X_UF = 7, X_M = 8, X_UB = 9 };

// A matrix operand resolved per record: element (i, j) of the logical matrix
// lives at base + i*rs + j*cs, with base = rec.p[slot] + off (bytes).  When
// slot2 >= 0 the operand is split along its k-index (columns of A, rows of B)
// at `split`: indices >= split come from the second segment, re-based at 0.
struct OpRef {
  int32_t slot = -1, slot2 = -1;
  int64_t off = 0, off2 = 0;
  int64_t rs = 0, cs = 0, rs2 = 0, cs2 = 0;
  int32_t split = 0;
};

struct GemmArgs {
  OpRef A, B, C, C0, Part;
  int32_t m = 0, n = 0, k = 0;
  double alpha = 1.0, beta = 0.0;
  int32_t ksplit = 1;  // > 1: partial sums go to Part as [kz][i + j*m]
  int32_t kchunk = 0;  // k range per split (multiple of the tile depth)
  // beta read from device memory (a double at rec.p[beta_slot] + beta_off)
  // when beta_slot >= 0; lets a launch use per-problem values computed on the GPU
  int32_t beta_slot = -1;
  int64_t beta_off = 0;
  // caller's promise: the A and B base pointers are 16-byte aligned (the
  // streamlined BF16 kernel loads them as 16-byte vectors; their strides are
  // checked there; C0 and C are accessed by element)
  int32_t aligned16 = 0;
  // caller's promise: C (and C0 when used) 16-byte aligned; with a unit row or
  // column stride the streamlined kernel then stores (and reads) 4 at once
  int32_t c_vec = 0;
  // caller's promise: B is upper triangular (B(k, j) = 0 for k > j), so a tile
  // of columns [n0, n0 + 128) only needs k < n0 + 128 (FP32 MFMA kernel)
  int32_t b_upper = 0;
  // caller's promise: C = A B is symmetric (A = B^T) and square: the FP64 MFMA
  // kernel computes the tiles on and above the diagonal and mirrors them
  int32_t sym = 0;
  // optional scalings of a single-term BF16 product without split-K:
  // C = alpha diag(r) (A B) + beta C0 diag(c), r and c FP32 vectors at
  // rec.p[rsc_slot] + rsc_off and rec.p[c0cs_slot] + c0cs_off (-1: none)
  int32_t rsc_slot = -1;
  int64_t rsc_off = 0;
  int32_t c0cs_slot = -1;
  int64_t c0cs_off = 0;
};

template <typename T>
__host__ __device__ inline T* at(const Rec& r, int slot, int64_t off) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(r.p[slot]) + off);
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Element type tags for the precision forms.
enum Prec { P64 = KFB_FP64, P32 = KFB_FP32, PMIX = KFB_BF16_MIXED };

}  // namespace kfb
