// Launch wrappers of the kfb device kernels (declarations).
#pragma once
#include "kfb_internal.h"

namespace kfb {

// Size limits of the per-problem stages, checked by the host entry points
// before anything is enqueued: the CholeskyQR factorisation kernels take at
// most MAX_QR_COLS columns, the eigensolver's finalize at most MAX_CORE modes.
constexpr int MAX_QR_COLS = 2048;
constexpr int MAX_CORE = 4096;

// ---- generic strided GEMM:  C = alpha * A(m x k) B(k x n) + beta * C0 -----
// TA/TB/TC/TC0: element types of the operands; TAcc: accumulation type.
// With g.ksplit > 1 the k range is cut into chunks whose partial products go
// to g.Part and are summed in a fixed order by splitk_reduce (deterministic).
template <typename TA, typename TB, typename TC, typename TC0, typename TAcc>
hipError_t gemm(const Rec* recs, int nrec, const GemmArgs& g, hipStream_t s);

// BF16 MFMA variant: A and B are read as FP32 or BF16, rounded to BF16 (and,
// with SPLIT = 3, also the BF16 remainders, so that hi*hi + hi*lo + lo*hi
// recovers ~16 bits), multiplied on MFMA with FP32 accumulation.
template <typename TA, typename TB, typename TC, typename TC0, int SPLIT>
hipError_t gemm_bf16(const Rec* recs, int nrec, const GemmArgs& g, hipStream_t s);

// Tile of the streamlined BF16 kernel for a product shape (tuning table):
// 0 = none (128), 128 or 256; gemm_tile_set returns -1 for invalid arguments.
int gemm_tile_lookup(int m, int n, int k);
int gemm_tile_set(int m, int n, int k, int tile);

// FP32 MFMA variant for FP32 products (A FP32, B FP32 or FP64 rounded to FP32,
// C FP32; two-segment operands and split-K as the FMA engine).
template <typename TB, typename TC0>
hipError_t gemm_f32_mfma(const Rec* recs, int nrec, const GemmArgs& g, hipStream_t s);
// FP64 products on FP64 MFMA (plain operands, no split-K): C = alpha A B + beta C0
hipError_t gemm_f64_mfma(const Rec* recs, int nrec, const GemmArgs& g, hipStream_t s);

// ---- small helpers ---------------------------------------------------------
hipError_t upload_recs(const Rec* host, int nrec, Rec* dev, hipStream_t s);

// dst(i,j) = src(i,j) for an m x n matrix (types converted)
template <typename TD, typename TS>
hipError_t copy2d(const Rec* recs, int nrec, OpRef dst, OpRef src, int m, int n, hipStream_t s);

// Cross-shape grouped update.  pad_in: U_FRONT (dp x r, ld dp) <- the state's
// front U (X_UF: z[0] x r, ld z[1]) and M_IN (dp x n, ld dp) <- the batch (X_M:
// z[0] x s[2] columns, ld z[2]), zero elsewhere.  crop_out: the state's back U
// (X_UB, ld z[1]) <- rows 0..z[0]-1 of U_BACK (dp x N, ld dp).
template <typename TU, typename TM>
hipError_t pad_in(const Rec* recs, int nrec, int64_t dp, int r, int n, hipStream_t s);
template <typename TU>
hipError_t crop_out(const Rec* recs, int nrec, int64_t dp, int N, hipStream_t s);

// fill int32 counters with zero (graph-safe, no memset nodes)
hipError_t zero_words(const Rec* recs, int nrec, int slot, int64_t off, int nwords, hipStream_t s);

// ---- Brand-update stages ---------------------------------------------------
// Upper blocks of the FP64 Gram W = Z^T Z (Z: d x n column-major, ld = d,
// d a multiple of 16), split over ks row chunks with fixed-order summation.
struct GramArgs {
  int n, ks, kchunk;
  int64_t d;
  int64_t off_Z, off_part, off_gram;  // in WS: Z, ks x n x n partials, n x n result
  // optional (>= 0): the reduction also writes R = upper triangle of the result
  // and X = 0 (n x n each), the starting point of the blocked Cholesky
  int64_t off_R = -1, off_X = -1;
};
template <typename TZ>
hipError_t gram_f64(const Rec* recs, int nrec, const GramArgs& a, hipStream_t s);

struct CholArgs {
  int n;
  int64_t off_gram, off_R, off_Rinv;  // n x n column-major in WS
  int64_t off_rowbuf;                  // n elements scratch
  double tau_rel;                      // pivot tolerance relative to max diagonal
  double shift_rel;                    // diagonal shift relative to trace(W) (shifted CholeskyQR)
  int prepped = 0;                     // R = upper(W) and R^-1 = 0 already written (Gram reduction)
};
template <typename T>
hipError_t chol_inv(const Rec* recs, int nrec, const CholArgs& a, hipStream_t s);

struct CoreArgs {
  int r, n, N, Np;
  int64_t off_P, off_P2, off_R;  // P, P2: r x n col-major (TP); R: n x n col-major (TG)
  int64_t off_B, off_V;          // Np x Np col-major (TCore)
  // optional pre-rotated new-direction block (off_preB >= 0): the trailing n
  // columns of B and the trailing n x n block of V are taken from the converged
  // B_R = sqrt(w) R^T V_R and V_R of a smaller eigensolve (preNp x preNp)
  int64_t off_preB = -1, off_preV = -1;
  int preNp = 0;
};
template <typename TCore, typename TP, typename TG, typename TD>
hipError_t assemble_core(const Rec* recs, int nrec, const CoreArgs& a, hipStream_t s);

struct JacArgs {
  int Np, N, b, max_sweeps;
  int64_t off_B, off_V, off_cnt;
  double tol;
};
// One round of the block one-sided Jacobi (all problems in parallel), or, if
// the panel holds every column (Np == 2b), the complete iteration.
template <typename T>
hipError_t jacobi_round(const Rec* recs, int nrec, const JacArgs& a, int sweep, int round,
                        hipStream_t s);
int jacobi_pick_block(int N, int elem_bytes, int* Np);
// Eigensolver configuration: the block width (4, 8, 16, 32), for the kernel
// that holds the panel in LDS, or JAC_STREAMED | width (32: FP64 or FP32;
// 16: FP64 only) for the kernels that read the panel from global memory.
constexpr int JAC_STREAMED = 0x100;
// mixed form with JAC_STREAMED | 32: the iteration runs in FP32 on FP32 MFMA and
// the eigenpairs are refined in FP64 (one Ogita-Aishima step on FP64 MFMA)
constexpr int JAC_REFINE = 0x200;
// padded size for a configuration, or 0 if it is not admissible for N
int jacobi_block_fits(int N, int elem_bytes, int cfg);

struct FinArgs {
  int N, Np, max_sweeps;
  int64_t off_B, off_V, off_cnt, off_lam, off_rank;
  int64_t off_W;  // N x N column-major (TW)
};
template <typename TCore, typename TW, typename TD>
hipError_t finalize_core(const Rec* recs, int nrec, const FinArgs& a, hipStream_t s);
// finalize from eigenvalues in lam[0, N) and eigenvector columns at off_V (N x N,
// scales lam[N + j]); requires Np == N
template <typename TW, typename TD>
hipError_t finalize_sorted(const Rec* recs, int nrec, const FinArgs& a, hipStream_t s);

// Eigenpair refinement (one Ogita-Aishima step) of the FP64 core K (N x N) from
// approximate eigenvectors X: with S = X^T K X and G = X^T X already formed,
// oa_prepare writes the eigenvalue estimates into lam[0, N) (scales lam[N + j]
// = 1) and the partial sums of the cluster threshold; oa_correct forms the
// threshold and overwrites G with the correction E, after which X' = X + X E.
constexpr int OA_BLOCKS = 32;  // workgroups per problem of oa_prepare
struct OaArgs {
  int N;
  int64_t off_K;  // a matrix whose Frobenius norm stands for ||K|| (K itself, or S)
  int64_t off_S, off_G, off_lam;
  int64_t off_delta;  // 1 + 3 OA_BLOCKS doubles: scratch of the threshold's partial sums
};
hipError_t oa_prepare(const Rec* recs, int nrec, const OaArgs& a, hipStream_t s);
hipError_t oa_correct(const Rec* recs, int nrec, const OaArgs& a, hipStream_t s);

// ---- preconditioner helpers -------------------------------------------------
// Per side: c_i = 1/(D_i + lam) - 1/lam for the modes used, stored as
// [c_G / lam_A..., c_G...] at off_cG and [c_A / lam_G..., c_A...] at off_cA
// (TAcc), followed (8-byte aligned) by three doubles: 1/(lam_G lam_A),
// 1/lam_G, 1/lam_A (lam after spectrum continuation when that flag is set).
struct CoefArgs {
  int kG, kA;              // modes used per side
  int64_t off_cG, off_cA;  // coefficient vectors (TAcc) in PWS
  uint32_t flags;
};
template <typename TD, typename TAcc>
hipError_t precond_coefs(const Rec* recs, int nrec, const CoefArgs& a, hipStream_t s);

// in place: X(i,j) *= rowscale[i] * colscale[j] * extra, optional vectors
struct ScaleArgs {
  int m, n;
  OpRef X;
  int row_slot, col_slot;  // -1 = none
  int64_t row_off, col_off;
  int extra_mode;          // 0: none, 1: multiply by 1/rec.s[0], 2: by 1/rec.s[1]
};
template <typename T, typename TS>
hipError_t scale2d(const Rec* recs, int nrec, const ScaleArgs& a, hipStream_t s);

// KFB_EV_ORTHO_DRIFT when a column j < ncols of the d x ncols matrix at
// rec.p[slot] (leading dimension ld) with eigenvalue rec.p[dslot][j] > 0 has
// |sum_i u_ij^2 - 1| > tol
template <typename T, typename TD>
hipError_t ortho_check(const Rec* recs, int nrec, int slot, int dslot, int64_t d, int64_t ld, int ncols, double tol,
                       hipStream_t s);

// KFB_EV_ORTHO_DRIFT into *status when a column j < k of U (d x k, leading
// dimension ld) with D[j] > 0 has |sum_i u_ij^2 - 1| > tol (plain pointers:
// checks a representation handed in by the caller)
template <typename T, typename TD>
hipError_t loaded_norms(const T* U, int64_t ld, int64_t d, int k, const TD* D, double tol, uint32_t* status,
                        hipStream_t s);

// x_i <- sqrt(max(x_i, 0)), i < count, for the vector at rec.p[slot] + off
template <typename T>
hipError_t sqrt_prefix(const Rec* recs, int nrec, int slot, int64_t off, int count, hipStream_t s);

// ---- light correction (B-KFAC-C) ---------------------------------------------
struct GatherArgs {
  int src_slot;
  int64_t lds, d;
  int n;
  int64_t off_idx, off_dst;  // in WS: n column indices (int32), d x n destination
};
template <typename T>
hipError_t gather_cols(const Rec* recs, int nrec, const GatherArgs& a, hipStream_t s);

struct MergeArgs {
  int k, n_crc;
  int64_t off_lam, off_idx, off_src;  // in WS: new eigenvalues (TC), chosen columns, source map (int32)
};
template <typename TC, typename TD>
hipError_t correct_merge(const Rec* recs, int nrec, const MergeArgs& a, hipStream_t s);

struct PermuteArgs {
  int64_t d, ldu;
  int k;
  int64_t off_src, off_ucw;  // in WS: source map, corrected columns (d x n_crc)
};
template <typename T>
hipError_t correct_permute(const Rec* recs, int nrec, const PermuteArgs& a, hipStream_t s);

}  // namespace kfb
