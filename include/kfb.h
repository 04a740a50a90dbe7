/*
 * kfb — Brand-update K-factor library for MI355X (gfx950).
 *
 * One K-factor (the input-side A or output-side Gamma factor of one
 * fully-connected layer) is held as a low-rank eigen-representation
 * U diag(D) U^T of its exponentially averaged value (Section 2.1, the EA
 * K-factor).  kfb_brand_update performs one B-KFAC step on it (Algorithm 4:
 * truncate to rank r, then the Symmetric Brand update of Algorithm 3 with the
 * batch scaled by sqrt(w)); kfb_precondition applies the regularised inverses
 * of the two factors of a layer on both sides of that layer's gradient
 * (Algorithm 1, its inverse-application lines; Algorithm 8 for the cost).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All matrix arguments are DEVICE pointers unless stated otherwise.
 *  - Column-major: a d x n batch M has element (i, j) at M[i + j*ldm].  A
 *    row-major PyTorch tensor of shape [n, d] is exactly this with ldm = d.
 *  - Row-major: the layer gradient G and the step S are d_out x d_in with
 *    element (i, j) at G[i*ldg + j] (the PyTorch weight-gradient layout).
 *  - Memory is owned by the caller.  The library never allocates or frees
 *    device memory; it records pointers.  kfb_state_bytes / *_workspace_bytes
 *    give the sizes to allocate (256-byte aligned pointers required).
 *  - Work is enqueued on the given HIP stream and is asynchronous; inputs must
 *    stay valid until it completes (the same contract as a PyTorch kernel).
 *  - A handle is not thread-safe; different handles may be driven from
 *    different host threads and streams.
 *  - Return codes are synchronous argument/launch checks.  Numerical events
 *    (non-finite input, Cholesky breakdown, rank deficiency) are recorded
 *    asynchronously in a device status word read by kfb_state_status.
 *
 * Precision forms
 *  KFB_FP64        every buffer and operation in FP64.
 *  KFB_FP32        every buffer and operation in FP32 (plain form).
 *  KFB_BF16_MIXED  batch M is BF16; U is kept in FP32; projection, residual
 *                  and rotation products run on BF16 MFMA with FP32
 *                  accumulation; the CholQR Gram/Cholesky, the core
 *                  eigensolve and D are FP64.  G and S are FP32.
 */
#ifndef KFB_H
#define KFB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kfb_state_s* kfb_state_t;
typedef void* kfb_stream_t; /* a hipStream_t; NULL = the default stream */

enum kfb_precision { KFB_FP64 = 0, KFB_FP32 = 1, KFB_BF16_MIXED = 2 };

enum kfb_status_code {
  KFB_OK = 0,
  KFB_EINVAL = 1,     /* null pointer, bad size, ld < d, n > n_max, r + n_max > d */
  KFB_EWORKSPACE = 2, /* workspace smaller than required */
  KFB_EHIP = 3,       /* a HIP runtime call failed */
  KFB_ESTATE = 4,     /* states incompatible with the call (widths, precision, same handle) */
  KFB_EEMPTY = 5      /* the state holds no modes yet */
};

/* kfb_precondition flags */
enum kfb_flags {
  KFB_SPECTRUM_CONTINUATION = 1, /* Section 3.5: lam += m, D -= m per factor, m the smallest
                                    positive eigenvalue of the modes used (a mode of eigenvalue 0
                                    is an empty slot: a dropped null direction or padding) */
  KFB_TRUNCATE_AFTER = 2,        /* apply with the leading r modes only (default: all r+n) */
  KFB_RELATIVE_DAMPING = 4       /* Section 6: lam = phi * lambda_max per factor, the lam argument
                                    being phi and lambda_max the largest eigenvalue of the modes
                                    used (lam = phi when that is not positive); applied before
                                    spectrum continuation */
};

/* bits of the device status word */
enum kfb_event {
  KFB_EV_NONFINITE = 1u,       /* a non-finite value reached the Gram of the residual */
  KFB_EV_CHOL_DEFICIENT = 2u,  /* a CholQR pivot was below tolerance: null directions dropped */
  KFB_EV_JACOBI_MAXSWEEPS = 4u, /* the core eigensolver hit its sweep limit */
  KFB_EV_ORTHO_DRIFT = 8u        /* after an update, a column of U with a positive eigenvalue has a
                                    squared norm off 1 by more than 1e-10 (FP64), 1e-4 (FP32) or
                                    1e-3 (mixed): U has drifted from orthonormality */
};

/* Bytes of the state buffer for a factor of width d, truncation rank r and
 * batch capacity n_max: two U buffers (d x (r+n_max), front/back) and two
 * eigenvalue vectors, plus a status word.  Returns 0 on invalid sizes:
 * d < 1, r < 0, n_max < 1, r + n_max > d (Brand needs r + n <= d, Section 2.3),
 * n_max > 2048 (the widest residual the CholeskyQR kernels factor) or
 * r + n_max > 4096 (the largest core the eigensolver finalises). */
size_t kfb_state_bytes(int64_t d, int32_t r, int32_t n_max, int32_t prec);

/* Create a handle over a caller-owned state buffer of kfb_state_bytes bytes.
 * rho is the EA decay (Section 2.1).  The state starts empty (no modes); the
 * first update uses batch weight 1/n, later ones (1 - rho)/n.
 * Requires the sizes kfb_state_bytes accepts and 0 <= rho < 1 (KFB_EINVAL). */
int kfb_state_create(kfb_state_t* out, int64_t d, int32_t r, int32_t n_max, double rho,
                     int32_t prec, void* state_buf, size_t state_bytes, kfb_stream_t stream);

/* Free the host-side handle (the caller frees the buffers it owns). */
int kfb_destroy(kfb_state_t st);

/* Workspace bytes for one kfb_brand_update on this state with batch width n. */
size_t kfb_update_workspace_bytes(kfb_state_t st, int32_t n);

/* One B-KFAC step (Algorithm 4) on one factor:
 *   truncate (U, D) to min(k_valid, r) modes, then
 *   U diag(D) U^T <- rho U diag(D) U^T + w M M^T   exactly (Algorithm 3),
 * with w = 1/n for the first update and (1 - rho)/n afterwards.
 * M: d x n column-major (ldm >= d); FP64 / FP32 / BF16 per the precision form.
 * After the call the state holds k_valid = min(k_valid, r) + n modes.
 * Errors (returned before anything is enqueued): KFB_EINVAL for a null
 * pointer, n < 1, n > n_max or ldm < d; KFB_EWORKSPACE. */
int kfb_brand_update(kfb_state_t st, const void* M, int64_t ldm, int32_t n, void* workspace,
                     size_t ws_bytes, kfb_stream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * update as kfb_brand_update with no workspace argument.  Its workspace is a
 * library-owned device array of kfb_scratch_bytes() bytes (64 MiB), one per
 * GPU, held until the process ends; the call allocates nothing.  Every call
 * on one GPU shares that array: calls that overlap in time on one GPU (on
 * different streams, or from different host threads) race and must be
 * serialised by the caller.  The device is the current HIP device, which must
 * be the one holding the state.  Errors as kfb_brand_update, plus
 * KFB_EWORKSPACE when the update needs more than kfb_scratch_bytes() (then
 * nothing is enqueued) and KFB_EHIP when the array's address cannot be
 * resolved. */
size_t kfb_scratch_bytes(void);
int kfb_brand_update_scratch(kfb_state_t st, const void* M, int64_t ldm, int32_t n, kfb_stream_t stream);

/* Grouped form: `count` independent updates in one set of launches.  All
 * states must share d, r, precision and current k_valid, and all batches the
 * same n and ldm (one shape bucket); results equal `count` separate calls. */
size_t kfb_update_batched_workspace_bytes(int32_t count, kfb_state_t const* states, int32_t n);
int kfb_brand_update_batched(int32_t count, kfb_state_t const* states, const void* const* Ms,
                             int64_t ldm, int32_t n, void* workspace, size_t ws_bytes,
                             kfb_stream_t stream);

/* Grouped update of batches of uneven widths (one launch sequence for a
 * group whose batches differ in n): batch i has widths[i] (1..n) real columns
 * followed by zero columns up to n (the caller pads).  Each problem takes the
 * weight of its own width, (1 - rho)/widths[i] (1/widths[i] on a first
 * update), so the result is the exact update by the real columns; the
 * padding's zero pivots in CholeskyQR are expected and not reported as rank
 * deficiency.  The state then holds min(k_valid, r) + n modes, the padded
 * ones empty (eigenvalue 0, zero column in U, sorted after every real mode):
 * they add nothing to the inverse and spectrum continuation takes its minimum
 * over the positive eigenvalues only, so a padded update leaves the same
 * inverse as the unpadded one; the next truncation drops them.
 * widths: HOST array of count values.  Workspace as
 * kfb_update_batched_workspace_bytes(count, states, n).  KFB_EINVAL for a
 * width outside 1..n. */
int kfb_brand_update_batched_widths(int32_t count, kfb_state_t const* states, const void* const* Ms,
                                    int64_t ldm, int32_t n, const int32_t* widths, void* workspace,
                                    size_t ws_bytes, kfb_stream_t stream);

/* Grouped update across factor shapes (one launch sequence for the updates
 * of many factors, Algorithm 4 per factor: the factors are independent).  The
 * states share the precision form and the number of kept modes
 * r_eff = min(k_valid, r) but may differ in width d_i, rank r, capacity n_max
 * and batch width: batch i is d_i x widths[i], column-major with leading
 * dimension ldms[i] >= d_i (HOST arrays of count values).  Every problem runs
 * at the group's shape, d = max d_i (rounded up to 64) and n = max widths[i]
 * (which must not exceed any state's n_max): the state's U and its batch are
 * copied into zero-padded workspace buffers, the update runs on them (the
 * zero rows stay zero through every stage) and the first d_i rows of the new
 * basis go to the state's back buffer.  Each problem takes the weight of its
 * own width, as kfb_brand_update_batched_widths; afterwards every state holds
 * r_eff + n modes, those beyond its own r_eff + widths[i] being empty slots
 * (eigenvalue 0, zero column).  Results equal separate calls within rounding
 * (the padded shape changes the blocking of the products).
 * Errors: KFB_ESTATE (forms or r_eff differ, a state twice), KFB_EINVAL (a
 * width outside 1..n_max of its state, n above some state's n_max, ldms[i] <
 * d_i, null pointers), KFB_EWORKSPACE. */
size_t kfb_update_grouped_workspace_bytes(int32_t count, kfb_state_t const* states, const int32_t* widths);
int kfb_brand_update_grouped(int32_t count, kfb_state_t const* states, const void* const* Ms,
                             const int64_t* ldms, const int32_t* widths, void* workspace, size_t ws_bytes,
                             kfb_stream_t stream);

/* Workspace bytes for kfb_precondition on this pair of states. */
size_t kfb_precondition_workspace_bytes(kfb_state_t st_gamma, kfb_state_t st_a);

/* Two-sided regularised inverse (Section 2.1, Algorithm 1 inverse lines):
 *   S = (U_G D_G U_G^T + lam_gamma I)^{-1} G (U_A D_A U_A^T + lam_a I)^{-1}
 * with G, S row-major d_out x d_in, d_out = st_gamma's d and d_in = st_a's d.
 * lam > 0 absolute (or relative with KFB_RELATIVE_DAMPING).  Uses all k_valid
 * modes (or r with KFB_TRUNCATE_AFTER).
 * G and S may not alias.  FP64 form: double G/S; FP32 and mixed: float. */
int kfb_precondition(kfb_state_t st_gamma, kfb_state_t st_a, const void* G, int64_t ldg, void* S,
                     int64_t lds, double lam_gamma, double lam_a, uint32_t flags, void* workspace,
                     size_t ws_bytes, kfb_stream_t stream);

/* Grouped form: `count` layers sharing (d_out, d_in, k_valid of each side,
 * precision, flags); lambdas per layer. */
size_t kfb_precondition_batched_workspace_bytes(int32_t count, kfb_state_t const* st_gamma,
                                                kfb_state_t const* st_a);
int kfb_precondition_batched(int32_t count, kfb_state_t const* st_gamma, kfb_state_t const* st_a,
                             const void* const* G, int64_t ldg, void* const* S, int64_t lds,
                             const double* lam_gamma, const double* lam_a, uint32_t flags,
                             void* workspace, size_t ws_bytes, kfb_stream_t stream);

/* Workspace bytes for kfb_precondition_factored on this pair of states and
 * factor width n (0 if n < 1). */
size_t kfb_precondition_factored_workspace_bytes(kfb_state_t st_gamma, kfb_state_t st_a, int32_t n);

/* Linear-cost application to a factored layer gradient (Section 5,
 * Algorithm 8).  When the gradient is the product G_k A_k^T of the layer's
 * per-sample output-gradient and activation matrices (the same matrices the
 * factors are built from), each side's regularised inverse is applied to its
 * own thin factor and the step is formed from the two results:
 *   Y_G = (U_G D_G U_G^T + lam_gamma I)^{-1} G_k = U_G c_G U_G^T G_k + G_k / lam_gamma,
 *   Y_A = (U_A D_A U_A^T + lam_a I)^{-1} A_k     = U_A c_A U_A^T A_k + A_k / lam_a,
 *   S   = Y_G Y_A^T,        c = diag(1/(D + lam) - 1/lam),
 * which equals kfb_precondition with G = G_k A_k^T, at O(N d n) cost per side
 * instead of O(N d_out d_in), plus the d_out x d_in x n product for S.
 * G_k: d_out x n and A_k: d_in x n, column-major (element (i, j) at
 * X[i + j*ld], ld >= the side's d: a PyTorch [n, d] row-major tensor), in the
 * element type of the state's batches (FP64: double, FP32: float, mixed:
 * bf16); n >= 1.  S: row-major d_out x d_in, lds >= d_in (double in the FP64
 * form, float otherwise); it may not alias G_k or A_k.  lam > 0 absolute,
 * flags as for kfb_precondition.  In the mixed form the per-side products run
 * on BF16 MFMA with U and the coefficients split into two BF16 terms, the
 * product for S on single-term BF16 MFMA, all with FP32 accumulation.
 * Errors: KFB_EINVAL (null pointer, n < 1, ld too small, lam <= 0),
 * KFB_ESTATE (precision or handle mismatch), KFB_EEMPTY (a state without
 * modes), KFB_EWORKSPACE. */
int kfb_precondition_factored(kfb_state_t st_gamma, kfb_state_t st_a, const void* G_k, int64_t ldgk,
                              const void* A_k, int64_t ldak, int32_t n, void* S, int64_t lds,
                              double lam_gamma, double lam_a, uint32_t flags, void* workspace,
                              size_t ws_bytes, kfb_stream_t stream);

/* Grouped form: `count` layers sharing (d_out, d_in, modes per side, n,
 * precision, flags); lambdas per layer.  Results equal the single calls bit
 * for bit. */
size_t kfb_precondition_factored_batched_workspace_bytes(int32_t count, kfb_state_t const* st_gamma,
                                                         kfb_state_t const* st_a, int32_t n);
int kfb_precondition_factored_batched(int32_t count, kfb_state_t const* st_gamma,
                                      kfb_state_t const* st_a, const void* const* G_k, int64_t ldgk,
                                      const void* const* A_k, int64_t ldak, int32_t n, void* const* S,
                                      int64_t lds, const double* lam_gamma, const double* lam_a,
                                      uint32_t flags, void* workspace, size_t ws_bytes,
                                      kfb_stream_t stream);

/* ---- B-R-KFAC (Section 3.3, Algorithm 5) ------------------------------------
 * Every T_RSVD steps B-R-KFAC replaces a factor's representation by a
 * randomized SVD of the dense EA factor of the previous step, in place of the
 * usual truncation, and then performs the B-update as usual.  The dense factor
 * X (d x d, column-major, ld ldx >= d; double in the FP64 form, float
 * otherwise) is caller memory, kept beside the state.
 *
 * kfb_dense_bytes: bytes of such a factor (0 on invalid sizes).
 * kfb_dense_update: one step of the EA definition (Section 2.1) for the
 * state's rho and batch convention:  X <- rho X + (1 - rho)/n M M^T, or, with
 * first != 0, X <- M M^T / n (X is not read).  M as for kfb_brand_update.
 * The workspace (kfb_dense_update_workspace_bytes, 256-byte aligned) holds the
 * call's record.  Mixed form: BF16 M on MFMA with FP32 accumulation.  X may not
 * overlap M.  Errors: KFB_EINVAL, KFB_EWORKSPACE. */
size_t kfb_dense_bytes(int64_t d, int64_t ldx, int32_t prec);
size_t kfb_dense_update_workspace_bytes(void);
int kfb_dense_update(kfb_state_t st, void* X, int64_t ldx, const void* M, int64_t ldm, int32_t n,
                     int32_t first, void* workspace, size_t ws_bytes, kfb_stream_t stream);

/* kfb_rsvd_overwrite: (U, D) <- the rank-r randomized SVD of X (r = the
 * state's truncation rank), with l = r + oversample sketch columns and
 * power_its re-orthonormalised power iterations (each a product with X^T and
 * one with X):
 *   Q = orth(X Omega); power_its times { Q = orth(X^T Q); Q = orth(X Q) };
 *   B = Q^T X = U_B S V_B^T;  U = Q U_B[:, :r],  D = S[:r]
 * (the paper writes the result as U~ D~ U~^T: the left singular vectors and
 * the singular values).  Omega: the d x l Gaussian test matrix (column-major,
 * ld ldo >= d, the element type of X) drawn by the caller.  Orthonormalisation
 * is CholeskyQR as in the B-update; the small SVD is the B-update's core
 * eigensolver on the triangular factor of X^T Q.  Writes the back buffers and
 * swaps (a preconditioning enqueued earlier still reads the old modes); the
 * state then holds r modes.  Requires 1 <= r, l <= min(d, r + n_max, 2048),
 * 0 <= power_its <= 16.  A sketch whose range has fewer than l directions
 * (X of low rank) sets KFB_EV_CHOL_DEFICIENT and yields zero singular values
 * for the missing directions.  Errors: KFB_EINVAL, KFB_EWORKSPACE. */
size_t kfb_rsvd_workspace_bytes(kfb_state_t st, int32_t oversample);
int kfb_rsvd_overwrite(kfb_state_t st, const void* X, int64_t ldx, const void* Omega, int64_t ldo,
                       int32_t oversample, int32_t power_its, void* workspace, size_t ws_bytes,
                       kfb_stream_t stream);

/* ---- B-KFAC-C (Section 3.4, Algorithms 6 and 7) -----------------------------
 * Light correction of the current representation against the dense EA factor
 * X of the same step (kept with kfb_dense_update):
 *   U_c = U[:, col_idx];  M_S = U_c^T X U_c = W L W^T;
 *   U[:, col_idx] = U_c W;  D[col_idx] = L;
 * then the modes are re-sorted by eigenvalue, descending, so the next
 * truncation keeps the largest (the paper writes the columns back in place).
 * col_idx: HOST array of n_crc distinct indices among the leading
 * min(r, k_valid) modes (the method's random choice, drawn by the caller;
 * validated, then copied to the workspace on the stream).  X as for
 * kfb_rsvd_overwrite.  The small EVD is the core eigensolver on the Cholesky
 * factor of M_S.  Writes the back buffers and swaps; k_valid is unchanged.
 * Errors: KFB_EINVAL (bad indices, n_crc out of range, k_valid > 4096),
 * KFB_EEMPTY, KFB_EWORKSPACE. */
size_t kfb_correct_workspace_bytes(kfb_state_t st, int32_t n_crc);
int kfb_light_correction(kfb_state_t st, const void* X, int64_t ldx, const int32_t* col_idx, int32_t n_crc,
                         void* workspace, size_t ws_bytes, kfb_stream_t stream);

/* Host-side metadata: modes held, updates applied, sizes. Any pointer may be NULL. */
int kfb_state_info(kfb_state_t st, int32_t* k_valid, int64_t* step, int64_t* d, int32_t* r,
                   int32_t* n_max, int32_t* prec);

/* Device pointers of the current (front) eigenvectors and eigenvalues:
 * U is d x k_valid column-major with leading dimension *ldu (FP64 for the
 * FP64 form, FP32 otherwise); D is k_valid values, descending (FP64, or FP32
 * in the FP32 form).  Valid until the next update is enqueued. */
int kfb_state_front(kfb_state_t st, const void** U, int64_t* ldu, const void** D);

/* Overwrite the state with a caller-supplied representation (checkpoint
 * restore, or seeding from a randomized SVD: Proposition 4.1 considers the
 * process started by an RSVD at k = 0).  U (device, same element type as the
 * state, d x k column-major, ld ldu) must be orthonormal; D (device, same
 * element type as the state's D) finite, non-negative and descending.
 * D is read back first (the call synchronises the stream) and a violation
 * returns KFB_EINVAL with the state untouched; U is then copied and its
 * column norms checked on the device: a column (of positive eigenvalue)
 * whose squared norm is off 1 by more than the drift detector's threshold
 * sets KFB_EV_ORTHO_DRIFT in the status word (see kfb_reorthonormalize).
 * KFB_EINVAL also for k > min(d, r + n_max), ldu < d, step < 0. */
int kfb_state_load(kfb_state_t st, const void* U, int64_t ldu, const void* D, int32_t k,
                   int64_t step, kfb_stream_t stream);

/* Drift recovery (the method assumes an orthonormal U, Section 2.3; BF16 and
 * FP32 products round it): re-orthonormalise the current representation
 * without changing the matrix it stands for.  U = Q R by CholeskyQR, so
 * U D U^T = Q (R D R^T) Q^T; the core R D R^T is diagonalised by the core
 * eigensolver (square factor R diag(sqrt D)) and the state becomes
 * (Q W, Lambda), modes descending; k_valid and the step count are unchanged.
 * Meant for a state whose status word reported KFB_EV_ORTHO_DRIFT.  Modes of
 * eigenvalue 0 with a zero column (empty slots) are dropped directions of the
 * factorisation and set KFB_EV_CHOL_DEFICIENT.  Writes the back buffers and
 * swaps.  Workspace: kfb_reorth_workspace_bytes (0 if k_valid > 2048).
 * Errors: KFB_EEMPTY (no modes), KFB_EINVAL (k_valid > 2048, null or
 * misaligned workspace), KFB_EWORKSPACE. */
size_t kfb_reorth_workspace_bytes(kfb_state_t st);
int kfb_reorthonormalize(kfb_state_t st, void* workspace, size_t ws_bytes, kfb_stream_t stream);

/* Read and clear the device status word (synchronises the given stream). */
int kfb_state_status(kfb_state_t st, uint32_t* events, kfb_stream_t stream);

/* Tuning table of the core eigensolver (filled by the project's autotuner,
 * paper_2210_08494_amd/tune.py): for cores of size N = r_eff + n in precision
 * form prec, use the configuration bw:
 *   4, 8, 16, 32             column blocks of that width, the block pair's
 *                            panel held in LDS (the LDS limit must admit it);
 *   KFB_JAC_STREAMED | 32     32-column blocks, panels read from global
 *                            memory, on FP64 MFMA (FP64 core: the FP64 and
 *                            BF16-mixed forms) or FP32 MFMA (the FP32 form);
 *   KFB_JAC_STREAMED | 16     16-column blocks, panels read from global
 *                            memory (FP64 core only);
 *   KFB_JAC_STREAMED | KFB_JAC_REFINE | 32
 *                            BF16-mixed form only: the iteration on FP32
 *                            copies of the core (FP32 MFMA), then one FP64
 *                            refinement step of the eigenpairs of the FP64
 *                            core (Ogita-Aishima iterative refinement on FP64
 *                            MFMA), which leaves eigenvalues and vectors of
 *                            FP64 accuracy outside clusters of near-equal
 *                            eigenvalues;
 * streamed configurations need at least four blocks.
 * Inadmissible values give KFB_EINVAL.  bw = 0 removes the entry, restoring
 * the built-in choice: KFB_JAC_STREAMED | 32 for N >= 256 (with
 * KFB_JAC_REFINE in the BF16-mixed form; also for the new-direction block
 * solve of an update), else the widest LDS block that fits.  Affects calls made after it returns; results of a given table are
 * deterministic.  kfb_tune_get_jacobi reports the configuration and padded
 * size a core of size N would use. */
#define KFB_JAC_STREAMED 0x100
#define KFB_JAC_REFINE 0x200
int kfb_tune_set_jacobi(int32_t prec, int32_t N, int32_t bw);
int kfb_tune_get_jacobi(int32_t prec, int32_t N, int32_t* bw, int32_t* Np);

/* Tuning table of the BF16 MFMA products of the mixed form (filled by the
 * project's autotuner, paper_2210_08494_amd/tune.py): the output tile of the
 * product C (m x n) = A (m x k) B (k x n), 128 (four waves of 64 x 64) or 256
 * (eight waves of 128 x 64; twice the flops per staged byte, a quarter of the
 * workgroups); 0 removes the entry (built-in: 128).  Products carrying the
 * hi/lo split (the update's) always use 128.  Results do not depend on the
 * tile (the k order of every sum is the same).  kfb_tune_get_gemm reports the
 * tile a product of that shape would use.  KFB_EINVAL for non-positive sizes
 * or another tile. */
int kfb_tune_set_gemm(int32_t m, int32_t n, int32_t k, int32_t tile);
int kfb_tune_get_gemm(int32_t m, int32_t n, int32_t k, int32_t* tile);

/* Optional stage timing (diagnostics).  While enabled, each stage of the
 * update and precondition calls (projection, residual, CholeskyQR, core
 * assembly, Jacobi rounds, finalize, rotation; the apply's products) is
 * bracketed by HIP events recorded on the call's stream, and the number of
 * kernel launches of the stage is counted.  kfb_profile_report synchronises
 * on the recorded events, then writes a JSON object
 *   {"stage": {"calls": C, "launches": L, "ms": T}, ...}
 * into buf (NUL-terminated, truncated to len) and optionally clears the
 * totals.  Not for use while a stream is being captured into a graph.
 * Returns KFB_OK, or KFB_EHIP if an event query fails. */
int kfb_profile_enable(int on);
int kfb_profile_report(char* buf, size_t len, int reset);

const char* kfb_strerror(int code);

/* Library build identification: "kfb gfx950 hip src=<digest>", the digest a
 * SHA-1 prefix over the library's sources, so a measurement can be tied to the
 * exact code it was taken on. */
const char* kfb_build_info(void);

#ifdef __cplusplus
}
#endif
#endif /* KFB_H */
