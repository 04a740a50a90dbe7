// Small dense linear algebra of the Brand update (Algorithm 3):
//   * Cholesky factor + triangular inverse of the residual Gram (CholeskyQR),
//   * assembly of the square factor of the core (eqn. for M_S, Section 2.3),
//   * block one-sided Jacobi eigensolver of the core,
//   * sort / gather of the eigenpairs,
// and the coefficient / scaling kernels of the two-sided inverse application.
#include "kfb_kernels.h"

namespace kfb {

template <typename T> __device__ __forceinline__ T dev_sqrt(T x);
template <> __device__ __forceinline__ double dev_sqrt<double>(double x) { return sqrt(x); }
template <> __device__ __forceinline__ float dev_sqrt<float>(float x) { return sqrtf(x); }

// 1/sqrt(x) from the hardware estimate refined by Newton steps
// (y <- y (3 - x y^2) / 2): two steps reach FP64 round-off from the FP64
// estimate, one step FP32 round-off.
template <typename T> __device__ __forceinline__ T dev_rsqrt(T x);
template <> __device__ __forceinline__ double dev_rsqrt<double>(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  return y * (1.5 - 0.5 * x * y * y);
}
template <> __device__ __forceinline__ float dev_rsqrt<float>(float x) {
  float y = __builtin_amdgcn_rsqf(x);
  return y * (1.5f - 0.5f * x * y * y);
}

// Orders the LDS accesses of one wave (performed in program order) without a
// workgroup barrier: keeps the compiler from moving them across this point.
// value of x held by lane `lane` of the wave (lane a compile-time constant in
// the unrolled loops that use it)
__device__ __forceinline__ double lane_value(double x, int lane) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), lane);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_value(float x, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
}

// four doubles: an FP64 MFMA 16x16x4 accumulator fragment
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double jac_d4;

template <typename T> struct Eps;
template <> struct Eps<double> { static constexpr double v = 2.220446049250313e-16; };
template <> struct Eps<float> { static constexpr float v = 1.1920929e-07f; };

template <typename To, typename From>
__device__ __forceinline__ To cvt(From x) { return static_cast<To>(x); }

// ---------------------------------------------------------------------------
// Cholesky of an n x n symmetric PSD Gram matrix W = R^T R (R upper) and the
// inverse X = R^{-1}, one workgroup per problem.  A pivot at or below
// tau_rel * max_i W_ii marks a numerically null direction of the residual:
// its row of R is set to zero and the matching row and column of X are zero,
// so the orthonormalised residual Q = Z X gets a zero column there (any
// orthonormal completion would do; zero columns carry zero eigenvalues and
// never influence the update or the inverse application).
// ---------------------------------------------------------------------------
constexpr int CHOL_NT = 1024;
constexpr int CHOL_MAXN = MAX_QR_COLS;

template <typename T>
__global__ __launch_bounds__(CHOL_NT) void chol_inv_kernel(const Rec* __restrict__ recs, CholArgs a) {
  const Rec& rec = recs[blockIdx.x];
  const int n = a.n;
  // columns at or beyond nreal are zero padding of the batch (a grouped update of
  // uneven widths): their zero pivots are expected, not a rank deficiency
  const int nreal = rec.s[2] > 0.0 ? (int)rec.s[2] : n;
  const T* Wg = at<const T>(rec, WS, a.off_gram);
  T* R = at<T>(rec, WS, a.off_R);
  T* X = at<T>(rec, WS, a.off_Rinv);
  __shared__ T row[CHOL_MAXN];
  __shared__ T red[CHOL_NT / 64];
  __shared__ T redt[CHOL_NT / 64];
  __shared__ int deficient, nonfinite;
  const int t = threadIdx.x;
  if (t == 0) { deficient = 0; nonfinite = 0; }
  __syncthreads();

  // max diagonal (tolerance scale) and finiteness (v - v is 0 only for finite v)
  T mx = T(0), tr = T(0);
  for (int i = t; i < n; i += CHOL_NT) {
    const T v = Wg[i + (int64_t)i * n];
    if (!(v - v == T(0))) nonfinite = 1;
    mx = v > mx ? v : mx;
    tr += v;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const T o = __shfl_xor(mx, off);
    mx = o > mx ? o : mx;
    tr += __shfl_xor(tr, off);
  }
  if ((t & 63) == 0) { red[t >> 6] = mx; redt[t >> 6] = tr; }
  // copy upper triangle, zero the rest
  for (int64_t e = t; e < (int64_t)n * n; e += CHOL_NT) {
    const int i = (int)(e % n), j = (int)(e / n);
    R[e] = (i <= j) ? Wg[e] : T(0);
    X[e] = T(0);
  }
  __syncthreads();
  if (t == 0) {
    T m = red[0], tt = redt[0];
    for (int w = 1; w < CHOL_NT / 64; ++w) { m = red[w] > m ? red[w] : m; tt += redt[w]; }
    red[0] = m;
    redt[0] = tt;
  }
  __syncthreads();
  const T tau = T(a.tau_rel) * red[0];
  // shifted CholeskyQR: factor W + s I (s = shift_rel * trace W); Z = Q1 R1 still holds
  // exactly with Q1 = Z R1^{-1}, which is then well conditioned for the next passes
  if (a.shift_rel > 0.0) {
    const T sh = T(a.shift_rel) * redt[0];
    for (int i = t; i < n; i += CHOL_NT) R[i + (int64_t)i * n] += sh;
    __syncthreads();
  }

  // right-looking Cholesky, row by row of R
  for (int j = 0; j < n; ++j) {
    const T p = R[j + (int64_t)j * n];
    const bool ok = p > tau && (red[0] > T(0));
    const T sp = ok ? dev_sqrt(p) : T(0);
    const T inv = ok ? T(1) / sp : T(0);
    for (int k = j + t; k < n; k += CHOL_NT) {
      const T v = (k == j) ? sp : R[j + (int64_t)k * n] * inv;
      R[j + (int64_t)k * n] = v;
      row[k] = v;
    }
    if (!ok && t == 0 && j < nreal) deficient = 1;
    __syncthreads();
    const int m = n - j - 1;
    if (ok && m > 0) {
      for (int64_t e = t; e < (int64_t)m * m; e += CHOL_NT) {
        const int ii = (int)(e % m), kk = (int)(e / m);
        if (ii <= kk) {
          const int gi = j + 1 + ii, gk = j + 1 + kk;
          R[gi + (int64_t)gk * n] -= row[gi] * row[gk];
        }
      }
    }
    __syncthreads();
  }

  // X = R^{-1}, rows bottom-up; threads of a sub-group share one column
  int tpc = 1;
  while (tpc * 2 * n <= CHOL_NT && tpc < 16) tpc *= 2;
  const int lane = t % tpc, colid = t / tpc, ncolgroups = CHOL_NT / tpc;
  for (int i = n - 1; i >= 0; --i) {
    const T rii = R[i + (int64_t)i * n];
    for (int k = i + 1 + t; k < n; k += CHOL_NT) row[k] = R[i + (int64_t)k * n];
    __syncthreads();
    const T dinv = rii > T(0) ? T(1) / rii : T(0);
    for (int j0 = i; j0 < n; j0 += ncolgroups) {
      const int j = j0 + colid;
      T sum = T(0);
      if (j < n && j > i) {
        for (int k = i + 1 + lane; k <= j; k += tpc) sum += row[k] * X[k + (int64_t)j * n];
      }
      for (int off = tpc / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
      if (j < n && lane == 0) {
        if (j == i) X[i + (int64_t)i * n] = dinv;
        else X[i + (int64_t)j * n] = -sum * dinv;
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    uint32_t ev = (deficient ? KFB_EV_CHOL_DEFICIENT : 0u) | (nonfinite ? KFB_EV_NONFINITE : 0u);
    if (ev) atomicOr(at<uint32_t>(rec, STATUS, 0), ev);
  }
}


// Blocked form of the same factorisation and inverse (n <= 272), in 32-wide
// blocks with the block row of R staged in LDS.  Per block column: one wave
// factors the diagonal block; the block row right of it is solved column by
// column (R_JJ^T Y = R_J,rest); the trailing upper triangle takes the rank-32
// update in 4 x 4 register blocks.  The inverse follows in two launches: the
// diagonal blocks X_JJ = R_JJ^{-1} (one wave each), then the block rows
// X_J,rest = -X_JJ (R_J,rest X_rest,rest) by column blocks.  The pivot rule,
// the shift and the zero rows are those of the column kernel; only the order
// of the sums differs.
// n <= 272: the inverse's column blocks (n x 32 of X and a 32 x (n - 32) block
// row of R, FP64) fit the 160 KB of LDS
constexpr int CB = 32, CHB_NT = 512, CHB_MAXN = 272;
static_assert((CHB_MAXN * CB + CB * (CHB_MAXN - CB)) * 8 <= 160 * 1024, "inverse column block exceeds LDS");

template <typename T>
__global__ __launch_bounds__(CHB_NT) void chol_blocked_kernel(const Rec* __restrict__ recs, CholArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char chb_smem[];
  const Rec& rec = recs[blockIdx.x];
  const int n = a.n;
  // columns at or beyond nreal are zero padding of the batch (a grouped update of
  // uneven widths): their zero pivots are expected, not a rank deficiency
  const int nreal = rec.s[2] > 0.0 ? (int)rec.s[2] : n;
  const int LDW = ((n + 3) / 4) * 4 + 4;  // row stride of the staged block rows
  T* Pn = reinterpret_cast<T*>(chb_smem);  // CB x LDW: block row of R
  __shared__ T Dg[CB][CB + 1];
  __shared__ T red[CHB_NT / 64], redt[CHB_NT / 64];
  __shared__ T invrow[CB];
  __shared__ T rowb[CB];  // row j of R during the diagonal block's step j
  __shared__ int okrow[CB];
  __shared__ int deficient, nonfinite;
  const T* Wg = at<const T>(rec, WS, a.off_gram);
  T* R = at<T>(rec, WS, a.off_R);
  T* X = at<T>(rec, WS, a.off_Rinv);
  const int t = threadIdx.x;
  if (t == 0) { deficient = 0; nonfinite = 0; }
  __syncthreads();
  T mx = T(0), tr = T(0);
  for (int i = t; i < n; i += CHB_NT) {
    const T v = Wg[i + (int64_t)i * n];
    if (!(v - v == T(0))) nonfinite = 1;
    mx = v > mx ? v : mx;
    tr += v;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const T o = __shfl_xor(mx, off);
    mx = o > mx ? o : mx;
    tr += __shfl_xor(tr, off);
  }
  if ((t & 63) == 0) { red[t >> 6] = mx; redt[t >> 6] = tr; }
  if (!a.prepped) {  // R = upper triangle of W, X = 0; eight consecutive elements per thread, loads first
    const int nn = n * n;
    for (int e0 = 8 * t; e0 < nn; e0 += 8 * CHB_NT) {
      T v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = e0 + q < nn ? Wg[e0 + q] : T(0);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int e = e0 + q;
        if (e < nn) {
          R[e] = (e % n) <= (e / n) ? v[q] : T(0);
          X[e] = T(0);
        }
      }
    }
  }
  __syncthreads();
  if (t == 0) {
    T m = red[0], tt = redt[0];
    for (int w = 1; w < CHB_NT / 64; ++w) { m = red[w] > m ? red[w] : m; tt += redt[w]; }
    red[0] = m;
    redt[0] = tt;
  }
  __syncthreads();
  const T dmax = red[0];
  const T tau = T(a.tau_rel) * dmax;
  if (a.shift_rel > 0.0) {
    const T sh = T(a.shift_rel) * redt[0];
    for (int i = t; i < n; i += CHB_NT) R[i + (int64_t)i * n] += sh;
    __syncthreads();
  }

  // ---- factorisation, block column by block column
  for (int kb = 0; kb < n; kb += CB) {
    const int nbk = min(CB, n - kb), c0 = kb + nbk, m = n - c0;
    for (int e = t; e < CB * CB; e += CHB_NT) {
      const int i = e % CB, j = e / CB;
      Dg[i][j] = (i <= j && j < nbk) ? R[(kb + i) + (int64_t)(kb + j) * n] : T(0);
    }
    const int mq = ((m + 3) / 4) * 4;  // columns read by the 4-wide blocks (zero beyond m)
#pragma unroll 4
    for (int e = t; e < CB * mq; e += CHB_NT) {
      const int i = e % CB, c = e / CB;
      Pn[i * LDW + c] = (i < nbk && c < m) ? R[(kb + i) + (int64_t)(c0 + c) * n] : T(0);
    }
    __syncthreads();
    if (t < CB) {
      // diagonal block, right-looking: lane c holds column c of the block in
      // registers (rows 0..c); step j takes the pivot from lane j, each lane
      // forms its entry of row j of R, the row goes through LDS, and each lane
      // updates its column with it (the rank-1 update of the rows below j)
      const int c = t;
      T a[CB];
#pragma unroll
      for (int i = 0; i < CB; ++i) a[i] = Dg[i][c];
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        if (j < nbk) {
          const T p = lane_value(a[j], j);
          const bool ok = p > tau && dmax > T(0);
          const T inv = ok ? dev_rsqrt(p) : T(0);
          const T sp = ok ? p * inv : T(0);
          const T rj = c > j ? a[j] * inv : (c == j ? sp : T(0));  // R[j][c]
          if (c >= j) a[j] = rj;
          if (t == 0) {
            okrow[j] = ok;
            invrow[j] = inv;
            if (!ok && kb + j < nreal) deficient = 1;
          }
          rowb[c] = rj;
          wave_sync();
#pragma unroll
          for (int i = j + 1; i < CB; ++i) {
            const T ri = rowb[i];  // R[j][i]
            if (i <= c) a[i] = fma(-ri, rj, a[i]);
          }
          wave_sync();  // every lane has read the row before the next step writes it
        }
      }
#pragma unroll
      for (int i = 0; i < CB; ++i) Dg[i][c] = i <= c ? a[i] : T(0);
    }
    __syncthreads();
    for (int e = t; e < nbk * nbk; e += CHB_NT) {
      const int i = e % nbk, j = e / nbk;
      if (i <= j) R[(kb + i) + (int64_t)(kb + j) * n] = Dg[i][j];
    }
    // block row: for each column, forward substitution with Dg^T
    for (int c = t; c < m; c += CHB_NT) {
      T y[CB];
#pragma unroll
      for (int i = 0; i < CB; ++i) y[i] = Pn[i * LDW + c];
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        if (j < nbk) {
          T s0 = y[j], s1 = T(0);  // two partial sums shorten the dependent chain
#pragma unroll
          for (int i = 0; i < j; ++i) {
            if (i & 1) s1 = fma(Dg[i][j], y[i], s1);
            else s0 = fma(-Dg[i][j], y[i], s0);
          }
          y[j] = okrow[j] ? (s0 - s1) * invrow[j] : T(0);
        }
      }
#pragma unroll
      for (int i = 0; i < CB; ++i)
        if (i < nbk) {
          Pn[i * LDW + c] = y[i];
          R[(kb + i) + (int64_t)(c0 + c) * n] = y[i];
        }
    }
    __syncthreads();
    // trailing upper triangle, 4 x 4 blocks (bi <= bk) in column-major triangular order
    const int nq = mq / 4;
    const int nblk = nq * (nq + 1) / 2;
    for (int b = t; b < nblk; b += CHB_NT) {
      int bk = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
      while ((bk + 1) * (bk + 2) / 2 <= b) ++bk;
      while (bk * (bk + 1) / 2 > b) --bk;
      const int bi = b - bk * (bk + 1) / 2;
      T acc[4][4];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = T(0);
      for (int j = 0; j < nbk; ++j) {
        const T* pr = Pn + j * LDW;
        T x[4], z[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          x[q] = pr[4 * bi + q];
          z[q] = pr[4 * bk + q];
        }
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[p][q] = fma(x[p], z[q], acc[p][q]);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = 4 * bk + q;
        if (k >= m) continue;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const int i = 4 * bi + p;
          if (i <= k) R[(c0 + i) + (int64_t)(c0 + k) * n] -= acc[p][q];
        }
      }
    }
    __syncthreads();
  }

  if (t == 0) {
    uint32_t ev = (deficient ? KFB_EV_CHOL_DEFICIENT : 0u) | (nonfinite ? KFB_EV_NONFINITE : 0u);
    if (ev) atomicOr(at<uint32_t>(rec, STATUS, 0), ev);
  }
}

// X_JJ = R_JJ^{-1} for every 32 x 32 diagonal block J (one wave each): lane j
// back-substitutes column j bottom-up in registers (R_JJ staged in LDS); a
// zero pivot (dropped direction) gives a zero row.
template <typename T>
__global__ __launch_bounds__(64) void chol_diag_inv_kernel(const Rec* __restrict__ recs, CholArgs a) {
  const Rec& rec = recs[blockIdx.y];
  const int n = a.n, b0 = blockIdx.x * CB;
  if (b0 >= n) return;
  const int nb = min(CB, n - b0);
  const T* R = at<const T>(rec, WS, a.off_R);
  T* X = at<T>(rec, WS, a.off_Rinv);
  __shared__ T Rd[CB][CB + 1];
  __shared__ T dinv[CB];
  const int j = threadIdx.x;
  for (int e = j; e < CB * CB; e += 64) {
    const int i = e % CB, c = e / CB;
    Rd[i][c] = (i <= c && c < nb) ? R[(b0 + i) + (int64_t)(b0 + c) * n] : T(0);
  }
  __syncthreads();
  if (j < CB) dinv[j] = Rd[j][j] > T(0) ? T(1) / Rd[j][j] : T(0);
  __syncthreads();
  if (j >= CB) return;
  T x[CB];
#pragma unroll
  for (int i = CB - 1; i >= 0; --i) {
    x[i] = T(0);
    if (i < nb) {
      T s0 = T(0), s1 = T(0);  // two partial sums shorten the dependent chain
#pragma unroll
      for (int k = i + 1; k < CB; ++k)
        if (k <= j && k < nb) {
          if (k & 1) s1 = fma(Rd[i][k], x[k], s1);
          else s0 = fma(Rd[i][k], x[k], s0);
        }
      x[i] = (j == i) ? dinv[i] : (j > i ? -(s0 + s1) * dinv[i] : T(0));
    }
  }
  if (j < nb)
#pragma unroll
    for (int i = 0; i < CB; ++i)
      if (i <= j) X[(b0 + i) + (int64_t)(b0 + j) * n] = x[i];
}

// The rest of R^{-1} (X), one workgroup per 32-column block cb: back
// substitution over the block rows above it,
//   X_ib,cb = -X_ib,ib (R_ib,(ib,cb] X_(ib,cb],cb),  ib = cb-1, ..., 0,
// with the diagonal-block inverses X_ib,ib from the factorisation.  The
// column block of X being built stays in LDS; each step stages the block row
// of R it needs.  Column blocks are independent, so all of them run at once.
constexpr int CHI_NT = 256;
template <typename T>
__global__ __launch_bounds__(CHI_NT) void chol_inv_cols_kernel(const Rec* __restrict__ recs, CholArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char chi_smem[];
  const Rec& rec = recs[blockIdx.y];
  const int n = a.n, cb = blockIdx.x, c0 = cb * CB;
  if (cb == 0 || c0 >= n) return;  // the first block is its diagonal inverse only
  const int nc = min(CB, n - c0), top = c0 + nc;  // rows 0 .. top-1 of the column block
  const T* R = at<const T>(rec, WS, a.off_R);
  T* X = at<T>(rec, WS, a.off_Rinv);
  T* Xc = reinterpret_cast<T*>(chi_smem);  // top x CB (row-major: Xc[i * CB + c])
  T* Rp = Xc + (size_t)top * CB;           // CB x (top - CB) block row of R (row-major)
  __shared__ T Dv[CB][CB + 1];
  __shared__ T Tt[CB][CB + 1];
  const int t = threadIdx.x;
  // the diagonal block of this column block
  for (int e = t; e < nc * CB; e += CHI_NT) {
    const int i = e / CB, c = e % CB;
    Xc[(size_t)(c0 + i) * CB + c] = c < nc ? X[(c0 + i) + (int64_t)(c0 + c) * n] : T(0);
  }
  __syncthreads();
  for (int ib = cb - 1; ib >= 0; --ib) {
    const int i0 = ib * CB, k0 = i0 + CB, K = top - k0;  // columns k0 .. top-1 of the block row
    for (int e = t; e < CB * K; e += CHI_NT) {  // R(i0 + i, k0 + k): 32 consecutive rows per column
      const int i = e % CB, k = e / CB;
      Rp[(size_t)i * K + k] = R[(i0 + i) + (int64_t)(k0 + k) * n];
    }
    for (int e = t; e < CB * CB; e += CHI_NT) {
      const int i = e % CB, j = e / CB;
      Dv[i][j] = X[(i0 + i) + (int64_t)(i0 + j) * n];
    }
    __syncthreads();
    // T = R_ib,(ib,cb] X_(ib,cb],cb: thread (i, four columns)
    {
      const int i = t / 8, cq = 4 * (t % 8);
      T acc[4] = {T(0), T(0), T(0), T(0)};
      const T* rr = Rp + (size_t)i * K;
      for (int k = 0; k < K; ++k) {
        const T rv = rr[k];
        const T* xr = Xc + (size_t)(k0 + k) * CB + cq;
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = fma(rv, xr[q], acc[q]);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) Tt[i][cq + q] = acc[q];
    }
    __syncthreads();
    {  // X_ib,cb = -Dv T (Dv upper triangular)
      const int i = t / 8, cq = 4 * (t % 8);
      T acc[4] = {T(0), T(0), T(0), T(0)};
      for (int s2 = i; s2 < CB; ++s2) {
        const T dv = Dv[i][s2];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = fma(dv, Tt[s2][cq + q], acc[q]);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) Xc[(size_t)(i0 + i) * CB + cq + q] = -acc[q];
    }
    __syncthreads();
  }
  for (int e = t; e < c0 * CB; e += CHI_NT) {  // rows above the diagonal block
    const int i = e % c0, c = e / c0;
    if (c < nc) X[i + (int64_t)(c0 + c) * n] = Xc[(size_t)i * CB + c];
  }
}

template <typename T>
hipError_t chol_inv(const Rec* recs, int nrec, const CholArgs& a, hipStream_t s) {
  if (a.n <= 0 || nrec <= 0) return hipSuccess;
  if (a.n > CHOL_MAXN) return hipErrorInvalidValue;
  if (a.n <= CHB_MAXN) {
    const int ldw = ((a.n + 3) / 4) * 4 + 4;
    const size_t lds = (size_t)CB * ldw * sizeof(T);
    static bool attr = false;
    if (!attr) {
      (void)hipFuncSetAttribute((const void*)chol_blocked_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(CB * (CHB_MAXN + 4) * sizeof(T)));
      attr = true;
    }
    hipLaunchKernelGGL((chol_blocked_kernel<T>), dim3(nrec), dim3(CHB_NT), lds, s, recs, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((chol_diag_inv_kernel<T>), dim3((a.n + CB - 1) / CB, nrec), dim3(64), 0, s, recs, a);
    e = hipGetLastError();
    if (e != hipSuccess || a.n <= CB) return e;
    const int nbc = (a.n + CB - 1) / CB;
    const size_t ilds = ((size_t)a.n * CB + (size_t)CB * (a.n - CB)) * sizeof(T);
    static bool iattr = false;
    if (!iattr) {
      (void)hipFuncSetAttribute((const void*)chol_inv_cols_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(((size_t)CHB_MAXN * CB + (size_t)CB * (CHB_MAXN - CB)) * sizeof(T)));
      iattr = true;
    }
    hipLaunchKernelGGL((chol_inv_cols_kernel<T>), dim3(nbc, nrec), dim3(CHI_NT), ilds, s, recs, a);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((chol_inv_kernel<T>), dim3(nrec), dim3(CHOL_NT), 0, s, recs, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gram matrix of the residual in FP64 for CholeskyQR (Algorithm 3's thin QR):
// W = Z^T Z for Z d x n (column-major, ld = d, FP32 or FP64 entries; FP32
// products are exact in FP64).  Only the blocks on and above the diagonal are
// formed (the Cholesky reads the upper triangle): a workgroup takes a 64 x 64
// block over a chunk of rows of Z, four waves 32 x 32 each on
// v_mfma_f64_16x16x4f64, each lane feeding four consecutive rows of its column
// to four MFMA steps; the result is issued transposed so partial stores
// coalesce.  Chunks are summed in a fixed order by gram_reduce_kernel.
// ---------------------------------------------------------------------------
template <typename TZ>
__device__ __forceinline__ jac_d4 gram_ld4(const TZ* p) {
  if constexpr (sizeof(TZ) == 8) {
    return *reinterpret_cast<const jac_d4*>(p);
  } else {
    typedef __attribute__((__vector_size__(16))) float f4;
    const f4 x = *reinterpret_cast<const f4*>(p);
    return jac_d4{(double)x[0], (double)x[1], (double)x[2], (double)x[3]};
  }
}

template <typename TZ>
__global__ __launch_bounds__(256) void gram_f64_kernel(const Rec* __restrict__ recs, GramArgs a) {
  const Rec& rec = recs[blockIdx.z];
  const int n = a.n, nb = (n + 63) / 64;
  // upper block index -> (bi, bj), bi <= bj, column-major triangular order
  int b = blockIdx.x, bj = 0;
  while (b > bj) { b -= bj + 1; ++bj; }
  const int bi = b;
  const int64_t d = a.d;
  const int64_t k0 = (int64_t)blockIdx.y * a.kchunk;
  const int64_t k1 = min(d, k0 + a.kchunk);
  const TZ* Z = at<const TZ>(rec, WS, a.off_Z);
  double* part = at<double>(rec, WS, a.off_part) + (int64_t)blockIdx.y * n * n;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int ci0 = 64 * bi + 32 * (w & 1), cj0 = 64 * bj + 32 * (w >> 1);
  // this lane's columns (clamped into range; columns >= n are never stored)
  const TZ* pa[2];
  const TZ* pb[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int ca = min(ci0 + 16 * u + (l & 15), n - 1), cb = min(cj0 + 16 * u + (l & 15), n - 1);
    pa[u] = Z + (int64_t)ca * d + 4 * (l >> 4);
    pb[u] = Z + (int64_t)cb * d + 4 * (l >> 4);
  }
  jac_d4 acc[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) acc[u][v] = jac_d4{0.0, 0.0, 0.0, 0.0};
  (void)nb;
  for (int64_t k = k0; k < k1; k += 16) {
    jac_d4 xa[2], xb[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      xa[u] = gram_ld4<TZ>(pa[u] + k);
      xb[u] = gram_ld4<TZ>(pb[u] + k);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)  // transposed issue: D[p][q] = W[ci_q][cj_p]
          acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(xb[v][e], xa[u][e], acc[u][v], 0, 0, 0);
  }
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = ci0 + 16 * u + (l & 15), j = cj0 + 16 * v + (l >> 4) + 4 * q;
        if (i < n && j < n) part[i + (int64_t)j * n] = acc[u][v][q];
      }
}

// Sums the split partials of the upper blocks in a fixed order.  With off_R >=
// 0 the grid covers every 64 x 64 block: upper blocks also write R = upper(W)
// and X = 0, blocks below the diagonal write zeros to both.
__global__ __launch_bounds__(256) void gram_reduce_kernel(const Rec* __restrict__ recs, GramArgs a) {
  const Rec& rec = recs[blockIdx.z];
  const int n = a.n, nb = (n + 63) / 64;
  const bool prep = a.off_R >= 0;
  int bi, bj;
  if (prep) {
    bi = blockIdx.x % nb;
    bj = blockIdx.x / nb;
  } else {
    int b = blockIdx.x;
    bj = 0;
    while (b > bj) { b -= bj + 1; ++bj; }
    bi = b;
  }
  const double* part = at<const double>(rec, WS, a.off_part);
  double* W = at<double>(rec, WS, a.off_gram);
  double* R = prep ? at<double>(rec, WS, a.off_R) : nullptr;
  double* X = prep ? at<double>(rec, WS, a.off_X) : nullptr;
  const int64_t nn = (int64_t)n * n;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int i = 64 * bi + (e & 63), j = 64 * bj + (e >> 6);
    if (i >= n || j >= n) continue;
    const int64_t o = i + (int64_t)j * n;
    if (bi > bj) {  // below the diagonal blocks (prep only)
      R[o] = 0.0;
      X[o] = 0.0;
      continue;
    }
    double s = 0.0;
    for (int kz = 0; kz < a.ks; ++kz) s += part[kz * nn + o];
    W[o] = s;
    if (prep) {
      R[o] = i <= j ? s : 0.0;
      X[o] = 0.0;
    }
  }
}

template <typename TZ>
hipError_t gram_f64(const Rec* recs, int nrec, const GramArgs& a0, hipStream_t s) {
  if (a0.n <= 0 || nrec <= 0) return hipSuccess;
  GramArgs a = a0;
  const int nb = (a.n + 63) / 64, nblk = nb * (nb + 1) / 2;
  if (a.ks < 1) a.ks = 1;
  a.kchunk = (int)(((a.d + a.ks - 1) / a.ks + 15) / 16 * 16);
  a.ks = (int)((a.d + a.kchunk - 1) / a.kchunk);
  hipLaunchKernelGGL((gram_f64_kernel<TZ>), dim3(nblk, a.ks, nrec), dim3(256), 0, s, recs, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gram_reduce_kernel, dim3(a.off_R >= 0 ? nb * nb : nblk, 1, nrec), dim3(256), 0, s, recs, a);
  return hipGetLastError();
}
template hipError_t gram_f64<float>(const Rec*, int, const GramArgs&, hipStream_t);
template hipError_t gram_f64<double>(const Rec*, int, const GramArgs&, hipStream_t);

// ---------------------------------------------------------------------------
// Core assembly.  With L = [[diag(sqrt(rho D)), sqrt(w) P], [0, sqrt(w) R]]
// (N x N, P = U^T M including the re-projection, R the residual's triangular
// factor), the Brand core is M_S = L L^T.  The Jacobi iteration orthogonalises
// the columns of B = L^T (B^T B = M_S), accumulating V; the kernel writes B
// and V = I padded to Np x Np (padding columns are zero and never rotate).
// ---------------------------------------------------------------------------
template <typename TCore, typename TP, typename TG, typename TD>
__global__ __launch_bounds__(256) void assemble_core_kernel(const Rec* __restrict__ recs, CoreArgs a) {
  const Rec& rec = recs[blockIdx.y];
  const int r = a.r, N = a.N, Np = a.Np, n = a.n;
  const double rho = rec.s[0], w = rec.s[1];
  const TCore sw = TCore(sqrt(w));
  TCore* Bm = at<TCore>(rec, WS, a.off_B);
  TCore* Vm = at<TCore>(rec, WS, a.off_V);
  const TD* D = r > 0 ? at<const TD>(rec, D_FRONT, 0) : nullptr;
  const TP* P = r > 0 ? at<const TP>(rec, WS, a.off_P) : nullptr;
  const TP* P2 = (r > 0 && a.off_P2 >= 0) ? at<const TP>(rec, WS, a.off_P2) : nullptr;
  const TG* R = at<const TG>(rec, WS, a.off_R);
  const TCore* pB = a.off_preB >= 0 ? at<const TCore>(rec, WS, a.off_preB) : nullptr;
  const TCore* pV = a.off_preV >= 0 ? at<const TCore>(rec, WS, a.off_preV) : nullptr;
  const int64_t tot = (int64_t)Np * Np;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % Np), j = (int)(e / Np);
    // B(i, j) = L(j, i)
    const int p = j, q = i;
    TCore v = TCore(0);
    if (p < N && q < N) {
      if (p < r) {
        if (q < r) {
          if (p == q) {
            const double dv = rho * (double)D[p];
            v = TCore(dv > 0.0 ? sqrt(dv) : 0.0);
          }
        } else {
          TCore pv = TCore(P[p + (int64_t)(q - r) * r]);
          if (P2) pv += TCore(P2[p + (int64_t)(q - r) * r]);
          v = sw * pv;
        }
      } else if (q >= r) {
        v = pB ? pB[(i - r) + (int64_t)(j - r) * a.preNp] : sw * TCore(R[(p - r) + (int64_t)(q - r) * n]);
      }
    }
    Bm[e] = v;
    TCore vv = (i == j) ? TCore(1) : TCore(0);
    if (pV && i >= r && j >= r && i < N && j < N) vv = pV[(i - r) + (int64_t)(j - r) * a.preNp];
    Vm[e] = vv;
  }
}

template <typename TCore, typename TP, typename TG, typename TD>
hipError_t assemble_core(const Rec* recs, int nrec, const CoreArgs& a, hipStream_t s) {
  const int64_t tot = (int64_t)a.Np * a.Np;
  int blocks = (int)((tot + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL((assemble_core_kernel<TCore, TP, TG, TD>), dim3(blocks, nrec), dim3(256), 0, s,
                     recs, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Block one-sided Jacobi (Hestenes) on the columns of B, accumulating V.
//
// The Np columns are cut into nb = Np / BW blocks.  A sweep is a round-robin
// tournament over the blocks (circle method, nb - 1 rounds of nb / 2 disjoint
// block pairs); one launch performs one round for all problems, one workgroup
// per block pair.  A visit of the pair (I, J) works on the panel
// C = [B_I B_J] (Np x P, P = 2 BW) held in LDS:
//   1. G = C^T C (P x P Gram of the panel columns);
//   2. one cyclic sweep of two-sided Jacobi on G (P - 1 steps of P/2 disjoint
//      plane rotations, G <- J^T G J), accumulating Z = J_1 J_2 ...;
//   3. C <- C Z and [V_I V_J] <- [V_I V_J] Z.
// The rotations are exactly those scalar one-sided Jacobi would apply to the
// panel columns, but their parameters come from the small Gram instead of
// long dot products, and the panel update is a dense product.  A rotation of
// columns (p, q) is skipped when |G_pq| <= tol sqrt(G_pp G_qq); otherwise
// zeta = (G_qq - G_pp) / (2 G_pq), t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
// c = 1/sqrt(1 + t^2), s = c t, and (x_p, x_q) <- (c x_p - s x_q, s x_p + c x_q).
// A visit without any rotation leaves C and V untouched.
//
// Convergence: every workgroup adds its rotation count to cnt[sweep]; a launch
// of sweep s > 0 returns at once when cnt[s-1] == 0 (no rotation anywhere in
// the previous sweep).  When one panel holds every column (nb == 2) the
// workgroup repeats steps 1-3 itself until a pass rotates nothing.
// ---------------------------------------------------------------------------
constexpr int JAC_NT = 512;
constexpr int JAC_LDS_BYTES = 128 * 1024;  // panel budget; G and Z come on top
constexpr int JAC_LDS_MAX = 156 * 1024;    // whole dynamic allocation (160 KB per CU on gfx950)

__device__ __forceinline__ void tour_pair(int P, int st, int q, int* x, int* y) {
  // circle method over P players, step st in [0, P-1), pair q in [0, P/2)
  const int R = P - 1;
  if (q == 0) { *x = st; *y = P - 1; }
  else { *x = (st + q) % R; *y = (st - q + R) % R; }
}


// G = C^T C for the panel C (Np x P, column stride LDP) into G (row-major P x P).
// FP64 with P >= 16: 16x16 tiles on MFMA (upper triangle, one wave per tile
// slot); otherwise 4x4 register blocks on FMA with rows split across lanes.
template <typename T, int P>
__device__ __forceinline__ void jac_gram(const T* pb, int Np, int LDP, T* G, T* scratch, int t) {
  if constexpr (sizeof(T) == 8 && P >= 16) {
    // upper-triangle 16x16 tiles x KP slices of the rows; slice 0 writes G, the
    // others write partial tiles into scratch (P x P doubles) that are added after
    // a barrier by the caller via jac_gram_finish
    constexpr int NT16 = P / 16;
    constexpr int NTILE = NT16 * (NT16 + 1) / 2;
    constexpr int NW = JAC_NT / 64;
    constexpr int KP = (NTILE * 2 <= NW) ? 2 : 1;
    const int w = t / 64, l = t % 64;
    for (int item = w; item < NTILE * KP; item += NW) {
      const int tile = item % NTILE, kp = item / NTILE;
      int ti = 0, rem = tile;
      while (rem >= NT16 - ti) { rem -= NT16 - ti; ++ti; }
      const int tj = ti + rem;
      jac_d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
      const T* ca = pb + (size_t)(ti * 16 + (l % 16)) * LDP + (l / 16);
      const T* cb = pb + (size_t)(tj * 16 + (l % 16)) * LDP + (l / 16);
      const int kb = kp * (Np / KP), ke = kb + Np / KP;
      for (int k0 = kb; k0 < ke; k0 += 8) {
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[k0], cb[k0], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[k0 + 4], cb[k0 + 4], acc1, 0, 0, 0);
      }
      T* dst = kp == 0 ? G : scratch + (size_t)(kp - 1) * P * P;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = ti * 16 + l / 16 + 4 * v, j = tj * 16 + l % 16;
        const T x = acc0[v] + acc1[v];
        dst[i * P + j] = x;
        if (kp == 0) G[j * P + i] = x;
      }
    }
    if constexpr (KP > 1) {
      __syncthreads();
      for (int e = t; e < P * P; e += JAC_NT) {
        const int i = e / P, j = e % P;
        if (i <= j && (i / 16) <= (j / 16)) {
          const T x = G[i * P + j] + scratch[i * P + j];
          G[i * P + j] = x;
          G[j * P + i] = x;
        }
      }
    }
  } else {
    constexpr int NBLK = (P / 4) * (P / 4);
    constexpr int RS0 = JAC_NT / NBLK;
    constexpr int RS = RS0 > 64 ? 64 : RS0;  // lanes of one wave share a block
    static_assert(RS >= 1 && (RS & (RS - 1)) == 0, "bad Gram split");
    if (t >= NBLK * RS) return;  // whole idle waves (NBLK * RS is a multiple of 64)
    const int blk = t / RS, rs = t % RS;
    const int bi = blk / (P / 4), bj = blk % (P / 4);
    T acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = T(0);
    if (bi <= bj) {
      for (int row = rs; row < Np; row += RS) {
        T x[4], y[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) x[i] = pb[(size_t)(bi * 4 + i) * LDP + row];
#pragma unroll
        for (int j = 0; j < 4; ++j) y[j] = pb[(size_t)(bj * 4 + j) * LDP + row];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = fma(x[i], y[j], acc[i][j]);
      }
    }
#pragma unroll
    for (int off = RS / 2; off > 0; off >>= 1)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += __shfl_xor(acc[i][j], off);
    if (rs == 0 && bi <= bj) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          G[(bi * 4 + i) * P + (bj * 4 + j)] = acc[i][j];
          G[(bj * 4 + j) * P + (bi * 4 + i)] = acc[i][j];
        }
    }
  }
}

// X <- X Z for a panel X (Np x P) read through xin(row, k) and written
// through xout(row, j, value); Z row-major P x P in LDS with row stride ZP.  FP64 with P >= 16
// runs on MFMA as (Z^T X^T), so each lane owns one row and stores coalesce;
// otherwise one row per thread with P independent FMA sums.
template <typename T, int P, int ZP, typename In, typename Out>
__device__ __forceinline__ void jac_apply(int Np, const T* Z, int t, In xin, Out xout) {
  if constexpr (sizeof(T) == 8 && P >= 16) {
    constexpr int NT16 = P / 16;
    const int w = t / 64, l = t % 64;
    for (int rb = w; rb < Np / 16; rb += JAC_NT / 64) {
      jac_d4 acc[NT16];
#pragma unroll
      for (int c = 0; c < NT16; ++c) acc[c] = jac_d4{0.0, 0.0, 0.0, 0.0};
      const int row = rb * 16 + (l % 16);
#pragma unroll 2
      for (int k0 = 0; k0 < P; k0 += 4) {
        const double xb = xin(row, k0 + l / 16);
#pragma unroll
        for (int c = 0; c < NT16; ++c) {
          const double za = Z[(k0 + l / 16) * ZP + c * 16 + (l % 16)];
          acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(za, xb, acc[c], 0, 0, 0);
        }
      }
#pragma unroll
      for (int c = 0; c < NT16; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) xout(rb * 16 + (l % 16), c * 16 + l / 16 + 4 * v, acc[c][v]);
    }
  } else {
    for (int row = t; row < Np; row += JAC_NT) {
      T acc[P];
#pragma unroll
      for (int j = 0; j < P; ++j) acc[j] = T(0);
#pragma unroll 1
      for (int k = 0; k < P; ++k) {
        const T xk = xin(row, k);
        const T* zr = Z + k * ZP;
#pragma unroll
        for (int j = 0; j < P; ++j) acc[j] = fma(xk, zr[j], acc[j]);
      }
#pragma unroll
      for (int j = 0; j < P; ++j) xout(row, j, acc[j]);
    }
  }
}

template <typename T, int BW>
__global__ __launch_bounds__(JAC_NT) void jacobi_kernel(const Rec* __restrict__ recs, JacArgs a, int sweep,
                                                        int round) {
  extern __shared__ __attribute__((aligned(16))) unsigned char jac_smem[];
  constexpr int P = 2 * BW;  // panel columns
  constexpr int NP2 = P / 2;
  constexpr int ZP = P + 1;  // row stride of Z: a column of Z spreads over the LDS banks
  const Rec& rec = recs[blockIdx.y];
  int32_t* cnt = at<int32_t>(rec, WS, a.off_cnt);
  const int Np = a.Np;
  const int nb = Np / BW;
  const bool single = (nb == 2);
  if (!single && sweep > 0 && cnt[sweep - 1] == 0) return;
  T* Bm = at<T>(rec, WS, a.off_B);
  T* Vm = at<T>(rec, WS, a.off_V);
  int I, J;
  if (single) { I = 0; J = 1; }
  else tour_pair(nb, round, blockIdx.x, &I, &J);

  const int LDP = Np + 16 / (int)sizeof(T);  // padded column stride, keeps 16-byte alignment
  T* pb = reinterpret_cast<T*>(jac_smem);   // panel: column c at pb + c*LDP
  T* G = pb + (size_t)P * LDP;               // G[i*P + j]
  T* Z = G + P * P;                          // Z(i, j) at Z[i*ZP + j] (row-major)
  T* rc = Z + P * ZP;                        // rotation c, s per pair of a step
  T* rsn = rc + NP2;
  __shared__ int pp[P / 2], qq[P / 2];
  __shared__ int wg_rot, pass_rot, any_rot, any_off;
  const int t = threadIdx.x;
  if (t == 0) { wg_rot = 0; any_rot = 0; }

  auto gcol = [&](int c) { return c < BW ? I * BW + c : J * BW + (c - BW); };
  // ---- load the panel (16-byte vectors, coalesced along the rows)
  constexpr int VE = 16 / sizeof(T);
  typedef __attribute__((__vector_size__(16))) T vec_t;
  {
    const int nv = Np / VE, cpp = JAC_NT / 256;  // columns per pass when nv <= 256
    const int lane = (nv <= 256) ? t % 256 : t, c0 = (nv <= 256) ? t / 256 : 0, cst = (nv <= 256) ? cpp : 1;
    const int vst = (nv <= 256) ? 256 : JAC_NT;
#pragma unroll 4
    for (int c = c0; c < P; c += cst) {
      const vec_t* src = reinterpret_cast<const vec_t*>(Bm + (int64_t)gcol(c) * Np);
      vec_t* dst = reinterpret_cast<vec_t*>(pb + (size_t)c * LDP);
      for (int v = lane; v < nv; v += vst) dst[v] = src[v];
    }
  }
  const T tol = T(a.tol);
  int sw = sweep;
  for (;;) {
    if (t == 0) pass_rot = 0;
    __syncthreads();
    // ---- 1. Gram of the panel
    jac_gram<T, P>(pb, Np, LDP, G, Z, t);
    if (t == 0) any_off = 0;
    __syncthreads();
    for (int e = t; e < P * P; e += JAC_NT) {
      const int i = e / P, j = e % P;
      Z[i * ZP + j] = (i == j) ? T(1) : T(0);
      // pairs this visit may rotate: every pair in round 0 / single panel, cross pairs otherwise
      if (i < j && (single || round == 0 || (i < BW && j >= BW))) {
        const T gij = G[e];
        if (gij != T(0) && gij * gij > tol * tol * (G[i * P + i] * G[j * P + j])) any_off = 1;
      }
    }
    __syncthreads();
    // ---- 2. plane rotations on G (G <- J^T G J), accumulating Z <- Z J.
    // Round 0 of a sweep (and the single-panel case) runs a full tournament over
    // the P columns; later rounds only the BW x BW pairs across the two blocks.
    const bool full = single || round == 0;
    const int nsteps = any_off ? (full ? P - 1 : BW) : 0;  // nothing to rotate: skip the sweep
    for (int st = 0; st < nsteps; ++st) {
      if (t < NP2) {
        int p, q;
        if (full) tour_pair(P, st, t, &p, &q);
        else { p = t; q = BW + (t + st) % BW; }
        const T gpp = G[p * P + p], gqq = G[q * P + q], gpq = G[p * P + q];
        T c = T(1), s = T(0);
        if (gpq != T(0) && gpq * gpq > tol * tol * (gpp * gqq)) {
          // tan(2 theta) = b / a with theta in (-pi/4, pi/4]:
          //   cos(2 theta) = |a| / r,  c = sqrt((1 + cos 2theta) / 2),  s = sin(2 theta) / (2 c)
          const T aa = gqq - gpp, bb = T(2) * gpq;
          const T ir = dev_rsqrt(aa * aa + bb * bb);
          const T y = T(0.5) * (T(1) + fabs(aa) * ir);
          const T ry = dev_rsqrt(y);
          c = y * ry;
          s = (aa >= T(0) ? bb : -bb) * ir * T(0.5) * ry;
          atomicAdd(&pass_rot, 1);
        }
        rc[t] = c;
        rsn[t] = s;
        pp[t] = p;
        qq[t] = q;
      }
      __syncthreads();
      // each 2x2 block (pair A rows, pair B columns) of G: J_A^T G_AB J_B
      for (int e = t; e < NP2 * NP2; e += JAC_NT) {
        const int ia = e / NP2, ib = e % NP2;
        const T sa = rsn[ia], sb = rsn[ib];
        if (sa == T(0) && sb == T(0)) continue;
        const T ca = rc[ia], cb = rc[ib];
        const int pa = pp[ia], qa = qq[ia], pbb = pp[ib], qb = qq[ib];
        const T g00 = G[pa * P + pbb], g01 = G[pa * P + qb], g10 = G[qa * P + pbb], g11 = G[qa * P + qb];
        const T r00 = cb * g00 - sb * g01, r01 = sb * g00 + cb * g01;
        const T r10 = cb * g10 - sb * g11, r11 = sb * g10 + cb * g11;
        G[pa * P + pbb] = ca * r00 - sa * r10;
        G[qa * P + pbb] = sa * r00 + ca * r10;
        G[pa * P + qb] = ca * r01 - sa * r11;
        G[qa * P + qb] = sa * r01 + ca * r11;
      }
      for (int e = t; e < NP2 * P; e += JAC_NT) {
        const int ia = e / P, i = e % P;
        const T sa = rsn[ia];
        if (sa == T(0)) continue;
        const T ca = rc[ia];
        const int pa = pp[ia], qa = qq[ia];
        const T zp = Z[i * ZP + pa], zq = Z[i * ZP + qa];
        Z[i * ZP + pa] = ca * zp - sa * zq;
        Z[i * ZP + qa] = sa * zp + ca * zq;
      }
      __syncthreads();
    }
    const int nrot = pass_rot;
    if (nrot > 0) {
      // ---- 3. C <- C Z in LDS, then V_panel <- V_panel Z in global memory
      jac_apply<T, P, ZP>(
          Np, Z, t, [&](int row, int k) { return pb[(size_t)k * LDP + row]; },
          [&](int row, int j, T v) { pb[(size_t)j * LDP + row] = v; });
      jac_apply<T, P, ZP>(
          Np, Z, t, [&](int row, int k) { return Vm[row + (int64_t)gcol(k) * Np]; },
          [&](int row, int j, T v) { Vm[row + (int64_t)gcol(j) * Np] = v; });
      if (t == 0) { wg_rot += nrot; any_rot = 1; }
    }
    __syncthreads();
    if (!single) break;
    if (t == 0) cnt[sw] = nrot;
    ++sw;
    if (nrot == 0 || sw >= a.max_sweeps) break;
  }
  __syncthreads();
  if (any_rot) {
    const int nv = Np / VE, cpp = JAC_NT / 256;
    const int lane = (nv <= 256) ? t % 256 : t, c0 = (nv <= 256) ? t / 256 : 0, cst = (nv <= 256) ? cpp : 1;
    const int vst = (nv <= 256) ? 256 : JAC_NT;
#pragma unroll 4
    for (int c = c0; c < P; c += cst) {
      vec_t* dst = reinterpret_cast<vec_t*>(Bm + (int64_t)gcol(c) * Np);
      const vec_t* src = reinterpret_cast<const vec_t*>(pb + (size_t)c * LDP);
      for (int v = lane; v < nv; v += vst) dst[v] = src[v];
    }
  }
  if (!single && t == 0 && wg_rot > 0) atomicAdd(&cnt[sweep], wg_rot);
}

// ---------------------------------------------------------------------------
// Streamed-panel variants (FP64).  P = 64: panels of two 32-column blocks.
//
// Same visit as above (Gram of the panel, one sweep of plane rotations on the
// Gram, panel and V times the accumulated rotation), but the panel is not
// staged in LDS: the Gram and the products read B and V straight from global
// memory as MFMA operands.  LDS holds only the 64 x 64 Gram and rotation
// (65 KB), so two workgroups share a CU, and the wider panel halves the
// number of visits per sweep (and the panel traffic) relative to 32 columns.
//
// Gram: waves (row quarter q = w % 4, tile group g = w / 4) read each of
// their column blocks once per 16-row step (each lane four consecutive rows
// of its column, fed to four MFMA steps); group 0 holds the upper 16 x 16
// tiles (0,0) (0,1) (0,2) (0,3) (1,1), group 1 (1,2) (1,3) (2,2) (2,3) (3,3).
// The four row quarters are summed in a fixed order through LDS.
// ---------------------------------------------------------------------------
constexpr int JG_NT = 512;
constexpr int JG_P = 64, JG_BW = 32;
template <typename T> constexpr int JG_LDS = (64 * 64 + 64 * 65) * (int)sizeof(T);  // G and Z

// MFMA 16x16x4 in the precision of the panel: FP64 (v_mfma_f64_16x16x4) or FP32
// (v_mfma_f32_16x16x4).  Both take one A and one B element per lane (A: row
// lane % 16, k lane / 16; B: k lane / 16, column lane % 16) and leave four
// results per lane in column lane % 16; the rows differ: result v of a lane is
// row lane / 16 + 4 v in FP64 and row 4 (lane / 16) + v in FP32 (row()).
template <typename T> struct JgMma;
template <> struct JgMma<double> {
  typedef jac_d4 v4;
  static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <> struct JgMma<float> {
  typedef __attribute__((__vector_size__(4 * sizeof(float)))) float v4;
  static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

__device__ __forceinline__ void jg_pair(bool full, int st, int ia, int* p, int* q) {
  // full: circle method over 64 columns (st < 63); otherwise cross pairs (st < 32)
  if (full) {
    if (ia == 0) { *p = st; *q = 63; }
    else {
      int x = st + ia, y = st - ia;
      x -= x >= 63 ? 63 : 0;
      y += y < 0 ? 63 : 0;
      *p = x;
      *q = y;
    }
  } else {
    *p = ia;
    *q = JG_BW + ((ia + st) & (JG_BW - 1));
  }
}

// tile u of group g: (block a, block b) of 16 panel columns each
__device__ __forceinline__ constexpr int jg_tile_a(int g, int u) { return g ? (u < 2 ? 1 : u < 4 ? 2 : 3) : (u < 4 ? 0 : 1); }
__device__ __forceinline__ constexpr int jg_tile_b(int g, int u) {
  return g ? (u == 0 || u == 2 ? 2 : 3) : (u < 4 ? u : 1);
}

// Partial Gram tiles of group GRP over the 16-row steps q, q + 4, ... of the
// panel (cp[i]: this lane's rows in column block i), the next step in flight.
template <typename T, int GRP>
__device__ __forceinline__ void jg_gram_part(const T* const* cp, int Ns, int q, typename JgMma<T>::v4* acc) {
  typedef typename JgMma<T>::v4 V4;
  constexpr int B0 = GRP;  // group 1 never reads column block 0
#pragma unroll
  for (int u = 0; u < 5; ++u) acc[u] = V4{T(0), T(0), T(0), T(0)};
  V4 x[4], y[4];
  int st = q;
  if (st < Ns)
#pragma unroll
    for (int i = B0; i < 4; ++i) x[i] = *reinterpret_cast<const V4*>(cp[i] + 16 * st);
  for (; st < Ns; st += 4) {
    if (st + 4 < Ns)
#pragma unroll
      for (int i = B0; i < 4; ++i) y[i] = *reinterpret_cast<const V4*>(cp[i] + 16 * (st + 4));
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int u = 0; u < 5; ++u)
        acc[u] = JgMma<T>::mma(x[jg_tile_a(GRP, u)][e], x[jg_tile_b(GRP, u)][e], acc[u]);
#pragma unroll
    for (int i = B0; i < 4; ++i) x[i] = y[i];
  }
}

// rotation (c, s) zeroing the (p, q) entry of a Gram, or false when the pair is
// already orthogonal to tolerance (c = 1, s = 0)
template <typename T>
__device__ __forceinline__ bool jg_rot(T gpp, T gqq, T gpq, T tol, T* c, T* s) {
  *c = T(1);
  *s = T(0);
  if (gpq != T(0) && gpq * gpq > tol * tol * (gpp * gqq)) {
    const T aa = gqq - gpp, bb = T(2) * gpq;
    const T ir = dev_rsqrt(aa * aa + bb * bb);
    const T yy = T(0.5) * (T(1) + fabs(aa) * ir);
    const T ry = dev_rsqrt(yy);
    *c = yy * ry;
    *s = (aa >= T(0) ? bb : -bb) * ir * T(0.5) * ry;
    return true;
  }
  return false;
}

// J_A^T g J_B for the 2 x 2 block g = {(pa, pb), (pa, qb), (qa, pb), (qa, qb)}
template <typename T>
__device__ __forceinline__ void jg_rot_block(T ca, T sa, T cb, T sb, T* g) {
  const T r00 = cb * g[0] - sb * g[1], r01 = sb * g[0] + cb * g[1];
  const T r10 = cb * g[2] - sb * g[3], r11 = sb * g[2] + cb * g[3];
  g[0] = ca * r00 - sa * r10;
  g[2] = sa * r00 + ca * r10;
  g[1] = ca * r01 - sa * r11;
  g[3] = sa * r01 + ca * r11;
}

template <typename T>
__global__ __launch_bounds__(JG_NT, 4) void jacobi_g_kernel(const Rec* __restrict__ recs, JacArgs a, int sweep,
                                                            int round) {
  extern __shared__ __attribute__((aligned(16))) unsigned char jg_smem[];
  constexpr int P = JG_P, BW = JG_BW, NP2 = P / 2;
  constexpr int ZP = P + 1;  // row stride of Z
  typedef typename JgMma<T>::v4 V4;
  T* G = reinterpret_cast<T*>(jg_smem);  // G[i*P + j]
  T* Z = G + P * P;                      // Z[i*ZP + j]
  T* slot = G;                           // Gram partials (5 tiles x 256 per slot), before G is formed
  __shared__ T rc[NP2], rsn[NP2];
  __shared__ T hc[2][NP2], hs[2][NP2];  // cross rounds: rotations of the current and next step
  __shared__ int pass_rot, any_off, step_any[2];
  const Rec& rec = recs[blockIdx.y];
  int32_t* cnt = at<int32_t>(rec, WS, a.off_cnt);
  const int Np = a.Np, Ns = Np / 16;
  const int nb = Np / BW;  // >= 4
  if (sweep > 0 && cnt[sweep - 1] == 0) return;
  T* Bm = at<T>(rec, WS, a.off_B);
  T* Vm = at<T>(rec, WS, a.off_V);
  int I, J;
  tour_pair(nb, round, blockIdx.x, &I, &J);
  auto gcol = [&](int c) { return c < BW ? I * BW + c : J * BW + (c - BW); };
  const int t = threadIdx.x, w = t / 64, l = t % 64;
  const T tol = T(a.tol);
  const bool full = round == 0;

  // ---- 1. Gram
  {
    const int q = w & 3, grp = w >> 2;
    const T* cp[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) cp[i] = Bm + (int64_t)gcol(16 * i + (l & 15)) * Np + 4 * (l >> 4);
    V4 acc[5];
    if (grp == 0) jg_gram_part<T, 0>(cp, Ns, q, acc);
    else jg_gram_part<T, 1>(cp, Ns, q, acc);
    // fixed-order sum over the row quarters: (q0 + q2) + (q1 + q3)
    auto put = [&](int sl) {
      T* d = slot + sl * 1280;
#pragma unroll
      for (int u = 0; u < 5; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) d[u * 256 + v * 64 + l] = acc[u][v];
    };
    auto add = [&](int sl) {
      const T* d = slot + sl * 1280;
#pragma unroll
      for (int u = 0; u < 5; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += d[u * 256 + v * 64 + l];
    };
    if (q >= 2) put(grp * 2 + (q - 2));
    __syncthreads();
    if (q < 2) add(grp * 2 + q);
    __syncthreads();
    if (q == 1) put(grp);
    __syncthreads();
    if (q == 0) add(grp);
    __syncthreads();
    if (q == 0) {
#pragma unroll
      for (int u = 0; u < 5; ++u) {
        const int ta = jg_tile_a(grp, u), tb = jg_tile_b(grp, u);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * ta + JgMma<T>::row(l, v), j = 16 * tb + (l & 15);
          G[i * P + j] = acc[u][v];
          if (ta != tb) G[j * P + i] = acc[u][v];
        }
      }
    }
  }
  if (t == 0) { any_off = 0; pass_rot = 0; step_any[0] = 0; }
  __syncthreads();
  for (int e = t; e < P * P; e += JG_NT) {
    const int i = e / P, j = e % P;
    Z[i * ZP + j] = (i == j) ? T(1) : T(0);
    if (i < j && (full || (i < BW && j >= BW))) {
      const T gij = G[e];
      if (gij != T(0) && gij * gij > tol * tol * (G[i * P + i] * G[j * P + j])) any_off = 1;
    }
  }
  __syncthreads();

  // ---- 2. plane rotations on G, accumulating Z
  const int nsteps = any_off ? (full ? P - 1 : BW) : 0;
  int nrot = 0;
  if (full) {
    // first round of a sweep: all pairs of the panel (circle method), Z in LDS
    for (int st = 0; st < nsteps; ++st) {
      if (t < NP2) {
        int p, q;
        jg_pair(true, st, t, &p, &q);
        T c, sn;
        if (jg_rot(G[p * P + p], G[q * P + q], G[p * P + q], tol, &c, &sn)) {
          ++nrot;
          step_any[st & 1] = 1;
        }
        rc[t] = c;
        rsn[t] = sn;
      }
      __syncthreads();
      // a step in which no pair rotates leaves G and Z as they are: skip its update
      // (the flag of the next step is cleared here, after everyone has read its last use)
      const bool upd = step_any[st & 1] != 0;
      if (t == 0) step_any[(st + 1) & 1] = 0;
      if (upd) {
        // thread: pair ib = t % 32 (columns) with pairs t/32 and t/32 + 16 (rows) of G,
        // and rows t/32 + 16k (k < 4) of Z in the columns of pair ib; every read first
        const int ib = t & 31, r0 = t >> 5;
        int pb, qb, pa[2], qa[2];
        jg_pair(true, st, ib, &pb, &qb);
        const T cb = rc[ib], sb = rsn[ib];
        T ca[2], sa[2], g[2][4], zv[4][2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int ia = r0 + 16 * k;
          jg_pair(true, st, ia, &pa[k], &qa[k]);
          ca[k] = rc[ia];
          sa[k] = rsn[ia];
          g[k][0] = G[pa[k] * P + pb];
          g[k][1] = G[pa[k] * P + qb];
          g[k][2] = G[qa[k] * P + pb];
          g[k][3] = G[qa[k] * P + qb];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int iz = r0 + 16 * k;
          zv[k][0] = Z[iz * ZP + pb];
          zv[k][1] = Z[iz * ZP + qb];
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          jg_rot_block(ca[k], sa[k], cb, sb, g[k]);
          G[pa[k] * P + pb] = g[k][0];
          G[pa[k] * P + qb] = g[k][1];
          G[qa[k] * P + pb] = g[k][2];
          G[qa[k] * P + qb] = g[k][3];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int iz = r0 + 16 * k;
          Z[iz * ZP + pb] = cb * zv[k][0] - sb * zv[k][1];
          Z[iz * ZP + qb] = sb * zv[k][0] + cb * zv[k][1];
        }
        __syncthreads();
      }
    }
  } else if (nsteps > 0) {
    // Later rounds: the BW x BW cross pairs, pair i = (i, BW + (i + st) % BW) at
    // step st.  G is symmetric and is only read again through its upper half,
    // so a step updates the 2 x 2 blocks (a, b) with a <= b only (528 of 1024)
    // and keeps the entries on and above the diagonal of the two diagonal
    // quadrants and the whole upper-right quadrant.  One barrier per step:
    // lanes i < 32 of wave 0 rotate the blocks (i, i) and {i, i + 1}, which
    // hold every entry the pair i of the next step needs (the third one comes
    // from lane i + 1), and compute that rotation at once; 464 other threads
    // rotate one block each.
    // Z stays in registers: thread t owns rows t/32 + 16k (k < 4) in column t%32
    // (zp) and in the column paired with it at the current step (zq); the
    // pairing advances by one column per step, a rotation of zq across the 32
    // lanes that share the rows.
    // Z and the other blocks live in waves 1..7 only, so wave 0 runs nothing but
    // the step's critical path.  Z: half-wave h = t/32 - 2 (0..13) owns rows
    // h + 14k (k < 5, rows < 64) in column t%32 and in its current partner.
    const int zib = t & 31, zh = (t >> 5) - 2;
    T zp[5], zq[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const int iz = zh + 14 * k;
      zp[k] = iz == zib ? T(1) : T(0);
      zq[k] = iz == BW + zib ? T(1) : T(0);
    }
    const int zsrc = (l & 32) | ((l + 1) & 31);  // lane holding the next step's column
    // storage of the block (a, b), a <= b: (a, b), (a, qb), (b, qa) [= (qa, b)], (min, max of qa, qb)
    auto blk_off = [&](int a, int b, int qa, int qb, int* o) {
      o[0] = a * P + b;
      o[1] = a * P + qb;
      o[2] = b * P + qa;
      o[3] = qa <= qb ? qa * P + qb : qb * P + qa;
    };
    // the blocks besides wave 0's, on waves 1..7 (448 threads; 16 take two):
    // e < 448 -> distance 2 + e / 32, e < 464 -> distance 16
    int oa[2] = {-1, -1}, ob[2] = {-1, -1};
    if (t >= 64) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int e = (t - 64) + 448 * h;
        if (e < 448) {
          const int x = e & (BW - 1), y = (x + 2 + (e >> 5)) & (BW - 1);
          oa[h] = min(x, y);
          ob[h] = max(x, y);
        } else if (e < 464) {
          oa[h] = e - 448;
          ob[h] = oa[h] + 16;
        }
      }
    }
    // lanes i < 32 of wave 0 carry their blocks (i, i) = {d0 d1; d1 d3} and
    // (i, i + 1) = {e00 e01; e10 e11} (rows of pair i, columns of pair i + 1)
    // from step to step in registers: after a step, pair i moves to the second-
    // block column of pair i + 1, so the new blocks consist of the lane's own
    // results, three results of lane i + 1, and one entry rotated by the owner
    // of the block (i, i + 2), read back from LDS.
    T d0 = T(0), d1 = T(0), d3 = T(0), e00 = T(0), e01 = T(0), e10 = T(0), e11 = T(0), ci = T(1), si = T(0);
    if (t < NP2) {  // step 0 from the Gram (still complete)
      const int i = t, j = (i + 1) & (BW - 1), qi = BW + i, qj = BW + j;
      d0 = G[i * P + i];
      d1 = G[i * P + qi];
      d3 = G[qi * P + qi];
      e00 = G[i * P + j];
      e01 = G[i * P + qj];
      e10 = G[qi * P + j];
      e11 = G[qi * P + qj];
      if (jg_rot(d0, d3, d1, tol, &ci, &si)) ++nrot;
      hc[0][t] = ci;
      hs[0][t] = si;
    }
    __syncthreads();
    for (int st = 0; st < BW; ++st) {
      const int cur = st & 1;
      if (t < NP2) {
        const int i = t, j = (t + 1) & (BW - 1);
        const int qi = BW + ((i + st) & (BW - 1)), qj = BW + ((j + st) & (BW - 1));
        if (st > 0) e01 = G[i * P + qj];  // rotated last step by the owner of the block (i, i + 2)
        const T cj = __shfl(ci, j), sj = __shfl(si, j);
        T gd[4] = {d0, d1, d1, d3};
        T ge[4] = {e00, e01, e10, e11};
        jg_rot_block(ci, si, ci, si, gd);
        jg_rot_block(ci, si, cj, sj, ge);
        G[i * P + i] = gd[0];
        G[i * P + qi] = gd[1];
        G[qi * P + qi] = gd[3];
        G[min(i, j) * P + max(i, j)] = ge[0];
        G[i * P + qj] = ge[1];
        G[j * P + qi] = ge[2];
        G[min(qi, qj) * P + max(qi, qj)] = ge[3];
        // step st + 1: pair i = (i, qj); blocks {i, qj} x {i, qj} and {i, qj} x {j, qk}
        d0 = gd[0];
        d1 = ge[1];
        e00 = ge[0];
        d3 = __shfl(gd[3], j);
        e10 = __shfl(gd[1], j);
        e11 = __shfl(ge[3], j);
        if (st + 1 < BW) {
          if (jg_rot(d0, d3, d1, tol, &ci, &si)) ++nrot;
          hc[cur ^ 1][i] = ci;
          hs[cur ^ 1][i] = si;
        }
      } else if (t >= 64) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (oa[h] < 0) continue;
          const int a = oa[h], b = ob[h];
          const int qa = BW + ((a + st) & (BW - 1)), qb = BW + ((b + st) & (BW - 1));
          int o[4];
          blk_off(a, b, qa, qb, o);
          T g[4] = {G[o[0]], G[o[1]], G[o[2]], G[o[3]]};
          jg_rot_block(hc[cur][a], hs[cur][a], hc[cur][b], hs[cur][b], g);
          G[o[0]] = g[0];
          G[o[1]] = g[1];
          G[o[2]] = g[2];
          G[o[3]] = g[3];
        }
        const T cz = hc[cur][zib], sz = hs[cur][zib];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          const T x = zp[k], y = zq[k];
          zp[k] = cz * x - sz * y;
          zq[k] = sz * x + cz * y;
        }
        if (st + 1 < BW)
#pragma unroll
          for (int k = 0; k < 5; ++k) zq[k] = __shfl(zq[k], zsrc);
      }
      __syncthreads();
    }
    // Z back to LDS for the panel products (the last step paired zib with BW + (zib + BW - 1) % BW)
    if (t >= 64)
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        const int iz = zh + 14 * k;
        if (iz >= P) continue;
        Z[iz * ZP + zib] = zp[k];
        Z[iz * ZP + BW + ((zib + BW - 1) & (BW - 1))] = zq[k];
      }
  }
  __syncthreads();
  if (t < 64) {  // rotations counted by the lanes that chose them (wave 0)
    int tot = nrot;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off);
    if (t == 0) pass_rot = tot;
  }
  __syncthreads();
  const int nrt = pass_rot;
  if (nrt == 0) return;

  // ---- 3. [B_I B_J] <- [B_I B_J] Z and [V_I V_J] <- [V_I V_J] Z, as (Z^T X^T) on MFMA
  int co[16];
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) co[kk] = gcol(4 * kk + (l >> 4)) * Np;
  const int njobs = 2 * Ns;  // (matrix, 16-row block)
  for (int job = w; job < njobs; job += JG_NT / 64) {
    const int64_t rofs = (job < Ns ? job : job - Ns) * 16 + (l & 15);
    T* X = (job < Ns ? Bm : Vm) + rofs;
    V4 acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = V4{T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int half = 0; half < 2; ++half) {  // k in two halves of 32 panel columns
      T xb[8];
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) xb[kk] = X[co[8 * half + kk]];
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        const int k = 4 * (8 * half + kk) + (l >> 4);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const T za = Z[k * ZP + 16 * c + (l & 15)];
          acc[c] = JgMma<T>::mma(za, xb[kk], acc[c]);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) X[(int64_t)gcol(16 * c + JgMma<T>::row(l, v)) * Np] = acc[c][v];
  }
  if (t == 0) atomicAdd(&cnt[sweep], nrt);
}

// P = 32 (two 16-column blocks), four waves, several workgroups per CU.  The
// Gram is split over the waves by 16-row steps and their partial tiles are
// summed in a fixed order; one wave runs the plane rotations on the 32 x 32
// Gram with no workgroup barrier between steps (a wave's LDS accesses are
// performed in program order); the panel products keep the rotation's MFMA
// operands in registers and prefetch the next 16-row block of the panel.
constexpr int JS_NT = 256, JS_P = 32, JS_BW = 16;


__device__ __forceinline__ void js_pair(bool full, int st, int ia, int* p, int* q) {
  if (full) tour_pair(JS_P, st, ia, p, q);
  else { *p = ia; *q = JS_BW + (ia + st) % JS_BW; }
}

__global__ __launch_bounds__(JS_NT, 3) void jacobi_s_kernel(const Rec* __restrict__ recs, JacArgs a, int sweep,
                                                            int round) {
  constexpr int P = JS_P, BW = JS_BW, NR = P / 2, NW = JS_NT / 64;
  constexpr int ZS = P + 1;  // row stride of Z: a column of Z spreads over the LDS banks
  __shared__ __attribute__((aligned(16))) double G[P * P];
  __shared__ __attribute__((aligned(16))) double red[NW * 3 * 256];  // Gram partials; Z (P x ZS) reuses it
  __shared__ double rc[NR], rsn[NR];
  __shared__ int pass_rot, any_off;
  double* Z = red;
  const Rec& rec = recs[blockIdx.y];
  int32_t* cnt = at<int32_t>(rec, WS, a.off_cnt);
  const int Np = a.Np, Ns = Np / 16;
  if (sweep > 0 && cnt[sweep - 1] == 0) return;
  double* Bm = at<double>(rec, WS, a.off_B);
  double* Vm = at<double>(rec, WS, a.off_V);
  int I, J;
  tour_pair(Np / BW, round, blockIdx.x, &I, &J);
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const double tol = a.tol;
  const bool full = round == 0;

  // ---- 1. Gram of the panel [B_I B_J]
  {
    const int r0 = 4 * (l >> 4);
    const double* ca = Bm + (int64_t)(I * BW + (l & 15)) * Np + r0;
    const double* cb = Bm + (int64_t)(J * BW + (l & 15)) * Np + r0;
    jac_d4 g00 = {0.0, 0.0, 0.0, 0.0}, g01 = g00, g11 = g00;
    jac_d4 xa = g00, xb = g00, ya = g00, yb = g00, za = g00, zb = g00;  // two 16-row steps ahead
    int st = w;
    if (st < Ns) {
      xa = *reinterpret_cast<const jac_d4*>(ca + 16 * st);
      xb = *reinterpret_cast<const jac_d4*>(cb + 16 * st);
    }
    if (st + NW < Ns) {
      ya = *reinterpret_cast<const jac_d4*>(ca + 16 * (st + NW));
      yb = *reinterpret_cast<const jac_d4*>(cb + 16 * (st + NW));
    }
    for (; st < Ns; st += NW) {
      if (st + 2 * NW < Ns) {
        za = *reinterpret_cast<const jac_d4*>(ca + 16 * (st + 2 * NW));
        zb = *reinterpret_cast<const jac_d4*>(cb + 16 * (st + 2 * NW));
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        g00 = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[e], xa[e], g00, 0, 0, 0);
        g01 = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[e], xb[e], g01, 0, 0, 0);
        g11 = __builtin_amdgcn_mfma_f64_16x16x4f64(xb[e], xb[e], g11, 0, 0, 0);
      }
      xa = ya;
      xb = yb;
      ya = za;
      yb = zb;
    }
    double* rw = red + w * 768;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int e = ((l >> 4) + 4 * v) * 16 + (l & 15);
      rw[e] = g00[v];
      rw[256 + e] = g01[v];
      rw[512 + e] = g11[v];
    }
  }
  if (t == 0) { any_off = 0; pass_rot = 0; }
  __syncthreads();
  for (int e = t; e < 768; e += JS_NT) {
    const double x = ((red[e] + red[768 + e]) + red[1536 + e]) + red[2304 + e];
    const int tile = e >> 8, i = (e >> 4) & 15, j = e & 15;
    const int ti = tile == 2 ? 16 : 0, tj = tile == 0 ? 0 : 16;
    G[(ti + i) * P + tj + j] = x;
    if (tile == 1) G[(16 + j) * P + i] = x;
  }
  __syncthreads();
  for (int e = t; e < P * P; e += JS_NT) {
    const int i = e >> 5, j = e & 31;
    Z[i * ZS + j] = (i == j) ? 1.0 : 0.0;
    if (i < j && (full || (i < BW && j >= BW))) {
      const double gij = G[e];
      if (gij != 0.0 && gij * gij > tol * tol * (G[i * P + i] * G[j * P + j])) any_off = 1;
    }
  }
  __syncthreads();

  // ---- 2. plane rotations on G, accumulated into Z, by wave 0
  if (w == 0 && any_off) {
    const int nsteps = full ? P - 1 : BW;
    int nrot = 0;
    for (int st = 0; st < nsteps; ++st) {
      bool rot = false;
      if (l < NR) {
        int p, q;
        js_pair(full, st, l, &p, &q);
        const double gpp = G[p * P + p], gqq = G[q * P + q], gpq = G[p * P + q];
        double c = 1.0, sn = 0.0;
        if (gpq != 0.0 && gpq * gpq > tol * tol * (gpp * gqq)) {
          const double aa = gqq - gpp, bb = 2.0 * gpq;
          const double ir = dev_rsqrt(aa * aa + bb * bb);
          const double y = 0.5 * (1.0 + fabs(aa) * ir);
          const double ry = dev_rsqrt(y);
          c = y * ry;
          sn = (aa >= 0.0 ? bb : -bb) * ir * 0.5 * ry;
          rot = true;
        }
        rc[l] = c;
        rsn[l] = sn;
      }
      const int nr = __popcll(__ballot(rot));
      nrot += nr;
      wave_sync();
      if (nr == 0) continue;  // nothing rotates in this step: G and Z stay as they are
      // lane l: 2x2 blocks (pair l/16 + 4k, pair l%16) of G, k < 4, and rows
      // l/16 + 4k, k < 8, of Z in the columns of pair l%16.  All operands are
      // read before any result is written (the blocks and Z entries of one
      // step are disjoint), so the reads overlap; a pair with s = 0 is an
      // exact identity and needs no test.
      int pg[4], qg[4], pb, qb;
      double cg[4], sg[4], g[4][4], zv[8][2];
      const int ib = l & 15;
      js_pair(full, st, ib, &pb, &qb);
      const double cb = rc[ib], sb = rsn[ib];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int ia = (l >> 4) + 4 * k;
        js_pair(full, st, ia, &pg[k], &qg[k]);
        cg[k] = rc[ia];
        sg[k] = rsn[ia];
        g[k][0] = G[pg[k] * P + pb];
        g[k][1] = G[pg[k] * P + qb];
        g[k][2] = G[qg[k] * P + pb];
        g[k][3] = G[qg[k] * P + qb];
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int iz = (l >> 4) + 4 * k;
        zv[k][0] = Z[iz * ZS + pb];
        zv[k][1] = Z[iz * ZS + qb];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double ca = cg[k], sa = sg[k];
        const double r00 = cb * g[k][0] - sb * g[k][1], r01 = sb * g[k][0] + cb * g[k][1];
        const double r10 = cb * g[k][2] - sb * g[k][3], r11 = sb * g[k][2] + cb * g[k][3];
        G[pg[k] * P + pb] = ca * r00 - sa * r10;
        G[qg[k] * P + pb] = sa * r00 + ca * r10;
        G[pg[k] * P + qb] = ca * r01 - sa * r11;
        G[qg[k] * P + qb] = sa * r01 + ca * r11;
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int iz = (l >> 4) + 4 * k;
        Z[iz * ZS + pb] = cb * zv[k][0] - sb * zv[k][1];
        Z[iz * ZS + qb] = sb * zv[k][0] + cb * zv[k][1];
      }
      wave_sync();
    }
    if (l == 0) pass_rot = nrot;
  }
  __syncthreads();
  const int nrot = pass_rot;
  if (nrot == 0) return;

  // ---- 3. [B_I B_J] <- [B_I B_J] Z and [V_I V_J] <- [V_I V_J] Z, as (Z^T X^T) on MFMA
  double za[2][8];
#pragma unroll
  for (int kk = 0; kk < 8; ++kk) {
    za[0][kk] = Z[(4 * kk + (l >> 4)) * ZS + (l & 15)];
    za[1][kk] = Z[(4 * kk + (l >> 4)) * ZS + 16 + (l & 15)];
  }
  int co[8], oo[8];  // source column offsets (k = 4 kk + l/16), destination (16 c + l/16 + 4 v)
#pragma unroll
  for (int kk = 0; kk < 8; ++kk) {
    const int k = 4 * kk + (l >> 4);
    co[kk] = (k < BW ? I * BW + k : J * BW + k - BW) * Np;
    const int c = (kk >> 2) * 16 + (l >> 4) + 4 * (kk & 3);
    oo[kk] = (c < BW ? I * BW + c : J * BW + c - BW) * Np;
  }
  const int njobs = 2 * Ns;  // (matrix, 16-row block)
  double xb[8], yb[8], zb[8];  // the job's panel rows and the next two jobs'
  auto fetch = [&](int jb, double* x) {
    const double* src = (jb < Ns ? Bm : Vm) + (jb < Ns ? jb : jb - Ns) * 16 + (l & 15);
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) x[kk] = src[co[kk]];
  };
  int job = w;
  if (job < njobs) fetch(job, xb);
  if (job + NW < njobs) fetch(job + NW, yb);
  for (; job < njobs; job += NW) {
    if (job + 2 * NW < njobs) fetch(job + 2 * NW, zb);
    jac_d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(za[0][kk], xb[kk], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(za[1][kk], xb[kk], acc1, 0, 0, 0);
    }
    double* dst = (job < Ns ? Bm : Vm) + (job < Ns ? job : job - Ns) * 16 + (l & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      dst[oo[v]] = acc0[v];
      dst[oo[4 + v]] = acc1[v];
    }
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      xb[kk] = yb[kk];
      yb[kk] = zb[kk];
    }
  }
  if (t == 0) atomicAdd(&cnt[sweep], nrot);
}

int jacobi_block_fits(int N, int elem_bytes, int cfg) {
  const int bw = cfg & 0xff;
  if (cfg & JAC_STREAMED) {
    // streamed panels: 32-column blocks in FP64 or FP32, 16-column blocks in FP64;
    // at least four blocks
    if ((cfg & ~(JAC_STREAMED | 0xff)) || (bw != 16 && bw != 32)) return 0;
    if (!(elem_bytes == 8 || (elem_bytes == 4 && bw == 32))) return 0;
    const int Np = ((N + 2 * bw - 1) / (2 * bw)) * (2 * bw);
    return Np / bw >= 4 ? Np : 0;
  }
  if (cfg & ~0xff) return 0;
  if (bw != 4 && bw != 8 && bw != 16 && bw != 32) return 0;
  const int Np = ((N + 2 * bw - 1) / (2 * bw)) * (2 * bw);
  const size_t P = 2 * (size_t)bw;
  const size_t ldp = (size_t)Np + 16 / elem_bytes;
  if ((size_t)Np * P * elem_bytes <= (size_t)JAC_LDS_BYTES && (ldp * P + 2 * P * P + 2 * P) * elem_bytes <= (size_t)JAC_LDS_MAX)
    return Np;
  return 0;
}

int jacobi_pick_block(int N, int elem_bytes, int* Np_out) {
  // largest panel (P = 2 BW <= 64 columns) whose Np x P slice fits the LDS budget
  const int cands[4] = {32, 16, 8, 4};
  for (int ci = 0; ci < 4; ++ci) {
    const int bw = cands[ci];
    const int Np = ((N + 2 * bw - 1) / (2 * bw)) * (2 * bw);
    const size_t P = 2 * (size_t)bw;
    const size_t ldp = (size_t)Np + 16 / elem_bytes;
    if ((size_t)Np * P * elem_bytes <= (size_t)JAC_LDS_BYTES &&
        (ldp * P + 2 * P * P + 2 * P) * elem_bytes <= (size_t)JAC_LDS_MAX) {
      *Np_out = Np;
      return bw;
    }
  }
  return 0;
}

template <typename T, int BW>
static hipError_t jac_launch(const Rec* recs, int nrec, const JacArgs& a, int sweep, int round,
                             hipStream_t s) {
  constexpr int P = 2 * BW;
  const int nb = a.Np / BW;
  const size_t lds = ((size_t)(a.Np + 16 / sizeof(T)) * P + 2 * P * P + 2 * P) * sizeof(T);
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)jacobi_kernel<T, BW>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              JAC_LDS_MAX);
    attr_set = true;
  }
  hipLaunchKernelGGL((jacobi_kernel<T, BW>), dim3(nb / 2, nrec), dim3(JAC_NT), lds, s, recs, a, sweep,
                     round);
  return hipGetLastError();
}

template <typename T>
hipError_t jacobi_round(const Rec* recs, int nrec, const JacArgs& a, int sweep, int round, hipStream_t s) {
  if (a.b & JAC_STREAMED) {
    if ((a.b & 0xff) == JS_BW) {  // 32-column panels: FP64 only
      if (sizeof(T) != 8) return hipErrorInvalidValue;
      hipLaunchKernelGGL(jacobi_s_kernel, dim3(a.Np / JS_BW / 2, nrec), dim3(JS_NT), 0, s, recs, a, sweep, round);
      return hipGetLastError();
    }
    static bool attr = false;
    const size_t lds = JG_LDS<T>;
    if (!attr) {
      (void)hipFuncSetAttribute((const void*)jacobi_g_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
      attr = true;
    }
    hipLaunchKernelGGL(jacobi_g_kernel<T>, dim3(a.Np / JG_BW / 2, nrec), dim3(JG_NT), lds, s, recs, a, sweep, round);
    return hipGetLastError();
  }
  switch (a.b) {
    case 32: return jac_launch<T, 32>(recs, nrec, a, sweep, round, s);
    case 16: return jac_launch<T, 16>(recs, nrec, a, sweep, round, s);
    case 8: return jac_launch<T, 8>(recs, nrec, a, sweep, round, s);
    case 4: return jac_launch<T, 4>(recs, nrec, a, sweep, round, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Finalize.  B and V received the same plane rotations, so B = L^T V up to
// rounding.  Rotations computed in floating point are orthogonal only to a
// few ulps, and over a full iteration the column norms of both drift by the
// same factor (visible in FP32); the eigenvalue estimate ||B_j||^2 / ||V_j||^2
// cancels that factor and W takes the normalised columns of V.  Eigenvalues
// are sorted descending (ties by column index); D and the permuted,
// normalised W are written.  The column norms are formed by many workgroups
// (one wave per column, the eigenvalue estimate stored unsorted in place),
// then one workgroup per problem ranks them.
// ---------------------------------------------------------------------------
constexpr int FIN_MAXN = MAX_CORE;

template <typename TCore>
__global__ __launch_bounds__(256) void fin_norms_kernel(const Rec* __restrict__ recs, FinArgs a) {
  const Rec& rec = recs[blockIdx.y];
  const int N = a.N, Np = a.Np;
  const int j = 4 * blockIdx.x + threadIdx.x / 64, ln = threadIdx.x % 64;
  if (j >= N) return;
  const TCore* col = at<const TCore>(rec, WS, a.off_B) + (int64_t)j * Np;
  const TCore* vc = at<const TCore>(rec, WS, a.off_V) + (int64_t)j * Np;
  TCore* lam = at<TCore>(rec, WS, a.off_lam);
  TCore sb = TCore(0), sv = TCore(0);
  for (int i = ln; i < Np; i += 64) {
    sb = fma(col[i], col[i], sb);
    sv = fma(vc[i], vc[i], sv);
  }
  for (int off = 32; off > 0; off >>= 1) {
    sb += __shfl_xor(sb, off);
    sv += __shfl_xor(sv, off);
  }
  if (ln == 0) {
    const bool ok = sv > TCore(0);
    lam[j] = ok ? sb / sv : sb;                          // unsorted estimate
    lam[Np + j] = ok ? TCore(1) / dev_sqrt(sv) : TCore(1);  // 1 / ||V_j||
  }
}

template <typename TCore, typename TD>
__global__ __launch_bounds__(256) void fin_sort_kernel(const Rec* __restrict__ recs, FinArgs a) {
  const Rec& rec = recs[blockIdx.x];
  const int N = a.N;
  TCore* lam = at<TCore>(rec, WS, a.off_lam);
  int32_t* rank = at<int32_t>(rec, WS, a.off_rank);
  TD* Dout = at<TD>(rec, D_BACK, 0);
  __shared__ TCore sl[FIN_MAXN];
  // the core is PSD: an estimate a rounding error below zero is taken as zero
  for (int j = threadIdx.x; j < N; j += 256) sl[j] = lam[j] > TCore(0) ? lam[j] : TCore(0);
  __syncthreads();  // every estimate is read before the sorted ones overwrite them
  for (int j = threadIdx.x; j < N; j += 256) {
    const TCore v = sl[j];
    int rk = 0;
    for (int i = 0; i < N; ++i) {
      const TCore u = sl[i];
      rk += (u > v) || (u == v && i < j);
    }
    rank[j] = rk;
    lam[rk] = v;
    Dout[rk] = TD(v);
  }
  if (threadIdx.x == 0) {
    const int32_t* cnt = at<const int32_t>(rec, WS, a.off_cnt);
    if (cnt[a.max_sweeps - 1] > 0) atomicOr(at<uint32_t>(rec, STATUS, 0), (uint32_t)KFB_EV_JACOBI_MAXSWEEPS);
  }
}

template <typename TCore, typename TW>
__global__ __launch_bounds__(256) void fin_gather_kernel(const Rec* __restrict__ recs, FinArgs a) {
  const Rec& rec = recs[blockIdx.y];
  const int N = a.N, Np = a.Np;
  const TCore* Vm = at<const TCore>(rec, WS, a.off_V);
  const int32_t* rank = at<const int32_t>(rec, WS, a.off_rank);
  const TCore* vscale = at<const TCore>(rec, WS, a.off_lam) + Np;
  TW* W = at<TW>(rec, WS, a.off_W);
  const int64_t tot = (int64_t)N * N;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % N), j = (int)(e / N);
    W[i + (int64_t)rank[j] * N] = TW(Vm[i + (int64_t)j * Np] * vscale[j]);
  }
}

template <typename TCore, typename TW, typename TD>
hipError_t finalize_core(const Rec* recs, int nrec, const FinArgs& a, hipStream_t s) {
  if (a.N > FIN_MAXN) return hipErrorInvalidValue;
  hipLaunchKernelGGL((fin_norms_kernel<TCore>), dim3((a.N + 3) / 4, nrec), dim3(256), 0, s, recs, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((fin_sort_kernel<TCore, TD>), dim3(nrec), dim3(256), 0, s, recs, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t tot = (int64_t)a.N * a.N;
  int blocks = (int)((tot + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL((fin_gather_kernel<TCore, TW>), dim3(blocks, nrec), dim3(256), 0, s, recs, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Preconditioner coefficients (Algorithm 1 inverse lines; Section 3.5):
//   c_i = 1/(D_i + lam) - 1/lam  per side, with optional spectrum continuation
//   (lam <- lam + min D, D <- D - min D).  Stored, with the 1/lam factors of
//   the cross terms folded in:
//     sG = c_G / lam_A   (rows of U_G^T G)      tG = c_G  (rows of the core)
//     sA = c_A / lam_G   (cols of G U_A)        tA = c_A  (cols of the core)
//     beta = 1 / (lam_G lam_A)                   (the G term), as a double.
// Layout at off_cG: [sG (kG)][tG (kG)]; at off_cA: [sA (kA)][tA (kA)];
// beta at off_cA + 2*kA*sizeof(TAcc) rounded to 8 bytes, then 1/lam_G and
// 1/lam_A (the factored form's X / lam terms).
// ---------------------------------------------------------------------------
template <typename TD, typename TAcc>
__global__ __launch_bounds__(256) void precond_coefs_kernel(const Rec* __restrict__ recs, CoefArgs a) {
  const Rec& rec = recs[blockIdx.x];
  const TD* DG = at<const TD>(rec, PD_G, 0);
  const TD* DA = at<const TD>(rec, PD_A, 0);
  __shared__ double mins[2], lams[2];
  if (threadIdx.x == 0) {
    double lG0 = rec.s[0], lA0 = rec.s[1];
    if (a.flags & KFB_RELATIVE_DAMPING) {  // lam = phi * lambda_max (Section 6)
      double xG = 0.0, xA = 0.0;
      for (int i = 0; i < a.kG; ++i) xG = fmax(xG, (double)DG[i]);
      for (int i = 0; i < a.kA; ++i) xA = fmax(xA, (double)DA[i]);
      lG0 = xG > 0.0 ? lG0 * xG : lG0;
      lA0 = xA > 0.0 ? lA0 * xA : lA0;
    }
    lams[0] = lG0;
    lams[1] = lA0;
    double mG = 0.0, mA = 0.0;
    if (a.flags & KFB_SPECTRUM_CONTINUATION) {
      // smallest positive eigenvalue: a mode of eigenvalue exactly 0 is an
      // empty slot (a dropped null direction of the residual, or the zero
      // padding of an uneven-width batch) with a zero column in U
      mG = INFINITY;
      for (int i = 0; i < a.kG; ++i)
        if ((double)DG[i] > 0.0) mG = fmin(mG, (double)DG[i]);
      mA = INFINITY;
      for (int i = 0; i < a.kA; ++i)
        if ((double)DA[i] > 0.0) mA = fmin(mA, (double)DA[i]);
      if (!(mG < INFINITY)) mG = 0.0;
      if (!(mA < INFINITY)) mA = 0.0;
    }
    mins[0] = mG;
    mins[1] = mA;
  }
  __syncthreads();
  const double mG = mins[0], mA = mins[1];
  const double lG = lams[0] + mG, lA = lams[1] + mA;
  TAcc* cG = at<TAcc>(rec, PWS, a.off_cG);
  TAcc* cA = at<TAcc>(rec, PWS, a.off_cA);
  for (int i = threadIdx.x; i < a.kG; i += 256) {
    const double d = fmax((double)DG[i] - mG, 0.0);
    const double c = 1.0 / (d + lG) - 1.0 / lG;
    cG[i] = TAcc(c / lA);
    cG[a.kG + i] = TAcc(c);
  }
  for (int i = threadIdx.x; i < a.kA; i += 256) {
    const double d = fmax((double)DA[i] - mA, 0.0);
    const double c = 1.0 / (d + lA) - 1.0 / lA;
    cA[i] = TAcc(c / lG);
    cA[a.kA + i] = TAcc(c);
  }
  if (threadIdx.x == 0) {
    const int64_t boff = ((a.off_cA + (int64_t)2 * a.kA * (int64_t)sizeof(TAcc)) + 7) & ~int64_t(7);
    *at<double>(rec, PWS, boff) = 1.0 / (lG * lA);
    *at<double>(rec, PWS, boff + 8) = 1.0 / lG;
    *at<double>(rec, PWS, boff + 16) = 1.0 / lA;
  }
}

template <typename TD, typename TAcc>
hipError_t precond_coefs(const Rec* recs, int nrec, const CoefArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((precond_coefs_kernel<TD, TAcc>), dim3(nrec), dim3(256), 0, s, recs, a);
  return hipGetLastError();
}

template <typename T, typename TS>
__global__ __launch_bounds__(256) void scale2d_kernel(const Rec* __restrict__ recs, ScaleArgs a) {
  const Rec& rec = recs[blockIdx.y];
  T* X = at<T>(rec, a.X.slot, a.X.off);
  const TS* rs = a.row_slot >= 0 ? at<const TS>(rec, a.row_slot, a.row_off) : nullptr;
  const TS* cs = a.col_slot >= 0 ? at<const TS>(rec, a.col_slot, a.col_off) : nullptr;
  const int64_t tot = (int64_t)a.m * a.n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    int i, j;
    if (a.X.rs == 1) { i = (int)(e % a.m); j = (int)(e / a.m); }
    else { j = (int)(e % a.n); i = (int)(e / a.n); }
    TS f = TS(1);
    if (rs) f *= rs[i];
    if (cs) f *= cs[j];
    T* px = X + i * a.X.rs + j * a.X.cs;
    *px = T(TS(*px) * f);
  }
}

template <typename T, typename TS>
hipError_t scale2d(const Rec* recs, int nrec, const ScaleArgs& a, hipStream_t s) {
  const int64_t tot = (int64_t)a.m * a.n;
  if (tot <= 0 || nrec <= 0) return hipSuccess;
  int blocks = (int)((tot + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL((scale2d_kernel<T, TS>), dim3(blocks, nrec), dim3(256), 0, s, recs, a);
  return hipGetLastError();
}

// x_i <- sqrt(max(x_i, 0)) for the first `count` entries (singular values from
// the eigenvalues of a Gram matrix)
template <typename T>
__global__ __launch_bounds__(256) void sqrt_prefix_kernel(const Rec* __restrict__ recs, int slot, int64_t off,
                                                          int count) {
  T* x = at<T>(recs[blockIdx.y], slot, off);
  for (int i = blockIdx.x * 256 + threadIdx.x; i < count; i += gridDim.x * 256) {
    const double v = (double)x[i];
    x[i] = T(v > 0.0 ? sqrt(v) : 0.0);
  }
}

template <typename T>
hipError_t sqrt_prefix(const Rec* recs, int nrec, int slot, int64_t off, int count, hipStream_t s) {
  if (count <= 0 || nrec <= 0) return hipSuccess;
  hipLaunchKernelGGL((sqrt_prefix_kernel<T>), dim3((count + 255) / 256, nrec), dim3(256), 0, s, recs, slot, off,
                     count);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Light correction (B-KFAC-C) helpers
// ---------------------------------------------------------------------------
// dst(:, j) = src(:, idx[j]): d x n column gather into the workspace
template <typename T>
__global__ __launch_bounds__(256) void gather_cols_kernel(const Rec* __restrict__ recs, GatherArgs a) {
  const Rec& rec = recs[blockIdx.y];
  const T* src = at<const T>(rec, a.src_slot, 0);
  const int32_t* idx = at<const int32_t>(rec, WS, a.off_idx);
  T* dst = at<T>(rec, WS, a.off_dst);
  const int64_t tot = a.d * a.n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e % a.d, j = e / a.d;
    dst[e] = src[i + (int64_t)idx[j] * a.lds];
  }
}

template <typename T>
hipError_t gather_cols(const Rec* recs, int nrec, const GatherArgs& a, hipStream_t s) {
  const int64_t tot = a.d * a.n;
  if (tot <= 0 || nrec <= 0) return hipSuccess;
  int blocks = (int)((tot + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL((gather_cols_kernel<T>), dim3(blocks, nrec), dim3(256), 0, s, recs, a);
  return hipGetLastError();
}

// New eigenvalues of the k modes (the chosen ones from the small EVD, sorted
// descending in lam), their stable descending order into D_BACK, and for each
// output position its source: a front column (>= 0) or corrected column t
// (-(t + 1)).  One workgroup per problem.
constexpr int MERGE_MAXK = 4096;
template <typename TC, typename TD>
__global__ __launch_bounds__(256) void correct_merge_kernel(const Rec* __restrict__ recs, MergeArgs a) {
  const Rec& rec = recs[blockIdx.x];
  __shared__ double dv[MERGE_MAXK];
  __shared__ int pos[MERGE_MAXK];
  const TD* Din = at<const TD>(rec, D_FRONT, 0);
  TD* Dout = at<TD>(rec, D_BACK, 0);
  const TC* lam = at<const TC>(rec, WS, a.off_lam);
  const int32_t* idx = at<const int32_t>(rec, WS, a.off_idx);
  int32_t* src = at<int32_t>(rec, WS, a.off_src);
  for (int j = threadIdx.x; j < a.k; j += 256) pos[j] = -1;
  __syncthreads();
  for (int t = threadIdx.x; t < a.n_crc; t += 256) pos[idx[t]] = t;
  __syncthreads();
  for (int j = threadIdx.x; j < a.k; j += 256) dv[j] = pos[j] >= 0 ? (double)lam[pos[j]] : (double)Din[j];
  __syncthreads();
  for (int j = threadIdx.x; j < a.k; j += 256) {
    const double v = dv[j];
    int rk = 0;
    for (int i = 0; i < a.k; ++i) rk += (dv[i] > v) || (dv[i] == v && i < j);
    Dout[rk] = TD(v);
    src[rk] = pos[j] >= 0 ? -(pos[j] + 1) : j;
  }
}

template <typename TC, typename TD>
hipError_t correct_merge(const Rec* recs, int nrec, const MergeArgs& a, hipStream_t s) {
  if (a.k > MERGE_MAXK || a.k <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL((correct_merge_kernel<TC, TD>), dim3(nrec), dim3(256), 0, s, recs, a);
  return hipGetLastError();
}

// U_BACK(:, p) = front column src[p], or corrected column -src[p] - 1
template <typename T>
__global__ __launch_bounds__(256) void correct_permute_kernel(const Rec* __restrict__ recs, PermuteArgs a) {
  const Rec& rec = recs[blockIdx.y];
  const T* Uf = at<const T>(rec, U_FRONT, 0);
  const T* Uc = at<const T>(rec, WS, a.off_ucw);
  const int32_t* src = at<const int32_t>(rec, WS, a.off_src);
  T* Ub = at<T>(rec, U_BACK, 0);
  const int64_t tot = a.d * a.k;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e % a.d, p = e / a.d;
    const int sc = src[p];
    Ub[i + p * a.ldu] = sc >= 0 ? Uf[i + (int64_t)sc * a.ldu] : Uc[i + (int64_t)(-sc - 1) * a.d];
  }
}

template <typename T>
hipError_t correct_permute(const Rec* recs, int nrec, const PermuteArgs& a, hipStream_t s) {
  const int64_t tot = a.d * a.k;
  if (tot <= 0 || nrec <= 0) return hipSuccess;
  int blocks = (int)((tot + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL((correct_permute_kernel<T>), dim3(blocks, nrec), dim3(256), 0, s, recs, a);
  return hipGetLastError();
}

// Check of a caller-supplied representation (kfb_state_load): one wave per
// column j < k of U (d x k, leading dimension ld) flags KFB_EV_ORTHO_DRIFT in
// *status when |sum_i u_ij^2 - 1| > tol (columns of eigenvalue 0 excepted).
template <typename T, typename TD>
__global__ __launch_bounds__(256) void loaded_norms_kernel(const T* __restrict__ U, int64_t ld, int64_t d, int k,
                                                            const TD* __restrict__ D, double tol,
                                                            uint32_t* status) {
  const int j = blockIdx.x * 4 + threadIdx.x / 64, l = threadIdx.x % 64;
  if (j >= k || !((double)D[j] > 0.0)) return;
  const T* u = U + (int64_t)j * ld;
  double sum = 0.0;
  for (int64_t i = l; i < d; i += 64) {
    const double v = (double)u[i];
    sum = fma(v, v, sum);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
  if (l == 0 && !(fabs(sum - 1.0) <= tol)) atomicOr(status, (uint32_t)KFB_EV_ORTHO_DRIFT);
}

template <typename T, typename TD>
hipError_t loaded_norms(const T* U, int64_t ld, int64_t d, int k, const TD* D, double tol, uint32_t* status,
                        hipStream_t s) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL((loaded_norms_kernel<T, TD>), dim3((k + 3) / 4), dim3(256), 0, s, U, ld, d, k, D, tol,
                     status);
  return hipGetLastError();
}

// Drift detector: one wave per column, FP64 sum of squares
// (columns of zero eigenvalue, left by a rank-deficient batch, are not checked)
template <typename T, typename TD>
__global__ __launch_bounds__(256) void ortho_check_kernel(const Rec* __restrict__ recs, int slot, int dslot,
                                                          int64_t d, int64_t ld, int ncols, double tol) {
  const Rec& rec = recs[blockIdx.y];
  const int j = blockIdx.x * 4 + threadIdx.x / 64, l = threadIdx.x % 64;
  if (j >= ncols || !((double)at<const TD>(rec, dslot, 0)[j] > 0.0)) return;
  const T* u = at<const T>(rec, slot, 0) + (int64_t)j * ld;
  double sum = 0.0;
  for (int64_t i = l; i < d; i += 64) {
    const double v = (double)u[i];
    sum = fma(v, v, sum);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
  if (l == 0 && !(fabs(sum - 1.0) <= tol)) atomicOr(at<uint32_t>(rec, STATUS, 0), (uint32_t)KFB_EV_ORTHO_DRIFT);
}

template <typename T, typename TD>
hipError_t ortho_check(const Rec* recs, int nrec, int slot, int dslot, int64_t d, int64_t ld, int ncols, double tol,
                       hipStream_t s) {
  if (ncols <= 0 || nrec <= 0) return hipSuccess;
  hipLaunchKernelGGL((ortho_check_kernel<T, TD>), dim3((ncols + 3) / 4, nrec), dim3(256), 0, s, recs, slot, dslot, d,
                     ld, ncols, tol);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
template hipError_t ortho_check<double, double>(const Rec*, int, int, int, int64_t, int64_t, int, double, hipStream_t);
template hipError_t ortho_check<float, float>(const Rec*, int, int, int, int64_t, int64_t, int, double, hipStream_t);
template hipError_t ortho_check<float, double>(const Rec*, int, int, int, int64_t, int64_t, int, double, hipStream_t);
template hipError_t loaded_norms<double, double>(const double*, int64_t, int64_t, int, const double*, double,
                                                 uint32_t*, hipStream_t);
template hipError_t loaded_norms<float, float>(const float*, int64_t, int64_t, int, const float*, double, uint32_t*,
                                               hipStream_t);
template hipError_t loaded_norms<float, double>(const float*, int64_t, int64_t, int, const double*, double,
                                                uint32_t*, hipStream_t);
template hipError_t gather_cols<double>(const Rec*, int, const GatherArgs&, hipStream_t);
template hipError_t gather_cols<float>(const Rec*, int, const GatherArgs&, hipStream_t);
template hipError_t correct_merge<double, double>(const Rec*, int, const MergeArgs&, hipStream_t);
template hipError_t correct_merge<float, float>(const Rec*, int, const MergeArgs&, hipStream_t);
template hipError_t correct_permute<double>(const Rec*, int, const PermuteArgs&, hipStream_t);
template hipError_t correct_permute<float>(const Rec*, int, const PermuteArgs&, hipStream_t);
template hipError_t sqrt_prefix<double>(const Rec*, int, int, int64_t, int, hipStream_t);
template hipError_t sqrt_prefix<float>(const Rec*, int, int, int64_t, int, hipStream_t);
template hipError_t chol_inv<double>(const Rec*, int, const CholArgs&, hipStream_t);
template hipError_t chol_inv<float>(const Rec*, int, const CholArgs&, hipStream_t);
// ---------------------------------------------------------------------------
// Eigenpair refinement of the FP64 core K from approximate eigenvectors X (the
// FP32 eigensolve's), one step of Ogita and Aishima's iterative refinement for
// the symmetric eigenvalue problem.  With S = X^T K X and G = X^T X (R = I - G),
// to first order X' = X (I + E) is orthonormal and diagonalises K when
//   E + E^T = R  and  S + E^T diag(lam) + diag(lam) E = diag(lam),
// giving lam_i = S_ii / G_ii and, for pairs whose estimates are separated by
// more than delta = 2 (||S - diag(lam)|| + ||K|| ||R||) (Frobenius norms, bounds
// of the spectral ones), E_ij = (S_ij + lam_j R_ij) / (lam_j - lam_i); closer
// pairs (and the diagonal) take E_ij = R_ij / 2, which restores orthonormality
// only.  The error of X drops from e to O(e^2) outside such clusters.
// ---------------------------------------------------------------------------
// OA_BLOCKS workgroups per problem, each over a contiguous range of the N^2
// entries: the eigenvalue estimates of its diagonal entries (into the finalize
// step's eigenvalue slots, the eigenvector scales at lam + N set to 1) and its
// partial sums of ||S - diag(lam)||^2, ||K||^2 and ||R||^2 (fixed order within
// the block); oa_correct sums the blocks' partials in block order, so delta is
// the same for every workgroup and every run.

__global__ __launch_bounds__(256) void oa_prepare_kernel(const Rec* __restrict__ recs, OaArgs a) {
  const Rec& rec = recs[blockIdx.y];
  const int N = a.N;
  const double* K = at<const double>(rec, WS, a.off_K);
  const double* S = at<const double>(rec, WS, a.off_S);
  const double* G = at<const double>(rec, WS, a.off_G);
  double* lam = at<double>(rec, WS, a.off_lam);
  double* part = at<double>(rec, WS, a.off_delta) + 1 + 3 * blockIdx.x;
  __shared__ double red[3][256];
  const int t = threadIdx.x;
  const int ic = (N + OA_BLOCKS - 1) / OA_BLOCKS;
  for (int i = blockIdx.x * ic + t; i < min(N, (int)(blockIdx.x + 1) * ic); i += 256) {
    const int64_t dii = i + (int64_t)i * N;
    lam[i] = G[dii] > 0.0 ? S[dii] / G[dii] : 0.0;
    lam[N + i] = 1.0;
  }
  const int64_t nn = (int64_t)N * N, ec = (nn + OA_BLOCKS - 1) / OA_BLOCKS;
  const int64_t e0 = blockIdx.x * ec, e1 = min(nn, e0 + ec);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int64_t e = e0 + t; e < e1; e += 256) {
    const int i = (int)(e % N), j = (int)(e / N);
    const double sij = S[e], kij = K[e], gij = G[e];
    const double off = i == j ? sij - (gij > 0.0 ? sij / gij : 0.0) : sij;
    const double rij = (i == j ? 1.0 : 0.0) - gij;
    s0 += off * off;
    s1 += kij * kij;
    s2 += rij * rij;
  }
  red[0][t] = s0;
  red[1][t] = s1;
  red[2][t] = s2;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h)
      for (int q = 0; q < 3; ++q) red[q][t] += red[q][t + h];
    __syncthreads();
  }
  if (t < 3) part[t] = red[t][0];
}

// E over G, element by element (each thread reads and writes its own entries)
__global__ __launch_bounds__(256) void oa_correct_kernel(const Rec* __restrict__ recs, OaArgs a) {
  const Rec& rec = recs[blockIdx.y];
  const int N = a.N;
  const double* S = at<const double>(rec, WS, a.off_S);
  double* G = at<double>(rec, WS, a.off_G);
  const double* lam = at<const double>(rec, WS, a.off_lam);
  __shared__ double dl_s;
  if (threadIdx.x == 0) {
    const double* part = at<const double>(rec, WS, a.off_delta) + 1;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int b = 0; b < OA_BLOCKS; ++b) {
      s0 += part[3 * b];
      s1 += part[3 * b + 1];
      s2 += part[3 * b + 2];
    }
    dl_s = 2.0 * (sqrt(s0) + sqrt(s1) * sqrt(s2));
  }
  __syncthreads();
  const double dl = dl_s;
  const int64_t nn = (int64_t)N * N;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % N), j = (int)(e / N);
    const double rij = (i == j ? 1.0 : 0.0) - G[e];
    const double gap = lam[j] - lam[i];
    G[e] = fabs(gap) > dl ? (S[e] + lam[j] * rij) / gap : 0.5 * rij;
  }
}

hipError_t oa_prepare(const Rec* recs, int nrec, const OaArgs& a, hipStream_t s) {
  if (a.N > FIN_MAXN) return hipErrorInvalidValue;
  hipLaunchKernelGGL(oa_prepare_kernel, dim3(OA_BLOCKS, nrec), dim3(256), 0, s, recs, a);
  return hipGetLastError();
}

hipError_t oa_correct(const Rec* recs, int nrec, const OaArgs& a, hipStream_t s) {
  const int64_t nn = (int64_t)a.N * a.N;
  int blocks = (int)((nn + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(oa_correct_kernel, dim3(blocks, nrec), dim3(256), 0, s, recs, a);
  return hipGetLastError();
}

// finalize from eigenvalue estimates already in lam[0, N) and eigenvectors in
// the columns of the N x N matrix at off_V (column scales lam[N + j]): ranks,
// D descending, W permuted
template <typename TW, typename TD>
hipError_t finalize_sorted(const Rec* recs, int nrec, const FinArgs& a, hipStream_t s) {
  if (a.N > FIN_MAXN || a.Np != a.N) return hipErrorInvalidValue;
  hipLaunchKernelGGL((fin_sort_kernel<double, TD>), dim3(nrec), dim3(256), 0, s, recs, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t tot = (int64_t)a.N * a.N;
  int blocks = (int)((tot + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL((fin_gather_kernel<double, TW>), dim3(blocks, nrec), dim3(256), 0, s, recs, a);
  return hipGetLastError();
}
template hipError_t finalize_sorted<float, double>(const Rec*, int, const FinArgs&, hipStream_t);
template hipError_t finalize_sorted<double, double>(const Rec*, int, const FinArgs&, hipStream_t);
template hipError_t assemble_core<float, float, double, double>(const Rec*, int, const CoreArgs&, hipStream_t);

template hipError_t assemble_core<double, double, double, double>(const Rec*, int, const CoreArgs&, hipStream_t);
template hipError_t assemble_core<float, float, float, float>(const Rec*, int, const CoreArgs&, hipStream_t);
template hipError_t assemble_core<double, float, double, double>(const Rec*, int, const CoreArgs&, hipStream_t);
template hipError_t jacobi_round<double>(const Rec*, int, const JacArgs&, int, int, hipStream_t);
template hipError_t jacobi_round<float>(const Rec*, int, const JacArgs&, int, int, hipStream_t);
template hipError_t finalize_core<double, double, double>(const Rec*, int, const FinArgs&, hipStream_t);
template hipError_t finalize_core<float, float, float>(const Rec*, int, const FinArgs&, hipStream_t);
template hipError_t finalize_core<double, float, double>(const Rec*, int, const FinArgs&, hipStream_t);
template hipError_t precond_coefs<double, double>(const Rec*, int, const CoefArgs&, hipStream_t);
template hipError_t precond_coefs<float, float>(const Rec*, int, const CoefArgs&, hipStream_t);
template hipError_t precond_coefs<double, float>(const Rec*, int, const CoefArgs&, hipStream_t);
template hipError_t scale2d<double, double>(const Rec*, int, const ScaleArgs&, hipStream_t);
template hipError_t scale2d<float, float>(const Rec*, int, const ScaleArgs&, hipStream_t);

}  // namespace kfb
