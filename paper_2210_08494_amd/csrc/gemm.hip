// Strided GEMM engine for the kfb stages (FP64 / FP32 FMA tiles) and helpers.
//
// Every launch covers `nrec` independent problems of one shape (blockIdx.z is
// the problem); operand pointers are resolved from the per-problem records.
#include "kfb_kernels.h"

namespace kfb {

template <typename To, typename From>
__device__ __forceinline__ To cv(From x) { return static_cast<To>(x); }
template <> __device__ __forceinline__ float cv<float, bf16>(bf16 x) { return __bfloat162float(x); }
template <> __device__ __forceinline__ double cv<double, bf16>(bf16 x) {
  return static_cast<double>(__bfloat162float(x));
}
template <> __device__ __forceinline__ bf16 cv<bf16, float>(float x) { return __float2bfloat16(x); }
template <> __device__ __forceinline__ bf16 cv<bf16, double>(double x) {
  return __float2bfloat16(static_cast<float>(x));
}

// Resolved operand with an optional second segment along its k index.
template <typename T>
struct Seg {
  const T* p;
  int64_t rs, cs;
  const T* p2;
  int64_t rs2, cs2;
  int split;
  __device__ Seg(const Rec& r, const OpRef& o) {
    p = o.slot >= 0 ? at<const T>(r, o.slot, o.off) : nullptr;
    rs = o.rs; cs = o.cs;
    p2 = o.slot2 >= 0 ? at<const T>(r, o.slot2, o.off2) : nullptr;
    rs2 = o.rs2; cs2 = o.cs2;
    split = o.slot2 >= 0 ? o.split : 0x7fffffff;
  }
  // A operand: k is the column index
  __device__ __forceinline__ T a(int i, int k) const {
    return k < split ? p[i * rs + k * cs] : p2[i * rs2 + (k - split) * cs2];
  }
  // B operand: k is the row index
  __device__ __forceinline__ T b(int k, int j) const {
    return k < split ? p[k * rs + j * cs] : p2[(k - split) * rs2 + j * cs2];
  }
};

constexpr int GBM = 64, GBN = 64, GBK = 16, GNT = 256;

template <typename TA, typename TB, typename TC, typename TC0, typename TAcc>
__global__ __launch_bounds__(GNT) void gemm_fma_kernel(const Rec* __restrict__ recs, GemmArgs g) {
  __shared__ TAcc As[GBK][GBM + 1];
  __shared__ TAcc Bs[GBK][GBN + 1];
  const Rec& rec = recs[blockIdx.z];
  const int tiles_m = (g.m + GBM - 1) / GBM;
  const int tm = blockIdx.x % tiles_m, kz = blockIdx.x / tiles_m, tn = blockIdx.y;
  const int kbeg = kz * g.kchunk;
  const int kend = min(g.k, kbeg + g.kchunk);
  const Seg<TA> A(rec, g.A);
  const Seg<TB> B(rec, g.B);
  const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
  const bool a_mc = (g.A.rs == 1);
  const bool b_nc = (g.B.cs == 1);
  // output mapping: consecutive threads walk the contiguous output dimension
  const bool c_nc = (g.ksplit == 1) && (g.C.cs == 1) && (g.C.rs != 1);
  const int r0 = c_nc ? ty : tx, c0 = c_nc ? tx : ty;

  TAcc acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = TAcc(0);

  for (int k0 = kbeg; k0 < kend; k0 += GBK) {
#pragma unroll
    for (int q = 0; q < (GBM * GBK) / GNT; ++q) {
      const int e = t + q * GNT;
      int ii, kk;
      if (a_mc) { ii = e % GBM; kk = e / GBM; } else { kk = e % GBK; ii = e / GBK; }
      const int gi = tm * GBM + ii, gk = k0 + kk;
      TAcc v = TAcc(0);
      if (gi < g.m && gk < kend) v = cv<TAcc>(A.a(gi, gk));
      As[kk][ii] = v;
    }
#pragma unroll
    for (int q = 0; q < (GBN * GBK) / GNT; ++q) {
      const int e = t + q * GNT;
      int jj, kk;
      if (b_nc) { jj = e % GBN; kk = e / GBN; } else { kk = e % GBK; jj = e / GBK; }
      const int gj = tn * GBN + jj, gk = k0 + kk;
      TAcc v = TAcc(0);
      if (gj < g.n && gk < kend) v = cv<TAcc>(B.b(gk, gj));
      Bs[kk][jj] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GBK; ++kk) {
      TAcc av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[kk][r0 + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Bs[kk][c0 + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
    }
    __syncthreads();
  }

  if (g.ksplit > 1) {
    TAcc* part = at<TAcc>(rec, g.Part.slot, g.Part.off) + (int64_t)kz * g.m * g.n;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int gi = tm * GBM + r0 + 16 * i, gj = tn * GBN + c0 + 16 * j;
        if (gi < g.m && gj < g.n) part[gi + (int64_t)gj * g.m] = acc[i][j];
      }
    return;
  }
  TC* C = at<TC>(rec, g.C.slot, g.C.off);
  const bool use_c0 = g.C0.slot >= 0 && (g.beta != 0.0 || g.beta_slot >= 0);
  const TC0* C0 = use_c0 ? at<const TC0>(rec, g.C0.slot, g.C0.off) : nullptr;
  const TAcc alpha = TAcc(g.alpha);
  const TAcc beta = g.beta_slot >= 0 ? TAcc(*at<const double>(rec, g.beta_slot, g.beta_off)) : TAcc(g.beta);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gi = tm * GBM + r0 + 16 * i, gj = tn * GBN + c0 + 16 * j;
      if (gi < g.m && gj < g.n) {
        TAcc v = alpha * acc[i][j];
        if (C0) v += beta * cv<TAcc>(C0[gi * g.C0.rs + gj * g.C0.cs]);
        C[gi * g.C.rs + gj * g.C.cs] = cv<TC>(v);
      }
    }
}

template <typename TC, typename TC0, typename TAcc>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(const Rec* __restrict__ recs, GemmArgs g) {
  const Rec& rec = recs[blockIdx.y];
  const int64_t mn = (int64_t)g.m * g.n;
  const TAcc* part = at<const TAcc>(rec, g.Part.slot, g.Part.off);
  TC* C = at<TC>(rec, g.C.slot, g.C.off);
  const bool use_c0 = g.C0.slot >= 0 && (g.beta != 0.0 || g.beta_slot >= 0);
  const TC0* C0 = use_c0 ? at<const TC0>(rec, g.C0.slot, g.C0.off) : nullptr;
  const TAcc beta = g.beta_slot >= 0 ? TAcc(*at<const double>(rec, g.beta_slot, g.beta_off)) : TAcc(g.beta);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < mn;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % g.m), j = (int)(e / g.m);
    TAcc sum = TAcc(0);
    for (int kz = 0; kz < g.ksplit; ++kz) sum += part[kz * mn + e];
    TAcc v = TAcc(g.alpha) * sum;
    if (C0) v += beta * cv<TAcc>(C0[i * g.C0.rs + j * g.C0.cs]);
    C[i * g.C.rs + j * g.C.cs] = cv<TC>(v);
  }
}

template <typename TA, typename TB, typename TC, typename TC0, typename TAcc>
hipError_t gemm(const Rec* recs, int nrec, const GemmArgs& g0, hipStream_t s) {
  if (g0.m <= 0 || g0.n <= 0 || nrec <= 0) return hipSuccess;
  GemmArgs g = g0;
  if (g.k <= 0) {
    // empty product: C = beta * C0 (only used with beta == 0 -> zeros)
    g.k = 0;
  }
  const int tiles_m = (g.m + GBM - 1) / GBM, tiles_n = (g.n + GBN - 1) / GBN;
  int ks = g.ksplit < 1 ? 1 : g.ksplit;
  if (ks > 1) {
    int chunk = (g.k + ks - 1) / ks;
    chunk = ((chunk + GBK - 1) / GBK) * GBK;
    ks = (g.k + chunk - 1) / chunk;
    g.kchunk = chunk;
  } else {
    g.kchunk = g.k > 0 ? g.k : 1;
  }
  g.ksplit = ks;
  dim3 grid(tiles_m * ks, tiles_n, nrec);
  hipLaunchKernelGGL((gemm_fma_kernel<TA, TB, TC, TC0, TAcc>), grid, dim3(GNT), 0, s, recs, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || ks == 1) return e;
  const int64_t mn = (int64_t)g.m * g.n;
  int blocks = (int)((mn + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL((splitk_reduce_kernel<TC, TC0, TAcc>), dim3(blocks, nrec), dim3(256), 0, s,
                     recs, g);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
constexpr int REC_CHUNK = 16;
struct RecChunk {
  Rec r[REC_CHUNK];
};

__global__ void upload_recs_kernel(RecChunk c, int count, Rec* dst) {
  const int i = threadIdx.x;
  if (i < count) dst[i] = c.r[i];
}

hipError_t upload_recs(const Rec* host, int nrec, Rec* dev, hipStream_t s) {
  for (int b = 0; b < nrec; b += REC_CHUNK) {
    RecChunk c;
    const int cnt = (nrec - b) < REC_CHUNK ? (nrec - b) : REC_CHUNK;
    for (int i = 0; i < cnt; ++i) c.r[i] = host[b + i];
    hipLaunchKernelGGL(upload_recs_kernel, dim3(1), dim3(64), 0, s, c, cnt, dev + b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename TD, typename TS>
__global__ __launch_bounds__(256) void copy2d_kernel(const Rec* __restrict__ recs, OpRef dst, OpRef src,
                                                      int m, int n) {
  const Rec& rec = recs[blockIdx.y];
  TD* D = at<TD>(rec, dst.slot, dst.off);
  const TS* S = at<const TS>(rec, src.slot, src.off);
  const int64_t mn = (int64_t)m * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < mn;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % m), j = (int)(e / m);
    D[i * dst.rs + j * dst.cs] = cv<TD>(S[i * src.rs + j * src.cs]);
  }
}

template <typename TD, typename TS>
hipError_t copy2d(const Rec* recs, int nrec, OpRef dst, OpRef src, int m, int n, hipStream_t s) {
  if (m <= 0 || n <= 0 || nrec <= 0) return hipSuccess;
  const int64_t mn = (int64_t)m * n;
  int blocks = (int)((mn + 255) / 256);
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL((copy2d_kernel<TD, TS>), dim3(blocks, nrec), dim3(256), 0, s, recs, dst, src, m, n);
  return hipGetLastError();
}

template <typename TU, typename TM>
__global__ __launch_bounds__(256) void pad_in_kernel(const Rec* __restrict__ recs, int64_t dp, int r, int n) {
  const Rec& rec = recs[blockIdx.y];
  const int64_t d = rec.z[0], ldu = rec.z[1], ldm = rec.z[2];
  const int nreal = rec.s[2] > 0.0 ? (int)rec.s[2] : n;
  const TU* Us = at<const TU>(rec, X_UF, 0);
  const TM* Ms = at<const TM>(rec, X_M, 0);
  TU* Ud = at<TU>(rec, U_FRONT, 0);
  TM* Md = at<TM>(rec, M_IN, 0);
  const int64_t nu = dp * r, tot = nu + dp * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    if (e < nu) {
      const int64_t i = e % dp, j = e / dp;
      Ud[e] = i < d ? Us[i + j * ldu] : TU(0);
    } else {
      const int64_t f = e - nu, i = f % dp, j = f / dp;
      Md[f] = (i < d && j < nreal) ? Ms[i + j * ldm] : TM(0.0f);
    }
  }
}

template <typename TU, typename TM>
hipError_t pad_in(const Rec* recs, int nrec, int64_t dp, int r, int n, hipStream_t s) {
  const int64_t tot = dp * (r + n);
  if (tot <= 0 || nrec <= 0) return hipSuccess;
  int blocks = (int)((tot + 255) / 256);
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL((pad_in_kernel<TU, TM>), dim3(blocks, nrec), dim3(256), 0, s, recs, dp, r, n);
  return hipGetLastError();
}

template <typename TU>
__global__ __launch_bounds__(256) void crop_out_kernel(const Rec* __restrict__ recs, int64_t dp, int N) {
  const Rec& rec = recs[blockIdx.y];
  const int64_t d = rec.z[0], ldu = rec.z[1];
  const TU* Us = at<const TU>(rec, U_BACK, 0);
  TU* Ud = at<TU>(rec, X_UB, 0);
  const int64_t tot = d * N;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % d, j = e / d;
    Ud[i + j * ldu] = Us[i + j * dp];
  }
}

template <typename TU>
hipError_t crop_out(const Rec* recs, int nrec, int64_t dp, int N, hipStream_t s) {
  const int64_t tot = dp * N;
  if (tot <= 0 || nrec <= 0) return hipSuccess;
  int blocks = (int)((tot + 255) / 256);
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL((crop_out_kernel<TU>), dim3(blocks, nrec), dim3(256), 0, s, recs, dp, N);
  return hipGetLastError();
}

__global__ void zero_words_kernel(const Rec* __restrict__ recs, int slot, int64_t off, int nwords) {
  int32_t* p = at<int32_t>(recs[blockIdx.y], slot, off);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += gridDim.x * blockDim.x) p[i] = 0;
}

hipError_t zero_words(const Rec* recs, int nrec, int slot, int64_t off, int nwords, hipStream_t s) {
  if (nwords <= 0 || nrec <= 0) return hipSuccess;
  int blocks = (nwords + 255) / 256;
  if (blocks > 64) blocks = 64;
  hipLaunchKernelGGL(zero_words_kernel, dim3(blocks, nrec), dim3(256), 0, s, recs, slot, off, nwords);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// explicit instantiations used by the host orchestration
// ---------------------------------------------------------------------------
template hipError_t pad_in<double, double>(const Rec*, int, int64_t, int, int, hipStream_t);
template hipError_t pad_in<float, float>(const Rec*, int, int64_t, int, int, hipStream_t);
template hipError_t pad_in<float, bf16>(const Rec*, int, int64_t, int, int, hipStream_t);
template hipError_t crop_out<double>(const Rec*, int, int64_t, int, hipStream_t);
template hipError_t crop_out<float>(const Rec*, int, int64_t, int, hipStream_t);

#define KFB_GEMM(TA, TB, TC, TC0, TACC) \
  template hipError_t gemm<TA, TB, TC, TC0, TACC>(const Rec*, int, const GemmArgs&, hipStream_t);
KFB_GEMM(double, double, double, double, double)
KFB_GEMM(float, float, float, float, float)
KFB_GEMM(float, bf16, float, float, float)
KFB_GEMM(float, float, float, bf16, float)
KFB_GEMM(float, float, double, double, double)
KFB_GEMM(float, double, float, float, float)
KFB_GEMM(float, float, float, float, double)
#undef KFB_GEMM

template hipError_t copy2d<double, double>(const Rec*, int, OpRef, OpRef, int, int, hipStream_t);
template hipError_t copy2d<float, float>(const Rec*, int, OpRef, OpRef, int, int, hipStream_t);
template hipError_t copy2d<float, bf16>(const Rec*, int, OpRef, OpRef, int, int, hipStream_t);
template hipError_t copy2d<float, double>(const Rec*, int, OpRef, OpRef, int, int, hipStream_t);
template hipError_t copy2d<double, float>(const Rec*, int, OpRef, OpRef, int, int, hipStream_t);

}  // namespace kfb
