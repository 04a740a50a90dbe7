// BF16 MFMA GEMM for the mixed precision form:  C = alpha A B + beta C0.
//
// Operands are FP32 or BF16 in memory, rounded to BF16 (round to nearest
// even) while staged into LDS; with SPLIT the FP32 remainder x - bf16(x) is
// staged as a second BF16 term and three products hi*hi + hi*lo + lo*hi are
// accumulated (about 16 significant bits per operand, FP32 accumulation).
// Tiles of 128 x 128 x 32 are computed by four waves (64 x 64 each) with
// v_mfma_f32_16x16x32_bf16.  Lane layout of that instruction: A element
// (i, k) sits in lane i + 16*(k/8), slot k%8; B element (k, j) in lane
// j + 16*(k/8), slot k%8; result (i, j) in lane j + 16*(i/4), slot i%4.
// When C is column-major the product is issued transposed (B^T A^T), so the
// 16 lanes that share a result slot hold 16 consecutive rows and the stores
// coalesce.  LDS is double buffered: the next k tile is loaded into registers
// while the current one is multiplied.  Split-K partials and the fixed-order
// reduction follow the same GemmArgs contract as the FMA engine.
#include <mutex>
#include <vector>

#include "kfb_kernels.h"

namespace kfb {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

template <typename T> __device__ __forceinline__ float to_f(T x);
template <> __device__ __forceinline__ float to_f<float>(float x) { return x; }
template <> __device__ __forceinline__ float to_f<bf16>(bf16 x) { return __bfloat162float(x); }

constexpr int MBM = 128, MBN = 128, MBK = 32, MNT = 256;
constexpr int MLD = MBK + 8;  // padded LDS row (bf16 elements)

template <typename T>
struct MSeg {
  const T* p;
  int64_t rs, cs;
  const T* p2;
  int64_t rs2, cs2;
  int split;
  __device__ MSeg(const Rec& r, const OpRef& o) {
    p = o.slot >= 0 ? at<const T>(r, o.slot, o.off) : nullptr;
    rs = o.rs; cs = o.cs;
    p2 = o.slot2 >= 0 ? at<const T>(r, o.slot2, o.off2) : nullptr;
    rs2 = o.rs2; cs2 = o.cs2;
    split = o.slot2 >= 0 ? o.split : 0x7fffffff;
  }
  // element (row, k) of an A operand / (k, col) of a B operand, k along the split
  __device__ __forceinline__ float a(int i, int k) const {
    return k < split ? to_f(p[i * rs + k * cs]) : to_f(p2[i * rs2 + (k - split) * cs2]);
  }
  __device__ __forceinline__ float b(int k, int j) const {
    return k < split ? to_f(p[k * rs + j * cs]) : to_f(p2[(k - split) * rs2 + j * cs2]);
  }
};

// One thread moves one 4 x 4 sub-block (rows x k) of a 128 x 32 operand tile.
// kc: k is the contiguous memory direction (4 k per row, 8 threads cover a
// 32-wide row segment); otherwise rows are contiguous (4 consecutive rows per
// k, transposed in registers).  In-range sub-blocks with aligned strides use
// 16-byte (FP32) or 8-byte (BF16) loads; the rest use element loads with
// zero fill.
struct Frag {
  float v[4][4];  // [row][k]
};

__device__ __forceinline__ void frag_pos(bool kc, int t, int* rb, int* kb) {
  if (kc) { *kb = t % 8; *rb = t / 8; } else { *rb = t % 32; *kb = t / 32; }
}

template <typename T, bool ISA>
__device__ __forceinline__ void load_frag(const MSeg<T>& s, bool kc, bool vec_ok, int row0, int nrows, int k0,
                                          int kend, int t, Frag& f) {
  int rb, kb;
  frag_pos(kc, t, &rb, &kb);
  const int gr = row0 + 4 * rb, gk = k0 + 4 * kb;
  const bool one_seg = (gk + 3 < s.split) || (gk >= s.split);
  if (vec_ok && one_seg && gr + 3 < nrows && gk + 3 < kend) {
    const bool seg2 = gk >= s.split;
    const T* base = seg2 ? s.p2 : s.p;
    const int64_t rsd = ISA ? (seg2 ? s.rs2 : s.rs) : (seg2 ? s.cs2 : s.cs);  // stride along rows
    const int64_t ksd = ISA ? (seg2 ? s.cs2 : s.cs) : (seg2 ? s.rs2 : s.rs);  // stride along k
    const int kk = seg2 ? gk - s.split : gk;
    if constexpr (sizeof(T) == 4) {
      typedef __attribute__((__vector_size__(16))) float v4;
      if (kc) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const v4 x = *reinterpret_cast<const v4*>(base + (int64_t)(gr + r) * rsd + (int64_t)kk * ksd);
#pragma unroll
          for (int c = 0; c < 4; ++c) f.v[r][c] = x[c];
        }
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const v4 x = *reinterpret_cast<const v4*>(base + (int64_t)gr * rsd + (int64_t)(kk + c) * ksd);
#pragma unroll
          for (int r = 0; r < 4; ++r) f.v[r][c] = x[r];
        }
      }
    } else {
      typedef __attribute__((__vector_size__(8))) unsigned short v4h;
      if (kc) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const v4h x = *reinterpret_cast<const v4h*>(base + (int64_t)(gr + r) * rsd + (int64_t)kk * ksd);
#pragma unroll
          for (int c = 0; c < 4; ++c) f.v[r][c] = __uint_as_float(((uint32_t)x[c]) << 16);
        }
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const v4h x = *reinterpret_cast<const v4h*>(base + (int64_t)gr * rsd + (int64_t)(kk + c) * ksd);
#pragma unroll
          for (int r = 0; r < 4; ++r) f.v[r][c] = __uint_as_float(((uint32_t)x[r]) << 16);
        }
      }
    }
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int rr = gr + r, k = gk + c;
        float v = 0.f;
        if (rr < nrows && k < kend) v = ISA ? s.a(rr, k) : s.b(k, rr);
        f.v[r][c] = v;
      }
  }
}

template <bool LO>
__device__ __forceinline__ void store_frag(const Frag& f, bool kc, int t, __bf16* hi, __bf16* lo) {
  int rb, kb;
  frag_pos(kc, t, &rb, &kb);
  typedef __attribute__((__vector_size__(8))) __bf16 v4b;
  typedef __attribute__((__vector_size__(16))) float v4f;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    // hardware conversion (round to nearest even), two values per instruction
    const v4f x = {f.v[r][0], f.v[r][1], f.v[r][2], f.v[r][3]};
    const v4b h = __builtin_convertvector(x, v4b);
    *reinterpret_cast<v4b*>(&hi[(4 * rb + r) * MLD + 4 * kb]) = h;
    if (LO) {
      const v4f hb = __builtin_convertvector(h, v4f);
      *reinterpret_cast<v4b*>(&lo[(4 * rb + r) * MLD + 4 * kb]) = __builtin_convertvector(x - hb, v4b);
    }
  }
}

// 4-element vectors along the contiguous direction need aligned bases, a
// 4-multiple stride in the other direction and a 4-multiple split point
template <typename T>
__device__ __forceinline__ bool vec_aligned(const MSeg<T>& s, bool kc, bool isa) {
  const uintptr_t al = sizeof(T) * 4 - 1;
  auto ok = [&](const T* p, int64_t rs, int64_t cs) {
    if (!p) return true;
    const int64_t along = kc ? (isa ? cs : rs) : (isa ? rs : cs);   // must be 1
    const int64_t other = kc ? (isa ? rs : cs) : (isa ? cs : rs);
    return along == 1 && (((uintptr_t)p) & al) == 0 && (other % 4) == 0;
  };
  return ok(s.p, s.rs, s.cs) && ok(s.p2, s.rs2, s.cs2) && (s.p2 == nullptr || (s.split % 4) == 0);
}

template <typename TA, typename TB, typename TC, typename TC0, int SPLIT>
__global__ __launch_bounds__(MNT) void gemm_bf16_kernel(const Rec* __restrict__ recs, GemmArgs g) {
  constexpr bool A_LO = SPLIT && sizeof(TA) == 4;  // BF16 inputs are exact: no remainder
  constexpr bool B_LO = SPLIT && sizeof(TB) == 4;
  __shared__ __attribute__((aligned(16))) __bf16 sAh[2][MBM * MLD];
  __shared__ __attribute__((aligned(16))) __bf16 sBh[2][MBN * MLD];
  __shared__ __attribute__((aligned(16))) __bf16 sAl[A_LO ? 2 : 1][A_LO ? MBM * MLD : 8];
  __shared__ __attribute__((aligned(16))) __bf16 sBl[B_LO ? 2 : 1][B_LO ? MBN * MLD : 8];
  const Rec& rec = recs[blockIdx.z];
  const int tiles_m = (g.m + MBM - 1) / MBM;
  const int tm = blockIdx.x % tiles_m, kz = blockIdx.x / tiles_m, tn = blockIdx.y;
  const int kbeg = kz * g.kchunk;
  const int kend = min(g.k, kbeg + g.kchunk);
  const MSeg<TA> A(rec, g.A);
  const MSeg<TB> B(rec, g.B);
  const bool a_kc = (g.A.cs == 1);
  const bool b_kc = (g.B.rs == 1);
  const bool a_vec = vec_aligned(A, a_kc, true);
  const bool b_vec = vec_aligned(B, b_kc, false);
  const int t = threadIdx.x, w = t / 64, l = t % 64;
  const int wm = (w & 1) * 64, wn = (w >> 1) * 64;  // wave's 64 x 64 sub-tile
  // transposed issue when the output (or the split-K partial) is column-major
  const bool swp = (g.ksplit > 1) || (g.C.rs == 1);

  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  Frag fa, fb;
  int cur = 0;
  if (kbeg < kend) {
    load_frag<TA, true>(A, a_kc, a_vec, tm * MBM, g.m, kbeg, kend, t, fa);
    load_frag<TB, false>(B, b_kc, b_vec, tn * MBN, g.n, kbeg, kend, t, fb);
    store_frag<A_LO>(fa, a_kc, t, sAh[0], sAl[0]);
    store_frag<B_LO>(fb, b_kc, t, sBh[0], sBl[0]);
  }
  __syncthreads();
  for (int k0 = kbeg; k0 < kend; k0 += MBK) {
    const bool more = k0 + MBK < kend;
    if (more) {  // prefetch the next k tile into registers
      load_frag<TA, true>(A, a_kc, a_vec, tm * MBM, g.m, k0 + MBK, kend, t, fa);
      load_frag<TB, false>(B, b_kc, b_vec, tn * MBN, g.n, k0 + MBK, kend, t, fb);
    }
    const int kq = 8 * (l / 16);
    bf16x8 af[4], bfr[4], afl[4], bfl[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      af[i] = *reinterpret_cast<const bf16x8*>(&sAh[cur][(wm + i * 16 + (l % 16)) * MLD + kq]);
      if (A_LO) afl[i] = *reinterpret_cast<const bf16x8*>(&sAl[A_LO ? cur : 0][(wm + i * 16 + (l % 16)) * MLD + kq]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      bfr[j] = *reinterpret_cast<const bf16x8*>(&sBh[cur][(wn + j * 16 + (l % 16)) * MLD + kq]);
      if (B_LO) bfl[j] = *reinterpret_cast<const bf16x8*>(&sBl[B_LO ? cur : 0][(wn + j * 16 + (l % 16)) * MLD + kq]);
    }
    if (!swp) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
          if (B_LO) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfl[j], acc[i][j], 0, 0, 0);
          if (A_LO) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afl[i], bfr[j], acc[i][j], 0, 0, 0);
        }
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[j], af[i], acc[i][j], 0, 0, 0);
          if (B_LO) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfl[j], af[i], acc[i][j], 0, 0, 0);
          if (A_LO) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[j], afl[i], acc[i][j], 0, 0, 0);
        }
    }
    if (more) {
      const int nx = cur ^ 1;
      store_frag<A_LO>(fa, a_kc, t, sAh[nx], sAl[A_LO ? nx : 0]);
      store_frag<B_LO>(fb, b_kc, t, sBh[nx], sBl[B_LO ? nx : 0]);
    }
    __syncthreads();
    cur ^= 1;
  }

  // result element positions: slot v of lane l in tile (i, j)
  //   normal:     row = 16i + 4(l/16) + v, col = 16j + l%16
  //   transposed: row = 16i + l%16,         col = 16j + 4(l/16) + v
  const int gm0 = tm * MBM + wm, gn0 = tn * MBN + wn;
  if (g.ksplit > 1) {
    float* part = at<float>(rec, g.Part.slot, g.Part.off) + (int64_t)kz * g.m * g.n;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int gi = gm0 + 16 * i + (l % 16), gj = gn0 + 16 * j + 4 * (l / 16) + v;
          if (gi < g.m && gj < g.n) part[gi + (int64_t)gj * g.m] = acc[i][j][v];
        }
    return;
  }
  TC* C = at<TC>(rec, g.C.slot, g.C.off);
  const bool use_c0 = g.C0.slot >= 0 && (g.beta != 0.0 || g.beta_slot >= 0);
  const TC0* C0 = use_c0 ? at<const TC0>(rec, g.C0.slot, g.C0.off) : nullptr;
  const float alpha = (float)g.alpha;
  const float beta = g.beta_slot >= 0 ? (float)*at<const double>(rec, g.beta_slot, g.beta_off) : (float)g.beta;
  // optional scalings C = alpha diag(r) (A B) + beta C0 diag(c) (single-term products)
  const float* rsc = nullptr;
  const float* ccs = nullptr;
  if constexpr (SPLIT == 0) {
    rsc = g.rsc_slot >= 0 ? at<const float>(rec, g.rsc_slot, g.rsc_off) : nullptr;
    ccs = g.c0cs_slot >= 0 ? at<const float>(rec, g.c0cs_slot, g.c0cs_off) : nullptr;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int gi, gj;
        if (swp) { gi = gm0 + 16 * i + (l % 16); gj = gn0 + 16 * j + 4 * (l / 16) + v; }
        else { gi = gm0 + 16 * i + 4 * (l / 16) + v; gj = gn0 + 16 * j + (l % 16); }
        if (gi < g.m && gj < g.n) {
          float val = alpha * acc[i][j][v];
          if (rsc) val *= rsc[gi];
          if (C0) {
            float c0 = to_f(C0[gi * g.C0.rs + gj * g.C0.cs]);
            if (ccs) c0 *= ccs[gj];
            val += beta * c0;
          }
          C[gi * g.C.rs + gj * g.C.cs] = TC(val);
        }
      }
}

// ---------------------------------------------------------------------------
// Streamlined variant for FP32 operands (single term, or the hi/lo split):
// every operand 16-byte aligned with a unit stride along rows (MN) or along k
// (KC), k, segment splits and split-K chunks multiples of 32, m and n
// multiples of 4; split-K partials go to the same fixed-order reduction.  The orientation of each operand is a template parameter and every
// per-thread address is formed once, so a k tile costs four vector loads,
// eight packed conversions and four LDS stores per operand.  LDS rows of
// MN-staged operands permute their four 16-byte k chunks by bits 4-5 of the
// row index, which spreads the transposed stores of a wave (rows 4 apart)
// over the banks while 16 consecutive rows still read conflict-free.
// ---------------------------------------------------------------------------
template <bool KC>
__device__ __forceinline__ int fast_lds_off(int row, int kb16) {  // kb16: bf16 offset in the row, multiple of 4
  return KC ? row * MLD + kb16 : row * MLD + 8 * ((kb16 >> 3) ^ ((row >> 4) & 3)) + (kb16 & 7);
}

typedef const float __attribute__((address_space(1)))* gfptr;  // global-memory float pointer

template <bool KC, int TR = 128>
struct FastSrc {
  gfptr p0;
  gfptr p1;             // this thread's base per segment (row offset applied, k offset not)
  int64_t k0s, k1s;     // stride along k per segment
  int64_t r0s, r1s;     // stride along rows per segment (KC: between the thread's four rows)
  int split;
  int nr;               // KC: rows of the thread's four in range; MN: 4 or 0
  __device__ void init(const Rec& rec, const OpRef& o, bool isa, int row0, int nrows, int t) {
    const int rb = KC ? t / 8 : t % (TR / 4), kb = KC ? t % 8 : t / (TR / 4);
    const int left = nrows - (row0 + 4 * rb);
    nr = KC ? (left < 0 ? 0 : left > 4 ? 4 : left) : (left > 0 ? 4 : 0);
    // rows outside the matrix read row 0 instead (always valid); they only feed
    // output rows / columns outside C, which the epilogue never stores
    const int gr = nr ? row0 + 4 * rb : 0;
    split = o.slot2 >= 0 ? o.split : 0x7fffffff;
    // A(i, k) = base[i*rs + k*cs];  B(k, j) = base[k*rs + j*cs]
    {
      const float* base = at<const float>(rec, o.slot, o.off);
      r0s = isa ? o.rs : o.cs;
      k0s = isa ? o.cs : o.rs;
      p0 = (gfptr)(base + (int64_t)gr * r0s + (int64_t)(4 * kb) * k0s);
    }
    if (o.slot2 >= 0) {
      const float* base = at<const float>(rec, o.slot2, o.off2);
      r1s = isa ? o.rs2 : o.cs2;
      k1s = isa ? o.cs2 : o.rs2;
      p1 = (gfptr)(base + (int64_t)gr * r1s + (int64_t)(4 * kb) * k1s);
    } else {
      p1 = p0; r1s = r0s; k1s = k0s;
    }
  }
  // the 4 x 4 sub-block (rows x k) of k tile k0 as four raw vectors (KC: x[r] =
  // row r, MN: x[c] = k column c); no branches around the loads (values of rows
  // outside the matrix are arbitrary: they never reach C)
  __device__ __forceinline__ void load(int k0, f32x4* x) const {
    const bool sg = k0 >= split;
    const int64_t kk = sg ? k0 - split : k0;
    const int64_t ks = sg ? k1s : k0s, rs = sg ? r1s : r0s;
    const gfptr b = (sg ? p1 : p0) + kk * ks;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t o = KC ? (q < nr ? q : 0) * rs : q * ks;
      x[q] = *reinterpret_cast<const __attribute__((address_space(1))) f32x4*>(b + o);
    }
  }
};

template <bool KC, bool LO = false, int TR = 128>
__device__ __forceinline__ void fast_store(const f32x4* x, int t, __bf16* dst, __bf16* dlo = nullptr) {
  const int rb = KC ? t / 8 : t % (TR / 4), kb = KC ? t % 8 : t / (TR / 4);
  typedef __attribute__((__vector_size__(8))) __bf16 v4b;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const f32x4 v = KC ? x[r] : f32x4{x[0][r], x[1][r], x[2][r], x[3][r]};  // row r, k = 4kb .. 4kb+3
    const int o = fast_lds_off<KC>(4 * rb + r, 4 * kb);
    const v4b h = __builtin_convertvector(v, v4b);
    *reinterpret_cast<v4b*>(&dst[o]) = h;
    if constexpr (LO) {  // remainder term: x - hi, exact in FP32, rounded to BF16
      const f32x4 rem = v - __builtin_convertvector(h, f32x4);
      *reinterpret_cast<v4b*>(&dlo[o]) = __builtin_convertvector(rem, v4b);
    }
  }
}

// XCD-aware tile order.  Workgroups go to the eight XCDs round-robin in
// dispatch order and each XCD has its own L2, so the linear workgroup index is
// remapped: XCD x takes a contiguous range of tiles, and within it the tiles
// run in groups of GM tile rows (column by column inside a group), so the
// workgroups resident on one XCD at a time share both their A row panels and
// their B column panels through that XCD's L2.
constexpr int XCDS = 8, TILE_GM = 8;
__device__ __forceinline__ void xcd_tile(int nx, int ny, int nz, int* tm, int* tn, int* tz) {
  const int total = nx * ny * nz;
  const int lin = blockIdx.x + nx * (blockIdx.y + ny * blockIdx.z);
  const int q = total / XCDS, rmd = total % XCDS, x = lin % XCDS;
  const int t = x * q + min(x, rmd) + lin / XCDS;
  const int per = nx * ny;
  *tz = t / per;
  const int u = t - *tz * per;
  const int in_group = TILE_GM * ny;
  const int first = (u / in_group) * TILE_GM;
  const int gsz = min(nx - first, TILE_GM);
  const int v = u % in_group;
  *tm = first + v % gsz;
  *tn = v / gsz;
}

// TT: square output tile (128: four waves of 64 x 64; 256: eight waves of
// 128 x 64, single-term products only, twice the flops per staged byte).
// ESC: the epilogue applies the optional scalings C = alpha diag(r) (A B) +
// beta C0 diag(c) (single term, no split-K); a template switch, so the other
// products keep their register budget.
template <typename TC, typename TC0, bool AKC, bool BKC, bool SWP, bool SPL = false, int TT = 128, bool ESC = false>
__global__ __launch_bounds__(2 * TT) void gemm_bf16_fast_kernel(const Rec* __restrict__ recs, GemmArgs g) {
  static_assert(TT == 128 || (TT == 256 && !SPL), "tile");
  static_assert(!(ESC && SPL), "scaled epilogue");
  constexpr int FM = TT / 32, FN = 4;  // 16 x 16 fragments per wave along rows / columns
  __shared__ __attribute__((aligned(16))) __bf16 sA[2][TT * MLD];
  __shared__ __attribute__((aligned(16))) __bf16 sB[2][TT * MLD];
  // SPL: BF16 remainders of both operands (hi*hi + hi*lo + lo*hi, ~16 bits)
  __shared__ __attribute__((aligned(16))) __bf16 sAl[SPL ? 2 : 1][SPL ? 128 * MLD : 8];
  __shared__ __attribute__((aligned(16))) __bf16 sBl[SPL ? 2 : 1][SPL ? 128 * MLD : 8];
  int tm, tn, tz;
  xcd_tile(gridDim.x, gridDim.y, gridDim.z, &tm, &tn, &tz);
  const Rec& rec = recs[tz];
  // split-K: blockIdx.x also enumerates the k chunks (tm = kz * tiles_m + tile row)
  const int tiles_m = (g.m + TT - 1) / TT, kz = tm / tiles_m;
  tm -= kz * tiles_m;
  const int kbeg = g.ksplit > 1 ? kz * g.kchunk : 0;
  const int kend = g.ksplit > 1 ? min(g.k, kbeg + g.kchunk) : g.k;
  const int t = threadIdx.x, w = t / 64, l = t % 64;
  const int wm = (w & 1) * (TT / 2), wn = (w >> 1) * 64;
  constexpr bool swp = SWP;  // output column-major: issue (B^T A^T) so stores coalesce
  FastSrc<AKC, TT> A;
  FastSrc<BKC, TT> B;
  A.init(rec, g.A, true, tm * TT, g.m, t);
  B.init(rec, g.B, false, tn * TT, g.n, t);
  // fragment read offsets (bf16 elements) into a stage
  const int kq = 8 * (l / 16);
  int offA[FM], offB[FN];
#pragma unroll
  for (int i = 0; i < FM; ++i) offA[i] = fast_lds_off<AKC>(wm + i * 16 + (l % 16), kq);
#pragma unroll
  for (int j = 0; j < FN; ++j) offB[j] = fast_lds_off<BKC>(wn + j * 16 + (l % 16), kq);
  f32x4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  f32x4 fa[4], fb[4];
  A.load(kbeg, fa);
  B.load(kbeg, fb);
  fast_store<AKC, SPL, TT>(fa, t, sA[0], sAl[0]);
  fast_store<BKC, SPL, TT>(fb, t, sB[0], sBl[0]);
  __syncthreads();
  int cur = 0;
  for (int k0 = kbeg; k0 < kend; k0 += MBK) {
    const bool more = k0 + MBK < kend;
    if (more) {
      A.load(k0 + MBK, fa);
      B.load(k0 + MBK, fb);
    }
    bf16x8 af[FM], bfr[FN], afl[SPL ? FM : 1], bfl[SPL ? FN : 1];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      af[i] = *reinterpret_cast<const bf16x8*>(&sA[cur][offA[i]]);
      if constexpr (SPL) afl[i] = *reinterpret_cast<const bf16x8*>(&sAl[cur][offA[i]]);
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      bfr[j] = *reinterpret_cast<const bf16x8*>(&sB[cur][offB[j]]);
      if constexpr (SPL) bfl[j] = *reinterpret_cast<const bf16x8*>(&sBl[cur][offB[j]]);
    }
    if constexpr (!swp) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
          if constexpr (SPL) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfl[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afl[i], bfr[j], acc[i][j], 0, 0, 0);
          }
        }
    } else {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[j], af[i], acc[i][j], 0, 0, 0);
          if constexpr (SPL) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfl[j], af[i], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[j], afl[i], acc[i][j], 0, 0, 0);
          }
        }
    }
    if (more) {
      fast_store<AKC, SPL, TT>(fa, t, sA[cur ^ 1], sAl[SPL ? cur ^ 1 : 0]);
      fast_store<BKC, SPL, TT>(fb, t, sB[cur ^ 1], sBl[SPL ? cur ^ 1 : 0]);
    }
    __syncthreads();
    cur ^= 1;
  }
  const int gm0 = tm * TT + wm, gn0 = tn * TT + wn;
  if (g.ksplit > 1) {  // raw partial of chunk kz, column-major (the launch issues SWP)
    float* part = at<float>(rec, g.Part.slot, g.Part.off) + (int64_t)kz * g.m * g.n;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int gi = gm0 + 16 * i + (l % 16), gj = gn0 + 16 * j + 4 * (l / 16) + v;
          if (gi < g.m && gj < g.n) part[gi + (int64_t)gj * g.m] = acc[i][j][v];
        }
    return;
  }
  TC* C = at<TC>(rec, g.C.slot, g.C.off);
  const bool use_c0 = g.C0.slot >= 0 && (g.beta != 0.0 || g.beta_slot >= 0);
  const TC0* C0 = use_c0 ? at<const TC0>(rec, g.C0.slot, g.C0.off) : nullptr;
  const float alpha = (float)g.alpha;
  const float beta = g.beta_slot >= 0 ? (float)*at<const double>(rec, g.beta_slot, g.beta_off) : (float)g.beta;
  const float* rsc = nullptr;
  const float* ccs = nullptr;
  if constexpr (ESC) {
    rsc = g.rsc_slot >= 0 ? at<const float>(rec, g.rsc_slot, g.rsc_off) : nullptr;
    ccs = g.c0cs_slot >= 0 ? at<const float>(rec, g.c0cs_slot, g.c0cs_off) : nullptr;
  }
  if constexpr (sizeof(TC) == 4 && sizeof(TC0) == 4) {
    // vector epilogue: each lane's four results are four consecutive columns of
    // a row-major C (transposed issue) or four consecutive rows of a
    // column-major C (plain issue); m and n are multiples of 4
    if (g.c_vec) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          int gi, gj;
          int64_t oc, oc0;
          if (SWP) {
            gi = gm0 + 16 * i + (l % 16); gj = gn0 + 16 * j + 4 * (l / 16);
            oc = (int64_t)gi * g.C.rs + gj; oc0 = (int64_t)gi * g.C0.rs + gj;
          } else {
            gi = gm0 + 16 * i + 4 * (l / 16); gj = gn0 + 16 * j + (l % 16);
            oc = gi + (int64_t)gj * g.C.cs; oc0 = gi + (int64_t)gj * g.C0.cs;
          }
          if (gi < g.m && gj < g.n) {
            f32x4 val = alpha * acc[i][j];
            if constexpr (ESC) {  // the lane's four results: one row (SWP) or four rows
              if (rsc) val *= SWP ? f32x4{rsc[gi], rsc[gi], rsc[gi], rsc[gi]}
                                  : *reinterpret_cast<const f32x4*>(&rsc[gi]);
            }
            if (C0) {
              f32x4 c0 = *reinterpret_cast<const f32x4*>(&C0[oc0]);
              if constexpr (ESC) {  // four columns (SWP) or one column
                if (ccs) c0 *= SWP ? *reinterpret_cast<const f32x4*>(&ccs[gj])
                                   : f32x4{ccs[gj], ccs[gj], ccs[gj], ccs[gj]};
              }
              val += beta * c0;
            }
            *reinterpret_cast<f32x4*>(&C[oc]) = val;
          }
        }
      return;
    }
  }
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int gi, gj;
        if (swp) { gi = gm0 + 16 * i + (l % 16); gj = gn0 + 16 * j + 4 * (l / 16) + v; }
        else { gi = gm0 + 16 * i + 4 * (l / 16) + v; gj = gn0 + 16 * j + (l % 16); }
        if (gi < g.m && gj < g.n) {
          float val = alpha * acc[i][j][v];
          if constexpr (ESC) {
            if (rsc) val *= rsc[gi];
          }
          if (C0) {
            float c0 = to_f(C0[gi * g.C0.rs + gj * g.C0.cs]);
            if constexpr (ESC) {
              if (ccs) c0 *= ccs[gj];
            }
            val += beta * c0;
          }
          C[gi * g.C.rs + gj * g.C.cs] = TC(val);
        }
      }
}

// orientation of an operand for the streamlined kernel: 1 = unit stride along
// k, 0 = unit stride along rows, -1 = not eligible
static int fast_orient(const OpRef& o, bool isa) {
  auto one = [&](int64_t rs, int64_t cs) -> int {
    const int64_t r_st = isa ? rs : cs, k_st = isa ? cs : rs;
    if (k_st == 1 && r_st % 4 == 0) return 1;
    if (r_st == 1 && k_st % 4 == 0) return 0;
    return -1;
  };
  const int a = one(o.rs, o.cs);
  if (o.slot2 < 0) return a;
  if (o.split % MBK) return -1;
  return one(o.rs2, o.cs2) == a ? a : -1;
}

template <typename TC, typename TC0>
__global__ __launch_bounds__(256) void mfma_splitk_reduce(const Rec* __restrict__ recs, GemmArgs g);

// Output tile of the streamlined kernel per product shape (m, n, k): the
// tuning table's entry (filled by the autotuner through kfb_tune_set_gemm),
// else 128.  Products with the hi/lo split always take 128 (their four LDS
// stages would not fit a 256 tile).
struct GemmTileEntry {
  int m, n, k, tile;
};
static std::mutex g_gemm_tile_mu;
static std::vector<GemmTileEntry> g_gemm_tiles;

int gemm_tile_lookup(int m, int n, int k) {
  std::lock_guard<std::mutex> lk(g_gemm_tile_mu);
  for (const auto& e : g_gemm_tiles)
    if (e.m == m && e.n == n && e.k == k) return e.tile;
  return 0;
}

int gemm_tile_set(int m, int n, int k, int tile) {
  if (m <= 0 || n <= 0 || k <= 0 || (tile != 0 && tile != 128 && tile != 256)) return -1;
  std::lock_guard<std::mutex> lk(g_gemm_tile_mu);
  for (size_t i = 0; i < g_gemm_tiles.size(); ++i)
    if (g_gemm_tiles[i].m == m && g_gemm_tiles[i].n == n && g_gemm_tiles[i].k == k) {
      if (tile == 0) g_gemm_tiles.erase(g_gemm_tiles.begin() + i);
      else g_gemm_tiles[i].tile = tile;
      return 0;
    }
  if (tile != 0) g_gemm_tiles.push_back(GemmTileEntry{m, n, k, tile});
  return 0;
}

template <typename TC, typename TC0, bool SPL = false>
static bool gemm_bf16_fast(const Rec* recs, int nrec, const GemmArgs& g0, hipStream_t s, hipError_t* err) {
  if (!g0.aligned16 || g0.k <= 0 || g0.k % MBK || g0.m % 4 || g0.n % 4) return false;
  const int ao = fast_orient(g0.A, true), bo = fast_orient(g0.B, false);
  if (ao < 0 || bo < 0) return false;
  const int tt = (!SPL && gemm_tile_lookup(g0.m, g0.n, g0.k) == 256) ? 256 : 128;
  GemmArgs g = g0;
  int ks = g.ksplit < 1 ? 1 : g.ksplit;
  if (ks > 1) {  // chunks of whole k tiles, the fixed-order reduction afterwards
    int chunk = (g.k + ks - 1) / ks;
    chunk = ((chunk + MBK - 1) / MBK) * MBK;
    ks = (g.k + chunk - 1) / chunk;
    g.kchunk = chunk;
  }
  g.ksplit = ks;
  const bool esc = g.rsc_slot >= 0 || g.c0cs_slot >= 0;
  if (esc && (SPL || ks > 1)) {  // the scaled epilogue takes whole single-term sums
    *err = hipErrorInvalidValue;
    return true;
  }
  dim3 grid(((g.m + tt - 1) / tt) * ks, (g.n + tt - 1) / tt, nrec);
  // vector epilogue (C and C0 as 16-byte vectors): a row-major C takes the
  // transposed issue (four consecutive columns per lane), a column-major C the
  // plain one (four consecutive rows per lane)
  const bool c0_used = g.C0.slot >= 0 && (g.beta != 0.0 || g.beta_slot >= 0);
  const bool vok = ks == 1 && g.c_vec && sizeof(TC) == 4 && sizeof(TC0) == 4;
  const bool vrow = vok && g.C.cs == 1 && g.C.rs % 4 == 0 && (!c0_used || (g.C0.cs == 1 && g.C0.rs % 4 == 0));
  const bool vcol = vok && !vrow && g.C.rs == 1 && g.C.cs % 4 == 0 &&
                    (!c0_used || (g.C0.rs == 1 && g.C0.cs % 4 == 0));
  g.c_vec = vrow || vcol;
  const bool swp = vrow || (!vcol && (ks > 1 || g.C.rs == 1));
#define KFB_FAST(AK, BK, SW)                                                                          \
  do {                                                                                                \
    if constexpr (SPL) {                                                                              \
      hipLaunchKernelGGL((gemm_bf16_fast_kernel<TC, TC0, AK, BK, SW, SPL, 128>), grid, dim3(MNT), 0, s, recs, g); \
    } else if (esc) {                                                                                 \
      if (tt == 256)                                                                                  \
        hipLaunchKernelGGL((gemm_bf16_fast_kernel<TC, TC0, AK, BK, SW, false, 256, true>), grid, dim3(512), 0, s, recs, g); \
      else                                                                                            \
        hipLaunchKernelGGL((gemm_bf16_fast_kernel<TC, TC0, AK, BK, SW, false, 128, true>), grid, dim3(MNT), 0, s, recs, g); \
    } else if (tt == 256) {                                                                           \
      hipLaunchKernelGGL((gemm_bf16_fast_kernel<TC, TC0, AK, BK, SW, false, 256>), grid, dim3(512), 0, s, recs, g); \
    } else {                                                                                          \
      hipLaunchKernelGGL((gemm_bf16_fast_kernel<TC, TC0, AK, BK, SW, false, 128>), grid, dim3(MNT), 0, s, recs, g); \
    }                                                                                                 \
  } while (0)
  if (swp) {
    if (ao && bo) KFB_FAST(true, true, true);
    else if (ao) KFB_FAST(true, false, true);
    else if (bo) KFB_FAST(false, true, true);
    else KFB_FAST(false, false, true);
  } else {
    if (ao && bo) KFB_FAST(true, true, false);
    else if (ao) KFB_FAST(true, false, false);
    else if (bo) KFB_FAST(false, true, false);
    else KFB_FAST(false, false, false);
  }
#undef KFB_FAST
  *err = hipGetLastError();
  if (*err != hipSuccess || ks == 1) return true;
  const int64_t mn = (int64_t)g.m * g.n;
  int blocks = (int)((mn + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL((mfma_splitk_reduce<TC, TC0>), dim3(blocks, nrec), dim3(256), 0, s, recs, g);
  *err = hipGetLastError();
  return true;
}

// fixed-order sum of split-K partials (FP32), then alpha / beta epilogue
template <typename TC, typename TC0>
__global__ __launch_bounds__(256) void mfma_splitk_reduce(const Rec* __restrict__ recs, GemmArgs g) {
  const Rec& rec = recs[blockIdx.y];
  const int64_t mn = (int64_t)g.m * g.n;
  const float* part = at<const float>(rec, g.Part.slot, g.Part.off);
  TC* C = at<TC>(rec, g.C.slot, g.C.off);
  const bool use_c0 = g.C0.slot >= 0 && (g.beta != 0.0 || g.beta_slot >= 0);
  const TC0* C0 = use_c0 ? at<const TC0>(rec, g.C0.slot, g.C0.off) : nullptr;
  const float beta = g.beta_slot >= 0 ? (float)*at<const double>(rec, g.beta_slot, g.beta_off) : (float)g.beta;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < mn;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % g.m), j = (int)(e / g.m);
    float sum = 0.f;
    for (int kz = 0; kz < g.ksplit; ++kz) sum += part[kz * mn + e];
    float v = (float)g.alpha * sum;
    if (C0) v += beta * to_f(C0[i * g.C0.rs + j * g.C0.cs]);
    C[i * g.C.rs + j * g.C.cs] = TC(v);
  }
}

template <typename TA, typename TB, typename TC, typename TC0, int SPLIT>
hipError_t gemm_bf16(const Rec* recs, int nrec, const GemmArgs& g0, hipStream_t s) {
  if (g0.m <= 0 || g0.n <= 0 || nrec <= 0) return hipSuccess;
  if constexpr (sizeof(TA) == 4 && sizeof(TB) == 4 && sizeof(TC) == 4) {
    hipError_t e;
    if (gemm_bf16_fast<TC, TC0, SPLIT != 0>(recs, nrec, g0, s, &e)) return e;
  }
  GemmArgs g = g0;
  if (g.k < 0) g.k = 0;
  const int tiles_m = (g.m + MBM - 1) / MBM, tiles_n = (g.n + MBN - 1) / MBN;
  int ks = g.ksplit < 1 ? 1 : g.ksplit;
  if (ks > 1) {
    int chunk = (g.k + ks - 1) / ks;
    chunk = ((chunk + MBK - 1) / MBK) * MBK;
    ks = (g.k + chunk - 1) / chunk;
    g.kchunk = chunk;
  } else {
    g.kchunk = g.k > 0 ? g.k : 1;
  }
  g.ksplit = ks;
  if ((g.rsc_slot >= 0 || g.c0cs_slot >= 0) && (SPLIT != 0 || ks > 1)) return hipErrorInvalidValue;
  dim3 grid(tiles_m * ks, tiles_n, nrec);
  hipLaunchKernelGGL((gemm_bf16_kernel<TA, TB, TC, TC0, SPLIT>), grid, dim3(MNT), 0, s, recs, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || ks == 1) return e;
  const int64_t mn = (int64_t)g.m * g.n;
  int blocks = (int)((mn + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL((mfma_splitk_reduce<TC, TC0>), dim3(blocks, nrec), dim3(256), 0, s, recs, g);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP32 products on FP32 MFMA (v_mfma_f32_16x16x4f32): FP32 operands (B may be
// FP64, rounded to FP32 on load, as the FMA engine does), FP32 accumulation:
// the FP32 form's products, and Q = Z R^-1 of the mixed form's CholeskyQR.
// 128 x 128 tiles of four waves (64 x 64 each), k in steps of 16 staged in LDS
// (k-major rows, so a wave's fragment reads are consecutive words), the next
// step's operands loaded while the current one is multiplied; XCD-aware tile
// order; column-major outputs issue (B^T A^T) so the stores coalesce.  Each
// operand is read along its contiguous dimension (consecutive threads take
// consecutive elements in memory) and may be a two-segment block matrix
// (A = [A1 | A2] split at column `split`, B = [B1 ; B2] split at row `split`,
// both segments of one orientation); split-K partials go to the fixed-order
// reduction.  With b_upper the k loop of a tile stops at its last column (the
// skipped terms are exact zeros).
// ---------------------------------------------------------------------------
constexpr int F32_BK = 16, F32_LD = 128 + 4;

template <typename TB, typename TC0, bool SWP>
__global__ __launch_bounds__(256) void gemm_f32_mfma_kernel(const Rec* __restrict__ recs, GemmArgs g) {
  __shared__ float sA[2][F32_BK][F32_LD];
  __shared__ float sB[2][F32_BK][F32_LD];
  int tm, tn, tz;
  xcd_tile(gridDim.x, gridDim.y, gridDim.z, &tm, &tn, &tz);
  const Rec& rec = recs[tz];
  // split-K: blockIdx.x also enumerates the k chunks (tm = kz * tiles_m + tile row)
  const int tiles_m = (g.m + 127) / 128, kz = tm / tiles_m;
  tm -= kz * tiles_m;
  const float* A = at<const float>(rec, g.A.slot, g.A.off);
  const float* A2 = g.A.slot2 >= 0 ? at<const float>(rec, g.A.slot2, g.A.off2) : nullptr;
  const TB* B = at<const TB>(rec, g.B.slot, g.B.off);
  const TB* B2 = g.B.slot2 >= 0 ? at<const TB>(rec, g.B.slot2, g.B.off2) : nullptr;
  const int asplit = A2 ? g.A.split : 0x7fffffff, bsplit = B2 ? g.B.split : 0x7fffffff;
  // contiguous dimension of each operand: A along k (row-major A) or along i;
  // B along j (row-major B) or along k
  const bool a_k = g.A.cs == 1 && g.A.rs != 1, b_j = g.B.cs == 1 && g.B.rs != 1;
  const int t = threadIdx.x, w = t / 64, l = t % 64;
  const int wm = (w & 1) * 64, wn = (w >> 1) * 64;
  const int m0 = tm * 128, n0 = tn * 128;
  const int kbeg = g.ksplit > 1 ? kz * g.kchunk : 0;
  int kend = g.ksplit > 1 ? min(g.k, kbeg + g.kchunk) : g.k;
  // an upper-triangular B contributes nothing below the tile's last column
  if (g.b_upper) kend = min(kend, n0 + 128);
  // staging: element e = t + 256 q of the 128 x 16 A tile is (i, k) = (e % 128, e / 128),
  // or (e / 16, e % 16) when A runs along k; of the 16 x 128 B tile (k, j) = (e % 16, e / 16),
  // or (e / 128, e % 128) when B runs along j
  float ra[8], rb[8];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = t + 256 * q;
      const int ia = a_k ? e / F32_BK : e % 128, ka = a_k ? e % F32_BK : e / 128;
      const int gi = m0 + ia, gk = k0 + ka;
      float va = 0.f;
      if (gi < g.m && gk < kend)
        va = gk < asplit ? A[(int64_t)gi * g.A.rs + (int64_t)gk * g.A.cs]
                         : A2[(int64_t)gi * g.A.rs2 + (int64_t)(gk - asplit) * g.A.cs2];
      ra[q] = va;
      const int kb = b_j ? e / 128 : e % F32_BK, jb = b_j ? e % 128 : e / F32_BK;
      const int gj = n0 + jb, gkb = k0 + kb;
      float vb = 0.f;
      if (gj < g.n && gkb < kend)
        vb = (float)(gkb < bsplit ? B[(int64_t)gkb * g.B.rs + (int64_t)gj * g.B.cs]
                                  : B2[(int64_t)(gkb - bsplit) * g.B.rs2 + (int64_t)gj * g.B.cs2]);
      rb[q] = vb;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = t + 256 * q;
      if (a_k) sA[buf][e % F32_BK][e / F32_BK] = ra[q];
      else sA[buf][e / 128][e % 128] = ra[q];
      if (b_j) sB[buf][e / 128][e % 128] = rb[q];
      else sB[buf][e % F32_BK][e / F32_BK] = rb[q];
    }
  };
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  load(kbeg);
  store(0);
  __syncthreads();
  int cur = 0;
  for (int k0 = kbeg; k0 < kend; k0 += F32_BK) {
    const bool more = k0 + F32_BK < kend;
    if (more) load(k0 + F32_BK);
#pragma unroll
    for (int ks = 0; ks < F32_BK / 4; ++ks) {
      const int kr = 4 * ks + l / 16;
      float af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        af[i] = sA[cur][kr][wm + 16 * i + (l % 16)];
        bf[i] = sB[cur][kr][wn + 16 * i + (l % 16)];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = SWP ? __builtin_amdgcn_mfma_f32_16x16x4f32(bf[j], af[i], acc[i][j], 0, 0, 0)
                          : __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
  if (g.ksplit > 1) {  // partial sums, [kz][i + j m]
    float* part = at<float>(rec, g.Part.slot, g.Part.off) + (int64_t)kz * g.m * g.n;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          int gi, gj;
          if (SWP) { gi = m0 + wm + 16 * i + (l % 16); gj = n0 + wn + 16 * j + 4 * (l / 16) + v; }
          else { gi = m0 + wm + 16 * i + 4 * (l / 16) + v; gj = n0 + wn + 16 * j + (l % 16); }
          if (gi < g.m && gj < g.n) part[gi + (int64_t)gj * g.m] = acc[i][j][v];
        }
    return;
  }
  float* C = at<float>(rec, g.C.slot, g.C.off);
  const bool use_c0 = g.C0.slot >= 0 && (g.beta != 0.0 || g.beta_slot >= 0);
  const TC0* C0 = use_c0 ? at<const TC0>(rec, g.C0.slot, g.C0.off) : nullptr;
  const float alpha = (float)g.alpha;
  const float beta = g.beta_slot >= 0 ? (float)*at<const double>(rec, g.beta_slot, g.beta_off) : (float)g.beta;
  if constexpr (!SWP) {
    if (g.c_vec) {  // column-major C: each lane's four results are four consecutive rows
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int gi = m0 + wm + 16 * i + 4 * (l / 16), gj = n0 + wn + 16 * j + (l % 16);
          if (gi < g.m && gj < g.n) {  // m % 4 == 0: all four rows in range
            f32x4 val = alpha * acc[i][j];
            if (C0)
#pragma unroll
              for (int v = 0; v < 4; ++v) val[v] += beta * to_f(C0[(gi + v) * g.C0.rs + gj * g.C0.cs]);
            *reinterpret_cast<f32x4*>(&C[gi + (int64_t)gj * g.C.cs]) = val;
          }
        }
      return;
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int gi, gj;
        if (SWP) { gi = m0 + wm + 16 * i + (l % 16); gj = n0 + wn + 16 * j + 4 * (l / 16) + v; }
        else { gi = m0 + wm + 16 * i + 4 * (l / 16) + v; gj = n0 + wn + 16 * j + (l % 16); }
        if (gi < g.m && gj < g.n) {
          float val = alpha * acc[i][j][v];
          if (C0) val += beta * to_f(C0[(int64_t)gi * g.C0.rs + (int64_t)gj * g.C0.cs]);
          C[(int64_t)gi * g.C.rs + (int64_t)gj * g.C.cs] = val;
        }
      }
}

template <typename TB, typename TC0>
hipError_t gemm_f32_mfma(const Rec* recs, int nrec, const GemmArgs& g0, hipStream_t s) {
  if (g0.m <= 0 || g0.n <= 0 || nrec <= 0) return hipSuccess;
  GemmArgs g = g0;
  if (g.k < 0) g.k = 0;
  // a segmented operand: both segments run along the same dimension
  auto seg_ok = [](const OpRef& o) {
    if (o.slot2 < 0) return true;
    const bool c1 = o.cs == 1 && o.rs != 1, c2 = o.cs2 == 1 && o.rs2 != 1;
    return c1 == c2 && o.split > 0;
  };
  if (!seg_ok(g.A) || !seg_ok(g.B)) return hipErrorInvalidValue;
  int ks = g.ksplit < 1 || g.k == 0 ? 1 : g.ksplit;
  if (ks > 1) {  // chunks of whole k steps, the fixed-order reduction afterwards
    if (g.Part.slot < 0) return hipErrorInvalidValue;
    int chunk = (g.k + ks - 1) / ks;
    chunk = ((chunk + F32_BK - 1) / F32_BK) * F32_BK;
    ks = (g.k + chunk - 1) / chunk;
    g.kchunk = chunk;
  }
  g.ksplit = ks;
  dim3 grid(((g.m + 127) / 128) * ks, (g.n + 127) / 128, nrec);
  // column-major C with 16-byte columns (c_vec): the plain issue gives each lane
  // four consecutive rows, stored as one vector
  g.c_vec = ks == 1 && g.c_vec && g.C.rs == 1 && g.C.cs % 4 == 0 && g.m % 4 == 0;
  const bool plain = g.c_vec || (ks == 1 && g.C.rs != 1);
  if (plain) hipLaunchKernelGGL((gemm_f32_mfma_kernel<TB, TC0, false>), grid, dim3(256), 0, s, recs, g);
  else hipLaunchKernelGGL((gemm_f32_mfma_kernel<TB, TC0, true>), grid, dim3(256), 0, s, recs, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || ks == 1) return e;
  const int64_t mn = (int64_t)g.m * g.n;
  int blocks = (int)((mn + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL((mfma_splitk_reduce<float, TC0>), dim3(blocks, nrec), dim3(256), 0, s, recs, g);
  return hipGetLastError();
}
template hipError_t gemm_f32_mfma<double, float>(const Rec*, int, const GemmArgs&, hipStream_t);
template hipError_t gemm_f32_mfma<float, float>(const Rec*, int, const GemmArgs&, hipStream_t);

// ---------------------------------------------------------------------------
// FP64 products on FP64 MFMA (v_mfma_f64_16x16x4f64): the small square
// products of the eigenpair refinement (Ogita-Aishima step) that follows the
// mixed form's FP32 core eigensolve.  C = alpha A B + beta C0, all FP64, plain
// operands.  64 x 64 tiles of four waves (32 x 32 each), k in steps of 16
// staged in LDS (k-major rows), the next step's operands loaded while the
// current one is multiplied; each operand read along its contiguous dimension;
// XCD-aware tile order.  Result v of a lane of the FP64 instruction is row
// lane / 16 + 4 v, column lane % 16: a column-major C takes the transposed issue
// (B^T A^T) so that 16 consecutive lanes store 16 consecutive rows.  A
// symmetric product (sym: X^T X, Y^T Y) computes the tiles on and above the
// diagonal and writes each result at both of its positions.
// ---------------------------------------------------------------------------
constexpr int D64_BM = 64, D64_BK = 16, D64_LD = 64 + 2;
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double f64x4;

template <bool SWP>
__global__ __launch_bounds__(256) void gemm_f64_mfma_kernel(const Rec* __restrict__ recs, GemmArgs g) {
  __shared__ double sA[2][D64_BK][D64_LD];
  __shared__ double sB[2][D64_BK][D64_LD];
  int tm, tn, tz;
  xcd_tile(gridDim.x, gridDim.y, gridDim.z, &tm, &tn, &tz);
  if (g.sym && tm > tn) return;  // the mirror of a tile above the diagonal
  const Rec& rec = recs[tz];
  const double* A = at<const double>(rec, g.A.slot, g.A.off);
  const double* B = at<const double>(rec, g.B.slot, g.B.off);
  const bool a_k = g.A.cs == 1 && g.A.rs != 1, b_j = g.B.cs == 1 && g.B.rs != 1;
  const int t = threadIdx.x, w = t / 64, l = t % 64;
  const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
  const int m0 = tm * D64_BM, n0 = tn * D64_BM;
  // staging: element e = t + 256 q (q < 4) of the 64 x 16 A tile is (i, k) =
  // (e % 64, e / 64), or (e / 16, e % 16) along k; of the 16 x 64 B tile (k, j) =
  // (e % 16, e / 16), or (e / 64, e % 64) along j
  double ra[4], rb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + 256 * q;
      const int ia = a_k ? e / D64_BK : e % D64_BM, ka = a_k ? e % D64_BK : e / D64_BM;
      const int gi = m0 + ia, gk = k0 + ka;
      ra[q] = (gi < g.m && gk < g.k) ? A[(int64_t)gi * g.A.rs + (int64_t)gk * g.A.cs] : 0.0;
      const int kb = b_j ? e / D64_BM : e % D64_BK, jb = b_j ? e % D64_BM : e / D64_BK;
      const int gj = n0 + jb, gkb = k0 + kb;
      rb[q] = (gj < g.n && gkb < g.k) ? B[(int64_t)gkb * g.B.rs + (int64_t)gj * g.B.cs] : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + 256 * q;
      if (a_k) sA[buf][e % D64_BK][e / D64_BK] = ra[q];
      else sA[buf][e / D64_BM][e % D64_BM] = ra[q];
      if (b_j) sB[buf][e / D64_BM][e % D64_BM] = rb[q];
      else sB[buf][e % D64_BK][e / D64_BK] = rb[q];
    }
  };
  f64x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  load(0);
  store(0);
  __syncthreads();
  int cur = 0;
  for (int k0 = 0; k0 < g.k; k0 += D64_BK) {
    const bool more = k0 + D64_BK < g.k;
    if (more) load(k0 + D64_BK);
#pragma unroll
    for (int ks = 0; ks < D64_BK / 4; ++ks) {
      const int kr = 4 * ks + l / 16;
      double af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        af[i] = sA[cur][kr][wm + 16 * i + (l % 16)];
        bf[i] = sB[cur][kr][wn + 16 * i + (l % 16)];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = SWP ? __builtin_amdgcn_mfma_f64_16x16x4f64(bf[j], af[i], acc[i][j], 0, 0, 0)
                          : __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
  double* C = at<double>(rec, g.C.slot, g.C.off);
  const bool use_c0 = g.C0.slot >= 0 && g.beta != 0.0;
  const double* C0 = use_c0 ? at<const double>(rec, g.C0.slot, g.C0.off) : nullptr;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int gi, gj;
        if (SWP) { gi = m0 + wm + 16 * i + (l % 16); gj = n0 + wn + 16 * j + (l / 16) + 4 * v; }
        else { gi = m0 + wm + 16 * i + (l / 16) + 4 * v; gj = n0 + wn + 16 * j + (l % 16); }
        if (gi < g.m && gj < g.n) {
          double val = g.alpha * acc[i][j][v];
          if (C0) val += g.beta * C0[(int64_t)gi * g.C0.rs + (int64_t)gj * g.C0.cs];
          C[(int64_t)gi * g.C.rs + (int64_t)gj * g.C.cs] = val;
          if (g.sym && tm < tn) C[(int64_t)gj * g.C.rs + (int64_t)gi * g.C.cs] = val;
        }
      }
}

hipError_t gemm_f64_mfma(const Rec* recs, int nrec, const GemmArgs& g, hipStream_t s) {
  if (g.m <= 0 || g.n <= 0 || nrec <= 0) return hipSuccess;
  if (g.A.slot2 >= 0 || g.B.slot2 >= 0 || g.ksplit > 1 || g.beta_slot >= 0 || g.k < 0 ||
      (g.sym && (g.m != g.n || g.C0.slot >= 0)))
    return hipErrorInvalidValue;
  dim3 grid((g.m + D64_BM - 1) / D64_BM, (g.n + D64_BM - 1) / D64_BM, nrec);
  if (g.C.rs == 1) hipLaunchKernelGGL((gemm_f64_mfma_kernel<true>), grid, dim3(256), 0, s, recs, g);
  else hipLaunchKernelGGL((gemm_f64_mfma_kernel<false>), grid, dim3(256), 0, s, recs, g);
  return hipGetLastError();
}

#define KFB_GEMM_BF16(TA, TB, TC, TC0, SP) \
  template hipError_t gemm_bf16<TA, TB, TC, TC0, SP>(const Rec*, int, const GemmArgs&, hipStream_t);
// mixed-form update: projections (U FP32 split, M BF16 exact), residuals, rotation
KFB_GEMM_BF16(float, bf16, float, float, 1)
KFB_GEMM_BF16(float, float, float, bf16, 1)
KFB_GEMM_BF16(float, float, float, float, 1)
// mixed-form preconditioner (single BF16 terms)
KFB_GEMM_BF16(float, float, float, float, 0)
// mixed-form dense EA factor: X = rho X + w M M^T from BF16 batches (exact products)
KFB_GEMM_BF16(bf16, bf16, float, float, 0)
#undef KFB_GEMM_BF16

}  // namespace kfb
