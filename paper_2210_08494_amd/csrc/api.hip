// C-ABI of the kfb library: state lifecycle, the Brand update (Algorithm 4 on
// top of Algorithm 3) and the two-sided inverse application (Algorithm 1
// inverse lines), as stream-ordered sequences of the stage kernels.
#include <string.h>
#include <stdlib.h>
#include <new>
#include <memory>
#include <mutex>
#include <string>
#include <vector>
#include <stdio.h>

#include "kfb_kernels.h"

using namespace kfb;

struct kfb_state_s {
  int64_t d = 0;
  int32_t r = 0, n_max = 0, prec = 0;
  double rho = 0.0;
  char* buf = nullptr;
  size_t bytes = 0;
  int64_t ldu = 0;
  size_t off_U[2] = {0, 0}, off_D[2] = {0, 0}, off_status = 0;
  int front = 0;
  int32_t k_valid = 0;
  int64_t step = 0;
};

namespace {

#define KFB_TRY(x)                                   \
  do {                                               \
    hipError_t _e = (x);                             \
    if (_e != hipSuccess) return KFB_EHIP;           \
  } while (0)

// ---------------------------------------------------------------------------
// Optional stage timing (kfb_profile_enable / kfb_profile_report)
// ---------------------------------------------------------------------------
struct ProfStage {
  const char* name;
  long calls = 0, launches = 0;
  double ms = 0.0;
};
struct ProfPending {
  int stage;
  hipEvent_t a, b;
};
struct Prof {
  bool on = false;
  std::mutex mu;
  std::vector<ProfStage> stages;
  std::vector<ProfPending> pending;
  std::vector<hipEvent_t> pool;
  int index(const char* nm) {
    for (size_t i = 0; i < stages.size(); ++i)
      if (strcmp(stages[i].name, nm) == 0) return (int)i;
    ProfStage st;
    st.name = nm;
    stages.push_back(st);
    return (int)stages.size() - 1;
  }
  hipEvent_t get() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
Prof g_prof;

// RAII bracket: records an event at construction and at destruction (on s)
struct StageTimer {
  const char* name;
  hipStream_t s;
  hipEvent_t a = nullptr;
  int launches;
  StageTimer(const char* nm, hipStream_t st, int nl) : name(nm), s(st), launches(nl) {
    if (!g_prof.on) return;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    a = g_prof.get();
    if (a) (void)hipEventRecord(a, s);
  }
  ~StageTimer() {
    if (!g_prof.on || !a) return;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    hipEvent_t b = g_prof.get();
    if (!b) return;
    (void)hipEventRecord(b, s);
    const int ix = g_prof.index(name);
    g_prof.stages[ix].calls += 1;
    g_prof.stages[ix].launches += launches;
    g_prof.pending.push_back(ProfPending{ix, a, b});
  }
};

// ---------------------------------------------------------------------------
// Tuning table: core eigensolver block width per (precision form, N)
// ---------------------------------------------------------------------------
struct TuneEntry {
  int prec, N, bw;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;

int tuned_bw(int prec, int N) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& e : g_tune)
    if (e.prec == prec && e.N == N) return e.bw;
  return 0;
}

// Eigensolver configuration for a core of size N (element size es): the tuning
// table's entry, else, where streamed panels are preferred (cores of N >= 256;
// the new-direction block solve always), 64-column panels streamed from global
// memory (the autotuner's pick at the headline core; in the mixed form the
// iteration in FP32 with the FP64 refinement, JAC_REFINE, where `refine`), else
// the widest LDS panel.  Writes the padded size; returns 0 if nothing fits.
int pick_jacobi(int prec, int N, int es, bool prefer_streamed, int* Np, bool refine = false) {
  int cfg = tuned_bw(prec, N);
  if (!cfg && prefer_streamed) cfg = JAC_STREAMED | 32 | (refine && prec == KFB_BF16_MIXED ? JAC_REFINE : 0);
  const int np = cfg ? jacobi_block_fits(N, es, cfg & ~JAC_REFINE) : 0;
  if (np) {
    *Np = np;
    return cfg;
  }
  return jacobi_pick_block(N, es, Np);
}

inline size_t u_elem(int prec) { return prec == KFB_FP64 ? 8 : 4; }
inline size_t d_elem(int prec) { return prec == KFB_FP32 ? 4 : 8; }
inline size_t m_elem(int prec) { return prec == KFB_FP64 ? 8 : (prec == KFB_FP32 ? 4 : 2); }
inline size_t g_elem(int prec) { return prec == KFB_FP64 ? 8 : 4; }
inline int64_t ldu_for(int64_t d, int prec) {
  const int64_t q = 256 / (int64_t)u_elem(prec);
  return ((d + q - 1) / q) * q;
}

// per-precision element types
template <int PR> struct Ty;
template <> struct Ty<KFB_FP64> {
  typedef double U, M, Z, P, G, Core, W, D, Acc;
};
template <> struct Ty<KFB_FP32> {
  typedef float U, M, Z, P, G, Core, W, D, Acc;
};
template <> struct Ty<KFB_BF16_MIXED> {
  typedef float U, Z, P, W, Acc;
  typedef bf16 M;
  typedef double G, Core, D;
};

constexpr int MAX_SWEEPS = 20;

// threshold of the orthonormality-drift detector on squared column norms
inline double drift_tol(int prec) { return prec == KFB_FP64 ? 1e-10 : (prec == KFB_FP32 ? 1e-4 : 1e-3); }

// ---------------------------------------------------------------------------
// Brand-update plan: workspace layout of one problem for a shape bucket.
// ---------------------------------------------------------------------------
struct UpdPlan {
  int64_t d, ldu, ldm;
  int r, n, N, Np, bw;
  int ksP, ksG;
  int64_t oZ, oZb, oP, oP2, oGram, oR1, oX1, oR2, oX2, oR3, oRt, oPart, oB, oV, oW, oLam, oRank, oCnt;
  // refine (mixed form, JAC_REFINE): FP32 copies of the core and its rotations,
  // and Y = L^T X, S = X^T K X, G = X^T X (then E) of the FP64 refinement
  bool refine = false;
  int64_t oB32 = -1, oV32 = -1, oK = -1, oS = -1, oG = -1, oDelta = -1;
  // pre-rotation of the new-direction block: eigensolve of size n first (pre)
  bool pre = false;
  int preNp = 0, prebw = 0;
  int64_t oPB = -1, oPV = -1, oPCnt = -1;
  size_t per_problem;
};

// The core's trailing n x n block (the new directions, w R R^T) is
// diagonalised first by an eigensolve of size n on sqrt(w) R^T; the main
// eigensolve then starts from B = L^T diag(I, V_R), V = diag(I, V_R), whose
// leading block (rho D + w P P^T) is already close to diagonal.  This cuts the
// main iteration's sweeps by about a third at the widths where the core is
// large enough for the eigensolver's cost to matter.
// The block solve is only a preconditioner (any orthogonal V_R is correct), so
// it stops after PRE_SWEEPS sweeps: more buys no further reduction.
constexpr int PRE_MIN_N = 128, PRE_SWEEPS = 5;

template <int PR>
bool make_upd_plan(int64_t d, int64_t ldu, int64_t ldm, int r, int n, int nrec, UpdPlan* p) {
  typedef Ty<PR> T;
  // the CholeskyQR kernels and the eigensolver's finalize bound the widths
  if (n < 1 || r < 0 || n > MAX_QR_COLS || r + n > MAX_CORE) return false;
  p->d = d; p->ldu = ldu; p->ldm = ldm; p->r = r; p->n = n; p->N = r + n;
  {
    const int cfg = pick_jacobi(PR, p->N, (int)sizeof(typename T::Core), p->N >= 256, &p->Np, true);
    p->refine = (cfg & JAC_REFINE) != 0;
    p->bw = cfg & ~JAC_REFINE;
  }
  if (p->bw == 0) return false;
  auto ks_for = [&](int m, int nn, int64_t k) {
    // split depends on the problem's own shape only, never on its batch-mates
    const int tiles = ((m + 63) / 64) * ((nn + 63) / 64);
    int ks = 1;
    // enough workgroups for one problem alone (64 tile-splits); more splits only
    // add partial-sum traffic, which a grouped call pays once per problem
    while (tiles * ks < 64 && (k / (ks * 2)) >= 256) ks *= 2;
    return ks;
  };
  p->ksP = r > 0 ? ks_for(r, n, d) : 1;
  p->ksG = ks_for(n, n, d);
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at_ = o; o = align256(o + bytes); return (int64_t)at_; };
  p->oZ = take((size_t)d * n * sizeof(typename T::Z));
  p->oZb = take((size_t)d * n * sizeof(typename T::Z));
  p->oP = take((size_t)(r > 0 ? r : 1) * n * sizeof(typename T::P));
  p->oP2 = take((size_t)(r > 0 ? r : 1) * n * sizeof(typename T::P));
  const size_t nn = (size_t)n * n * sizeof(typename T::G);
  p->oGram = take(nn); p->oR1 = take(nn); p->oX1 = take(nn); p->oR2 = take(nn); p->oX2 = take(nn);
  p->oR3 = take(nn);
  p->oRt = take(nn);
  const size_t partP = (size_t)p->ksP * (r > 0 ? r : 1) * n * sizeof(typename T::P);
  const size_t partG = (size_t)p->ksG * n * n * sizeof(typename T::G);
  p->oPart = take(partP > partG ? partP : partG);
  const size_t core = (size_t)p->Np * p->Np * sizeof(typename T::Core);
  p->oB = take(core); p->oV = take(core);
  p->oW = take((size_t)p->N * p->N * sizeof(typename T::W));
  p->oLam = take((size_t)2 * p->Np * sizeof(typename T::Core));  // eigenvalues, then 1/||V_j||
  p->oRank = take((size_t)p->Np * 4);
  p->oCnt = take((size_t)MAX_SWEEPS * 4);
  p->pre = r > 0 && n >= PRE_MIN_N;
  if (p->pre) {
    p->prebw = pick_jacobi(PR, n, (int)sizeof(typename T::Core), true, &p->preNp) & ~JAC_REFINE;
    // the FP32 iteration runs its block solve on the FP32 streamed kernel as well
    if (p->refine) {
      p->prebw = JAC_STREAMED | 32;
      p->preNp = jacobi_block_fits(n, 4, JAC_STREAMED | 32);
    }
    if (p->prebw == 0 || p->preNp == 0) p->pre = false;
  }
  if (p->refine) {
    const size_t c32 = (size_t)p->Np * p->Np * 4, k64 = (size_t)p->N * p->N * 8;
    p->oB32 = take(c32); p->oV32 = take(c32);
    p->oK = take(k64); p->oS = take(k64); p->oG = take(k64);
    p->oDelta = take(8 * (1 + 3 * OA_BLOCKS));  // the refinement threshold's partial sums
  }
  if (p->pre) {
    const size_t pc = (size_t)p->preNp * p->preNp * sizeof(typename T::Core);
    p->oPB = take(pc); p->oPV = take(pc);
    p->oPCnt = take((size_t)MAX_SWEEPS * 4);
  }
  p->per_problem = o;
  return true;
}

inline OpRef op(int slot, int64_t off, int64_t rs, int64_t cs) {
  OpRef o;
  o.slot = slot; o.off = off; o.rs = rs; o.cs = cs;
  return o;
}

// Product dispatch: the mixed form runs its FP32 products on BF16 MFMA
// (SPLIT = 1: operands carried as BF16 hi + lo terms), the FP32 form its
// products on FP32 MFMA (FP32 operands and accumulation), the FP64 form on the
// FP64 FMA engine.
template <int PR, int SPLIT, typename TA, typename TB, typename TC, typename TC0, typename TAcc>
hipError_t mm(const Rec* recs, int nrec, const GemmArgs& g, hipStream_t s) {
  if constexpr (PR == KFB_BF16_MIXED && sizeof(TA) == 4 && sizeof(TC) == 4 && sizeof(TAcc) == 4 &&
                (sizeof(TB) == 4 || sizeof(TB) == 2)) {
    return gemm_bf16<TA, TB, TC, TC0, SPLIT>(recs, nrec, g, s);
  } else if constexpr (PR == KFB_FP32 && sizeof(TA) == 4 && sizeof(TB) == 4 && sizeof(TC) == 4 &&
                       sizeof(TC0) == 4 && sizeof(TAcc) == 4) {
    return gemm_f32_mfma<TB, TC0>(recs, nrec, g, s);
  } else {
    return gemm<TA, TB, TC, TC0, TAcc>(recs, nrec, g, s);
  }
}

// Thin QR of the d x n matrix at srcZ (Algorithm 3's QR of the residual; the
// re-orthonormalisation of the randomized range finder) by CholeskyQR: two
// passes when the Gram is formed in FP64; in the FP32 form a shifted first pass
// (shifted CholeskyQR3) keeps the factorisation stable for ill-conditioned
// inputs.  Ping-pongs between srcZ and altZ; returns the offsets of Q and of R
// (n x n upper triangular, the product of the passes' factors).
template <int PR>
int thin_qr(const Rec* drecs, int nrec, const UpdPlan& p, int64_t srcZ, int64_t altZ, int64_t* oQ_out,
            int64_t* oR_out, hipStream_t s) {
  typedef Ty<PR> T;
  typedef typename T::Z TZ; typedef typename T::G TG; typedef typename T::Acc TA;
  const int64_t d = p.d;
  const int n = p.n;
  const bool fp32_chol = sizeof(TG) == 4;
  const int passes = fp32_chol ? 3 : 2;
  const double ueps = fp32_chol ? 1.1920929e-07 : 2.220446049250313e-16;
  const double tau = 64.0 * ueps;
  int64_t dstZ = altZ;
  const int64_t oR[3] = {p.oR1, p.oR2, p.oR3}, oX[2] = {p.oX1, p.oX2};
  for (int pass = 0; pass < passes; ++pass) {
    bool prepped = false;
    if constexpr (sizeof(TG) == 8) {
      if (d % 16 == 0) {  // upper blocks on FP64 MFMA
        GramArgs ga;
        ga.n = n; ga.ks = p.ksG; ga.kchunk = 0; ga.d = d;
        ga.off_Z = srcZ; ga.off_part = p.oPart; ga.off_gram = p.oGram;
        ga.off_R = oR[pass]; ga.off_X = oX[pass & 1];  // the Cholesky's starting point
        KFB_TRY(gram_f64<TZ>(drecs, nrec, ga, s));
        prepped = true;
      } else {
        GemmArgs gg;
        gg.A = op(WS, srcZ, d, 1); gg.B = op(WS, srcZ, 1, d); gg.C = op(WS, p.oGram, 1, n);
        gg.m = n; gg.n = n; gg.k = (int)d; gg.ksplit = p.ksG; gg.Part = op(WS, p.oPart, 1, n);
        KFB_TRY((gemm<TZ, TZ, TG, TG, TG>(drecs, nrec, gg, s)));
      }
    } else {
      GemmArgs gg;
      gg.A = op(WS, srcZ, d, 1); gg.B = op(WS, srcZ, 1, d); gg.C = op(WS, p.oGram, 1, n);
      gg.m = n; gg.n = n; gg.k = (int)d; gg.ksplit = p.ksG; gg.Part = op(WS, p.oPart, 1, n);
      KFB_TRY((gemm<TZ, TZ, TG, TG, TG>(drecs, nrec, gg, s)));
    }
    CholArgs ca;
    ca.n = n; ca.off_gram = p.oGram; ca.off_R = oR[pass]; ca.off_Rinv = oX[pass & 1]; ca.off_rowbuf = 0;
    ca.tau_rel = tau;
    ca.shift_rel = (fp32_chol && pass == 0) ? 11.0 * ((double)d * n + (double)n * (n + 1)) * ueps : 0.0;
    ca.prepped = prepped ? 1 : 0;
    KFB_TRY(chol_inv<TG>(drecs, nrec, ca, s));
    GemmArgs q;
    q.A = op(WS, srcZ, 1, d); q.B = op(WS, oX[pass & 1], 1, n); q.C = op(WS, dstZ, 1, d);
    q.m = (int)d; q.n = n; q.k = n;
    q.b_upper = 1;  // R^-1 is upper triangular
    q.c_vec = 1;    // Q in the workspace
    if constexpr (sizeof(TZ) == 4 && sizeof(TA) == 4) {  // Q = Z R^-1 on FP32 MFMA
      if constexpr (sizeof(TG) == 8) {
        // R^-1 rounded to FP32 once (the FP32 product would round its operand on
        // every tile load): half the operand bytes.  The copy goes to oRt, which
        // no pass reads or writes (the product of the passes' factors lands
        // there only after the last pass), so it aliases nothing in flight.
        KFB_TRY((copy2d<float, TG>(drecs, nrec, op(WS, p.oRt, 1, n), op(WS, oX[pass & 1], 1, n), n, n, s)));
        q.B = op(WS, p.oRt, 1, n);
        KFB_TRY((gemm_f32_mfma<float, TZ>(drecs, nrec, q, s)));
      } else {
        KFB_TRY((gemm_f32_mfma<TG, TZ>(drecs, nrec, q, s)));
      }
    } else {
      KFB_TRY((gemm<TZ, TG, TZ, TZ, TA>(drecs, nrec, q, s)));
    }
    const int64_t tmp = srcZ; srcZ = dstZ; dstZ = tmp;
  }
  *oQ_out = srcZ;  // the orthonormal Q after the last pass
  // R = R_last ... R_1 (products of upper-triangular factors)
  {
    GemmArgs rr;
    rr.A = op(WS, p.oR2, 1, n); rr.B = op(WS, p.oR1, 1, n); rr.C = op(WS, p.oRt, 1, n);
    rr.m = n; rr.n = n; rr.k = n;
    KFB_TRY((gemm<TG, TG, TG, TG, TG>(drecs, nrec, rr, s)));
    if (passes == 3) {
      GemmArgs r3 = rr;
      r3.A = op(WS, p.oR3, 1, n); r3.B = op(WS, p.oRt, 1, n); r3.C = op(WS, p.oGram, 1, n);
      KFB_TRY((gemm<TG, TG, TG, TG, TG>(drecs, nrec, r3, s)));
    }
  }
  *oR_out = passes == 3 ? p.oGram : p.oRt;
  return KFB_OK;
}

// launches of one thin_qr (for the stage counters)
inline int thin_qr_launches(int prec, int ksG) {
  const int passes = prec == KFB_FP32 ? 3 : 2, kl = ksG > 1 ? 2 : 1;
  const int copies = prec == KFB_BF16_MIXED ? passes : 0;  // FP32 copy of R^-1 per pass
  return passes * (kl + 2) + passes - 1 + copies;
}

// Jacobi eigensolve of the assembled core (B, V in the plan's workspace) and
// finalize: eigenvalues descending into D_BACK, eigenvectors into W.
template <int PR>
int core_evd(const Rec* drecs, int nrec, const UpdPlan& p, hipStream_t s, bool fin = true,
             const char* stage = "jacobi", int sweeps = MAX_SWEEPS) {
  typedef Ty<PR> T;
  typedef typename T::Core TC; typedef typename T::W TW; typedef typename T::D TD;
  const int N = p.N;
  JacArgs ja;
  ja.Np = p.Np; ja.N = N; ja.b = p.bw; ja.max_sweeps = sweeps;
  ja.off_B = p.oB; ja.off_V = p.oV; ja.off_cnt = p.oCnt;
  const double eps = sizeof(TC) == 8 ? 2.220446049250313e-16 : 1.1920929e-07;
  // stopping rule |g_pq| <= tol sqrt(g_pp g_qq): machine precision in the FP64 and
  // FP32 forms; in the mixed form 1e-6, the FP32 form's scale (eps_32 sqrt(N) is
  // 1.7e-6 at N = 256), FP64 arithmetic throughout; the form's inputs are
  // rounded to BF16 (relative 3.9e-3), so the core's residual rotations stay
  // orders of magnitude below its own error
  ja.tol = PR == KFB_BF16_MIXED ? 1e-6 : eps * sqrt((double)N);
  const int nb = p.Np / (p.bw & 0xff);
  {
  StageTimer st_jac(stage, s, nb == 2 ? 1 : sweeps * (nb - 1));
  if (nb == 2) {
    KFB_TRY(jacobi_round<TC>(drecs, nrec, ja, 0, 0, s));
  } else {
    for (int sw = 0; sw < sweeps; ++sw)
      for (int rd = 0; rd < nb - 1; ++rd) KFB_TRY(jacobi_round<TC>(drecs, nrec, ja, sw, rd, s));
  }
  }
  if (!fin) return KFB_OK;
  FinArgs fa;
  fa.N = N; fa.Np = p.Np; fa.max_sweeps = MAX_SWEEPS; fa.off_B = p.oB; fa.off_V = p.oV;
  fa.off_cnt = p.oCnt; fa.off_lam = p.oLam; fa.off_rank = p.oRank; fa.off_W = p.oW;
  {
    StageTimer st_fin("finalize", s, 3);
    KFB_TRY((finalize_core<TC, TW, TD>(drecs, nrec, fa, s)));
  }
  return KFB_OK;
}

// Core eigensolve of the mixed form with JAC_REFINE: the one-sided Jacobi
// iteration (new-direction block, then the main one) runs on FP32 copies of the
// core on FP32 MFMA; its rotations X then start one FP64 refinement step of the
// eigenpairs of the FP64 core K = L L^T (Ogita-Aishima) on FP64 MFMA, with
// X^T K X formed as Y^T Y from Y = L^T X, so the eigenvalues and W carry FP64
// accuracy outside clusters of near-equal eigenvalues.  `co` describes the core
// (without pre-rotation).
template <int PR>
int core_evd_refined(const Rec* drecs, int nrec, const UpdPlan& p, const CoreArgs& co, hipStream_t s) {
  if constexpr (PR != KFB_BF16_MIXED) {
    return KFB_EINVAL;
  } else {
    typedef Ty<PR> T;
    typedef typename T::P TP; typedef typename T::G TG; typedef typename T::D TD; typedef typename T::W TW;
    const int N = p.N, n = p.n, Np = p.Np;
    {
      // B = L^T in FP64 (kept for the refinement)
      StageTimer st("core", s, 1);
      CoreArgs c64 = co;
      KFB_TRY((assemble_core<double, TP, TG, TD>(drecs, nrec, c64, s)));
    }
    // the FP32 iteration stops at 1e-5 rather than at FP32 round-off (eps_32 sqrt(N),
    // 2.7e-6 at N = 512): the refinement's error is quadratic in its input's, and
    // the last partial sweep it saves (~1 ms per 48-core call at the headline
    // shape) moved the tests' errors by less than 1e-7
    auto iterate = [&](int Nc, int Npc, int bw, int64_t oB, int64_t oV, int64_t oCnt, int sweeps,
                       const char* stage) -> int {
      JacArgs ja;
      ja.Np = Npc; ja.N = Nc; ja.b = bw; ja.max_sweeps = sweeps;
      ja.off_B = oB; ja.off_V = oV; ja.off_cnt = oCnt;
      ja.tol = 1e-5;
      const int nb = Npc / (bw & 0xff);
      StageTimer st(stage, s, sweeps * (nb - 1));
      for (int sw = 0; sw < sweeps; ++sw)
        for (int rd = 0; rd < nb - 1; ++rd) KFB_TRY(jacobi_round<float>(drecs, nrec, ja, sw, rd, s));
      return KFB_OK;
    };
    CoreArgs c32 = co;
    c32.off_B = p.oB32; c32.off_V = p.oV32;
    if (p.pre) {
      // block solve of sqrt(w) R^T in FP32 (the pre-rotation buffers hold FP32 here)
      CoreArgs cr;
      cr.r = 0; cr.n = n; cr.N = n; cr.Np = p.preNp; cr.off_P = p.oP; cr.off_P2 = -1;
      cr.off_R = co.off_R; cr.off_B = p.oPB; cr.off_V = p.oPV;
      {
        StageTimer st("core", s, 2);
        KFB_TRY((assemble_core<float, TP, TG, TD>(drecs, nrec, cr, s)));
        KFB_TRY(zero_words(drecs, nrec, WS, p.oPCnt, MAX_SWEEPS, s));
      }
      const int rc = iterate(n, p.preNp, p.prebw, p.oPB, p.oPV, p.oPCnt, PRE_SWEEPS, "jacobi_pre");
      if (rc != KFB_OK) return rc;
      c32.off_preB = p.oPB; c32.off_preV = p.oPV; c32.preNp = p.preNp;
    }
    {
      StageTimer st("core", s, 2);
      KFB_TRY((assemble_core<float, TP, TG, TD>(drecs, nrec, c32, s)));
      KFB_TRY(zero_words(drecs, nrec, WS, p.oCnt, MAX_SWEEPS, s));
    }
    {
      const int rc = iterate(N, Np, p.bw, p.oB32, p.oV32, p.oCnt, MAX_SWEEPS, "jacobi");
      if (rc != KFB_OK) return rc;
    }
    {
      // X = V (FP64, N x N at oV); Y = L^T X (the first N rows of B times X, at oK);
      // S = Y^T Y = X^T K X; G = X^T X; E over G; X' = X + X E (over B).  ||K|| in
      // the cluster threshold is taken as ||S|| (X is orthonormal to the FP32 level).
      StageTimer st("refine", s, 7);
      KFB_TRY((copy2d<double, float>(drecs, nrec, op(WS, p.oV, 1, N), op(WS, p.oV32, 1, Np), N, N, s)));
      GemmArgs g;
      g.m = N; g.n = N; g.k = N;
      g.A = op(WS, p.oB, 1, Np); g.B = op(WS, p.oV, 1, N); g.C = op(WS, p.oK, 1, N);
      KFB_TRY(gemm_f64_mfma(drecs, nrec, g, s));
      g.sym = 1;  // S and G: the tiles on and above the diagonal, mirrored
      g.A = op(WS, p.oK, N, 1); g.B = op(WS, p.oK, 1, N); g.C = op(WS, p.oS, 1, N);
      KFB_TRY(gemm_f64_mfma(drecs, nrec, g, s));
      g.A = op(WS, p.oV, N, 1); g.B = op(WS, p.oV, 1, N); g.C = op(WS, p.oG, 1, N);
      KFB_TRY(gemm_f64_mfma(drecs, nrec, g, s));
      g.sym = 0;
      OaArgs oa;
      oa.N = N; oa.off_K = p.oS; oa.off_S = p.oS; oa.off_G = p.oG; oa.off_lam = p.oLam; oa.off_delta = p.oDelta;
      KFB_TRY(oa_prepare(drecs, nrec, oa, s));
      KFB_TRY(oa_correct(drecs, nrec, oa, s));
      g.A = op(WS, p.oV, 1, N); g.B = op(WS, p.oG, 1, N); g.C = op(WS, p.oB, 1, N);
      g.C0 = op(WS, p.oV, 1, N); g.beta = 1.0;
      KFB_TRY(gemm_f64_mfma(drecs, nrec, g, s));
    }
    FinArgs fa;
    fa.N = N; fa.Np = N; fa.max_sweeps = MAX_SWEEPS; fa.off_B = p.oB; fa.off_V = p.oB;
    fa.off_cnt = p.oCnt; fa.off_lam = p.oLam; fa.off_rank = p.oRank; fa.off_W = p.oW;
    StageTimer st_fin("finalize", s, 2);
    KFB_TRY((finalize_sorted<TW, TD>(drecs, nrec, fa, s)));
    return KFB_OK;
  }
}

template <int PR>
int run_update(const Rec* drecs, int nrec, const UpdPlan& p, hipStream_t s) {
  typedef Ty<PR> T;
  typedef typename T::U TU; typedef typename T::M TM; typedef typename T::Z TZ;
  typedef typename T::P TP; typedef typename T::G TG; typedef typename T::Core TC;
  typedef typename T::W TW; typedef typename T::D TD; typedef typename T::Acc TA;
  const int64_t d = p.d, ldu = p.ldu, ldm = p.ldm;
  const int r = p.r, n = p.n, N = p.N;

  const int kl_P = p.ksP > 1 ? 2 : 1;
  if (r > 0) {
    // P = U_r^T M   (Algorithm 3: projection)
    StageTimer st_proj("proj", s, 2 * kl_P + 2);
    GemmArgs g;
    g.A = op(U_FRONT, 0, ldu, 1); g.B = op(M_IN, 0, 1, ldm); g.C = op(WS, p.oP, 1, r);
    g.m = r; g.n = n; g.k = (int)d; g.ksplit = p.ksP; g.Part = op(WS, p.oPart, 1, r);
    KFB_TRY((mm<PR, 1, TU, TM, TP, TP, TP>(drecs, nrec, g, s)));
    // Z = M - U_r P   (component outside span(U))
    GemmArgs z;
    z.A = op(U_FRONT, 0, 1, ldu); z.B = op(WS, p.oP, 1, r); z.C0 = op(M_IN, 0, 1, ldm);
    z.C = op(WS, p.oZ, 1, d); z.m = (int)d; z.n = n; z.k = r; z.alpha = -1.0; z.beta = 1.0;
    z.aligned16 = (d % 4 == 0) && (r % 4 == 0);  // U columns (ldu: 256 B multiples), P columns (ld r)
    z.c_vec = 1;  // Z in the workspace (the BF16 batch as C0 keeps the element-wise epilogue)
    KFB_TRY((mm<PR, 1, TU, TP, TZ, TM, TA>(drecs, nrec, z, s)));
    // re-projection: P2 = U_r^T Z;  Z -= U_r P2  (P + P2 enters the core)
    GemmArgs g2 = g;
    g2.B = op(WS, p.oZ, 1, d); g2.C = op(WS, p.oP2, 1, r);
    g2.aligned16 = (d % 4 == 0) && (r % 4 == 0);  // U and Z columns (the result goes through split-K)
    KFB_TRY((mm<PR, 1, TU, TZ, TP, TP, TP>(drecs, nrec, g2, s)));
    GemmArgs z2 = z;
    z2.B = op(WS, p.oP2, 1, r); z2.C0 = op(WS, p.oZ, 1, d);
    KFB_TRY((mm<PR, 1, TU, TP, TZ, TZ, TA>(drecs, nrec, z2, s)));
  } else {
    StageTimer st_copy("proj", s, 1);
    KFB_TRY((copy2d<TZ, TM>(drecs, nrec, op(WS, p.oZ, 1, d), op(M_IN, 0, 1, ldm), (int)d, n, s)));
  }
  int64_t oQ, oRfin;
  std::unique_ptr<StageTimer> st_qr(new StageTimer("cholqr", s, thin_qr_launches(PR, p.ksG)));
  {
    const int rc = thin_qr<PR>(drecs, nrec, p, p.oZ, p.oZb, &oQ, &oRfin, s);
    if (rc != KFB_OK) return rc;
  }
  st_qr.reset();
  // core square factor and Jacobi eigensolve (Algorithm 3: EVD of M_S)
  CoreArgs co;
  co.r = r; co.n = n; co.N = N; co.Np = p.Np; co.off_P = p.oP; co.off_P2 = r > 0 ? p.oP2 : -1;
  co.off_R = oRfin; co.off_B = p.oB; co.off_V = p.oV;
  if (p.refine) {
    const int rc = core_evd_refined<PR>(drecs, nrec, p, co, s);
    if (rc != KFB_OK) return rc;
  } else {
  if (p.pre) {
    // eigensolve of the new-direction block sqrt(w) R^T (same arithmetic, size n)
    UpdPlan pp = p;
    pp.N = n; pp.Np = p.preNp; pp.bw = p.prebw; pp.oB = p.oPB; pp.oV = p.oPV; pp.oCnt = p.oPCnt;
    CoreArgs cr;
    cr.r = 0; cr.n = n; cr.N = n; cr.Np = p.preNp; cr.off_P = p.oP; cr.off_P2 = -1;
    cr.off_R = oRfin; cr.off_B = p.oPB; cr.off_V = p.oPV;
    {
      StageTimer st_pc("core", s, 2);
      KFB_TRY((assemble_core<TC, TP, TG, TD>(drecs, nrec, cr, s)));
      KFB_TRY(zero_words(drecs, nrec, WS, p.oPCnt, MAX_SWEEPS, s));
    }
    const int rc = core_evd<PR>(drecs, nrec, pp, s, false, "jacobi_pre", PRE_SWEEPS);
    if (rc != KFB_OK) return rc;
    co.off_preB = p.oPB; co.off_preV = p.oPV; co.preNp = p.preNp;
  }
  {
    StageTimer st_core("core", s, 2);
    KFB_TRY((assemble_core<TC, TP, TG, TD>(drecs, nrec, co, s)));
    KFB_TRY(zero_words(drecs, nrec, WS, p.oCnt, MAX_SWEEPS, s));
  }
  {
    const int rc = core_evd<PR>(drecs, nrec, p, s);
    if (rc != KFB_OK) return rc;
  }
  }
  // rotation: U' = [U_r Q] W  (Algorithm 3), into the back buffer
  GemmArgs ro;
  ro.A = op(U_FRONT, 0, 1, ldu);
  ro.A.slot2 = WS; ro.A.off2 = oQ; ro.A.rs2 = 1; ro.A.cs2 = d; ro.A.split = r;
  if (r == 0) ro.A = op(WS, oQ, 1, d);
  ro.B = op(WS, p.oW, 1, N); ro.C = op(U_BACK, 0, 1, ldu);
  ro.m = (int)d; ro.n = N; ro.k = N;
  ro.aligned16 = (d % 4 == 0) && (N % 4 == 0);  // U, Q (ld d) and W (ld N) columns
  ro.c_vec = 1;                                  // the back buffer's columns (ldu: 256-byte multiples)
  StageTimer st_rot("rotate", s, 2);
  KFB_TRY((mm<PR, 1, TU, TW, TU, TU, TA>(drecs, nrec, ro, s)));
  // drift detector on the new basis (column norms)
  KFB_TRY((ortho_check<TU, TD>(drecs, nrec, U_BACK, D_BACK, d, ldu, N, drift_tol(PR), s)));
  return KFB_OK;
}

// ---------------------------------------------------------------------------
// Preconditioner plan (one layer)
// ---------------------------------------------------------------------------
struct PrePlan {
  int64_t dG, dA, lduG, lduA, ldg, lds;
  int aligned16;  // every G and S pointer 16-byte aligned and ldg, lds multiples of 4
  int NG, NA, ks3;
  int64_t oT1, oT2, oT3, oPart, ocG, ocA, oBeta;
  size_t per_problem;
};

template <int PR>
void make_pre_plan(int64_t dG, int64_t dA, int64_t lduG, int64_t lduA, int NG, int NA, int64_t ldg,
                   int64_t lds, int nrec, PrePlan* p) {
  typedef typename Ty<PR>::Acc TA;
  p->dG = dG; p->dA = dA; p->lduG = lduG; p->lduA = lduA; p->NG = NG; p->NA = NA;
  p->ldg = ldg; p->lds = lds;
  const int tiles = ((NG + 63) / 64) * ((NA + 63) / 64);  // own shape only
  int ks = 1;
  // T3's inner dimension: dA (T1 U_A), or dG in the mixed form (U_G^T T2)
  const int64_t k3 = PR == KFB_BF16_MIXED ? dG : dA;
  while (tiles * ks < 512 && (k3 / (ks * 2)) >= 256) ks *= 2;
  p->ks3 = ks;
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at_ = o; o = align256(o + bytes); return (int64_t)at_; };
  p->oT1 = take((size_t)NG * dA * sizeof(TA));
  p->oT2 = take((size_t)dG * NA * sizeof(TA));
  p->oT3 = take((size_t)NG * NA * sizeof(TA));
  p->oPart = take((size_t)ks * NG * NA * sizeof(TA));
  p->ocG = take((size_t)2 * NG * sizeof(TA));
  p->ocA = take((size_t)2 * NA * sizeof(TA) + 32);  // + the three doubles of precond_coefs
  p->oBeta = ((p->ocA + (int64_t)2 * NA * (int64_t)sizeof(TA)) + 7) & ~int64_t(7);
  p->per_problem = o;
}

template <int PR>
int run_precond(const Rec* drecs, int nrec, const PrePlan& p, uint32_t flags, hipStream_t s) {
  typedef Ty<PR> T;
  typedef typename T::U TU; typedef typename T::D TD; typedef typename T::Acc TA;
  typedef TA TGrad;  // G and S element type (FP64 form: double, else float)
  const int NG = p.NG, NA = p.NA;
  const int64_t dG = p.dG, dA = p.dA;
  std::unique_ptr<StageTimer> st_pre(new StageTimer("pre_coef_T1_T2_T3", s, 4 + (p.ks3 > 1 ? 1 : 0)));
  CoefArgs ca;
  ca.kG = NG; ca.kA = NA; ca.off_cG = p.ocG; ca.off_cA = p.ocA; ca.flags = flags;
  KFB_TRY((precond_coefs<TD, TA>(drecs, nrec, ca, s)));
  // Mixed form: the coefficient scalings of X1 and of T2 are folded into the
  // epilogues of the BF16 products (T1's rows, X2's C0 columns), so T3 is formed
  // from the unscaled T2 (U_G^T G U_A either way) and no separate pass rereads
  // T1 or T2.
  constexpr bool FOLD = PR == KFB_BF16_MIXED;
  // T1 = U_G^T G   (NG x dA, row-major; mixed form: X1 = diag(c_G / lam_A) T1)
  GemmArgs g1;
  g1.A = op(PU_G, 0, p.lduG, 1); g1.B = op(P_G, 0, p.ldg, 1); g1.C = op(PWS, p.oT1, dA, 1);
  g1.m = NG; g1.n = (int)dA; g1.k = (int)dG; g1.aligned16 = p.aligned16; g1.c_vec = 1;  // workspace
  if (FOLD) { g1.rsc_slot = PWS; g1.rsc_off = p.ocG; }
  KFB_TRY((mm<PR, 0, TU, TGrad, TA, TA, TA>(drecs, nrec, g1, s)));
  // T2 = G U_A     (dG x NA, column-major)
  GemmArgs g2;
  g2.A = op(P_G, 0, p.ldg, 1); g2.B = op(PU_A, 0, 1, p.lduA); g2.C = op(PWS, p.oT2, 1, dG);
  g2.m = (int)dG; g2.n = NA; g2.k = (int)dA; g2.aligned16 = p.aligned16; g2.c_vec = 1;  // workspace
  KFB_TRY((mm<PR, 0, TGrad, TU, TA, TA, TA>(drecs, nrec, g2, s)));
  // T3 = T1 U_A    (NG x NA); mixed form: U_G^T T2 (T1 already holds X1)
  GemmArgs g3;
  if (FOLD) {
    g3.A = op(PU_G, 0, p.lduG, 1); g3.B = op(PWS, p.oT2, 1, dG); g3.k = (int)dG;
  } else {
    g3.A = op(PWS, p.oT1, dA, 1); g3.B = op(PU_A, 0, 1, p.lduA); g3.k = (int)dA;
  }
  g3.C = op(PWS, p.oT3, 1, NG);
  g3.m = NG; g3.n = NA; g3.ksplit = p.ks3; g3.Part = op(PWS, p.oPart, 1, NG);
  g3.aligned16 = p.aligned16;  // T1 rows need dA % 4 == 0 as well (checked with the strides)
  KFB_TRY((mm<PR, 0, TA, TU, TA, TA, TA>(drecs, nrec, g3, s)));
  st_pre.reset(new StageTimer("pre_scale_X2", s, FOLD ? 2 : 4));
  // X1 = diag(c_G / lam_A) T1;  T2 <- T2 diag(c_A / lam_G);  T3 <- diag(c_G) T3 diag(c_A)
  if (!FOLD) {
    ScaleArgs s1;
    s1.m = NG; s1.n = (int)dA; s1.X = op(PWS, p.oT1, dA, 1); s1.row_slot = PWS; s1.row_off = p.ocG;
    s1.col_slot = -1; s1.col_off = 0; s1.extra_mode = 0;
    KFB_TRY((scale2d<TA, TA>(drecs, nrec, s1, s)));
    ScaleArgs s2;
    s2.m = (int)dG; s2.n = NA; s2.X = op(PWS, p.oT2, 1, dG); s2.row_slot = -1; s2.row_off = 0;
    s2.col_slot = PWS; s2.col_off = p.ocA; s2.extra_mode = 0;
    KFB_TRY((scale2d<TA, TA>(drecs, nrec, s2, s)));
  }
  ScaleArgs s3;
  s3.m = NG; s3.n = NA; s3.X = op(PWS, p.oT3, 1, NG); s3.row_slot = PWS;
  s3.row_off = p.ocG + (int64_t)NG * sizeof(TA); s3.col_slot = PWS;
  s3.col_off = p.ocA + (int64_t)NA * sizeof(TA); s3.extra_mode = 0;
  KFB_TRY((scale2d<TA, TA>(drecs, nrec, s3, s)));
  // X2 = T2 + U_G T3   (in place over T2)
  GemmArgs g4;
  g4.A = op(PU_G, 0, 1, p.lduG); g4.B = op(PWS, p.oT3, 1, NG); g4.C0 = op(PWS, p.oT2, 1, dG);
  g4.C = op(PWS, p.oT2, 1, dG); g4.m = (int)dG; g4.n = NA; g4.k = NG; g4.beta = 1.0;
  g4.aligned16 = p.aligned16;  // U_G columns (256-byte multiples) and the workspace blocks
  g4.c_vec = 1;                // T2 (C0 and C) in the workspace
  if (FOLD) { g4.c0cs_slot = PWS; g4.c0cs_off = p.ocA; }  // X2 = T2 diag(c_A / lam_G) + U_G T3
  KFB_TRY((mm<PR, 0, TU, TA, TA, TA, TA>(drecs, nrec, g4, s)));
  st_pre.reset();
  StageTimer st_s("pre_S", s, 1);
  // S = G / (lam_G lam_A) + [U_G | X2] [X1 ; U_A^T]
  GemmArgs g5;
  g5.A = op(PU_G, 0, 1, p.lduG);
  g5.A.slot2 = PWS; g5.A.off2 = p.oT2; g5.A.rs2 = 1; g5.A.cs2 = dG; g5.A.split = NG;
  g5.B = op(PWS, p.oT1, dA, 1);
  g5.B.slot2 = PU_A; g5.B.off2 = 0; g5.B.rs2 = p.lduA; g5.B.cs2 = 1; g5.B.split = NG;
  g5.C0 = op(P_G, 0, p.ldg, 1); g5.beta_slot = PWS; g5.beta_off = p.oBeta;
  g5.C = op(P_S, 0, p.lds, 1);
  g5.m = (int)dG; g5.n = (int)dA; g5.k = NG + NA; g5.aligned16 = p.aligned16;
  g5.c_vec = p.aligned16;  // S and G pointers 16-byte aligned, lds and ldg multiples of 4
  KFB_TRY((mm<PR, 0, TU, TA, TGrad, TGrad, TA>(drecs, nrec, g5, s)));
  return KFB_OK;
}

// ---------------------------------------------------------------------------
// Factored preconditioner (Algorithm 8): per-side inverse applied to the thin
// factors G_k (dG x n) and A_k (dA x n), then S = Y_G Y_A^T.
// ---------------------------------------------------------------------------
struct FacPlan {
  int64_t dG, dA, lduG, lduA, ldgk, ldak, lds;
  int NG, NA, n, ksG, ksA, aligned16;
  int64_t ocG, ocA, oBeta, oTG, oTA, oPart, oYG, oYA;
  size_t per_problem;
};

template <int PR>
void make_fac_plan(int64_t dG, int64_t dA, int64_t lduG, int64_t lduA, int NG, int NA, int n, FacPlan* p) {
  typedef typename Ty<PR>::Acc TA;
  p->dG = dG; p->dA = dA; p->lduG = lduG; p->lduA = lduA; p->NG = NG; p->NA = NA; p->n = n;
  auto ks_for = [&](int m, int nn, int64_t k) {  // the problem's own shape only
    const int tiles = ((m + 63) / 64) * ((nn + 63) / 64);
    int ks = 1;
    while (tiles * ks < 512 && (k / (ks * 2)) >= 256) ks *= 2;
    return ks;
  };
  p->ksG = ks_for(NG, n, dG);
  p->ksA = ks_for(NA, n, dA);
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at_ = o; o = align256(o + bytes); return (int64_t)at_; };
  p->ocG = take((size_t)2 * NG * sizeof(TA));
  p->ocA = take((size_t)2 * NA * sizeof(TA) + 32);
  p->oBeta = ((p->ocA + (int64_t)2 * NA * (int64_t)sizeof(TA)) + 7) & ~int64_t(7);
  p->oTG = take((size_t)NG * n * sizeof(TA));
  p->oTA = take((size_t)NA * n * sizeof(TA));
  const size_t pg = (size_t)p->ksG * NG * n, pa = (size_t)p->ksA * NA * n;
  p->oPart = take((pg > pa ? pg : pa) * sizeof(TA));
  p->oYG = take((size_t)dG * n * sizeof(TA));
  p->oYA = take((size_t)dA * n * sizeof(TA));
  p->per_problem = o;
}

template <int PR>
int run_fac(const Rec* drecs, int nrec, const FacPlan& p, uint32_t flags, hipStream_t s) {
  typedef Ty<PR> T;
  typedef typename T::U TU; typedef typename T::M TM; typedef typename T::D TD; typedef typename T::Acc TA;
  typedef TA TGrad;  // S element type
  const int n = p.n;
  {
    StageTimer st_side("fac_sides", s, 7 + (p.ksG > 1 ? 1 : 0) + (p.ksA > 1 ? 1 : 0));
    CoefArgs ca;
    ca.kG = p.NG; ca.kA = p.NA; ca.off_cG = p.ocG; ca.off_cA = p.ocA; ca.flags = flags;
    KFB_TRY((precond_coefs<TD, TA>(drecs, nrec, ca, s)));
    for (int side = 0; side < 2; ++side) {
      const int slotU = side ? PU_A : PU_G, slotX = side ? P_AK : P_G;
      const int64_t d = side ? p.dA : p.dG, ldu = side ? p.lduA : p.lduG, ldx = side ? p.ldak : p.ldgk;
      const int N = side ? p.NA : p.NG, ks = side ? p.ksA : p.ksG;
      const int64_t oT = side ? p.oTA : p.oTG, oY = side ? p.oYA : p.oYG;
      const int64_t oc = side ? p.ocA : p.ocG;
      // T = U^T X   (N x n)
      GemmArgs g;
      g.A = op(slotU, 0, ldu, 1); g.B = op(slotX, 0, 1, ldx); g.C = op(PWS, oT, 1, N);
      g.m = N; g.n = n; g.k = (int)d; g.ksplit = ks; g.Part = op(PWS, p.oPart, 1, N);
      KFB_TRY((mm<PR, 1, TU, TM, TA, TA, TA>(drecs, nrec, g, s)));
      // T <- diag(c) T
      ScaleArgs sc;
      sc.m = N; sc.n = n; sc.X = op(PWS, oT, 1, N); sc.row_slot = PWS; sc.row_off = oc + (int64_t)N * sizeof(TA);
      sc.col_slot = -1; sc.col_off = 0; sc.extra_mode = 0;
      KFB_TRY((scale2d<TA, TA>(drecs, nrec, sc, s)));
      // Y = X / lam + U T
      GemmArgs y;
      y.A = op(slotU, 0, 1, ldu); y.B = op(PWS, oT, 1, N); y.C0 = op(slotX, 0, 1, ldx);
      y.beta_slot = PWS; y.beta_off = p.oBeta + (side ? 16 : 8);
      y.C = op(PWS, oY, 1, d); y.m = (int)d; y.n = n; y.k = N;
      // the vector loads touch only A (a state's U, 256-byte aligned columns) and
      // B (workspace); C0 and C are read and written element by element
      y.aligned16 = 1;
      KFB_TRY((mm<PR, 1, TU, TA, TA, TM, TA>(drecs, nrec, y, s)));
    }
  }
  StageTimer st_s("fac_S", s, 1);
  // S = Y_G Y_A^T   (dG x dA row-major, inner dimension n)
  GemmArgs g5;
  g5.A = op(PWS, p.oYG, 1, p.dG); g5.B = op(PWS, p.oYA, p.dA, 1); g5.C = op(P_S, 0, p.lds, 1);
  g5.m = (int)p.dG; g5.n = (int)p.dA; g5.k = n; g5.aligned16 = p.aligned16; g5.c_vec = p.aligned16;
  KFB_TRY((mm<PR, 0, TA, TA, TGrad, TGrad, TA>(drecs, nrec, g5, s)));
  return KFB_OK;
}

// ---------------------------------------------------------------------------
// B-R-KFAC (Algorithm 5): dense EA factor and the randomized-SVD overwrite
// ---------------------------------------------------------------------------
// X = beta X + alpha M M^T   (X: d x d column-major; M: d x n batch)
template <int PR>
int run_dense(const Rec* drecs, int64_t d, int64_t ldx, int64_t ldm, int n, double alpha, double beta,
              hipStream_t s) {
  typedef Ty<PR> T;
  typedef typename T::U TX; typedef typename T::M TM; typedef typename T::Acc TA;
  GemmArgs g;
  g.A = op(M_IN, 0, 1, ldm); g.B = op(M_IN, 0, ldm, 1);
  g.C0 = op(B_X, 0, 1, ldx); g.C = op(B_X, 0, 1, ldx);
  g.m = (int)d; g.n = (int)d; g.k = n; g.alpha = alpha; g.beta = beta;
  StageTimer st("dense_ea", s, 1);
  if constexpr (PR == KFB_BF16_MIXED) {
    KFB_TRY((gemm_bf16<TM, TM, TX, TX, 0>(drecs, 1, g, s)));
  } else {
    KFB_TRY((gemm<TM, TM, TX, TX, TA>(drecs, 1, g, s)));
  }
  return KFB_OK;
}

// Randomized SVD of X truncated to r, written into the back buffers:
//   Y = X Omega;  q times { Q = qr(Y); Y = X^T Q; Q = qr(Y); Y = X Q };  Q = qr(Y);
//   B = Q^T X = Y'^T with Y' = X^T Q = Q' R';  the left singular vectors of B are
//   the eigenvectors of R'^T R' (the Jacobi core with square factor R'), the
//   singular values the square roots of its eigenvalues;  U = Q W[:, :r].
template <int PR>
int run_rsvd(const Rec* drecs, const UpdPlan& p, int64_t oZc, int r, int64_t ldx, int64_t ldo, int power_its,
             hipStream_t s) {
  typedef Ty<PR> T;
  typedef typename T::U TU; typedef typename T::Z TZ; typedef typename T::P TP; typedef typename T::G TG;
  typedef typename T::Core TC; typedef typename T::W TW; typedef typename T::D TD; typedef typename T::Acc TA;
  const int64_t d = p.d;
  const int l = p.n;
  int64_t oQ = -1, oR = -1;
  // the three d x l buffers: the product lands in one not holding Q
  const int64_t bufs[3] = {p.oZ, p.oZb, oZc};
  auto product = [&](bool transposed, int64_t src, int64_t dst, bool omega) -> int {
    GemmArgs g;
    g.A = transposed ? op(B_X, 0, ldx, 1) : op(B_X, 0, 1, ldx);
    g.B = omega ? op(B_OMEGA, 0, 1, ldo) : op(WS, src, 1, d);
    g.C = op(WS, dst, 1, d);
    g.m = (int)d; g.n = l; g.k = (int)d;
    KFB_TRY((mm<PR, 1, TU, TU, TZ, TZ, TA>(drecs, 1, g, s)));
    return KFB_OK;
  };
  auto other = [&](int64_t a, int64_t b) {
    for (int i = 0; i < 3; ++i)
      if (bufs[i] != a && bufs[i] != b) return bufs[i];
    return bufs[0];
  };
  auto qr = [&](int64_t y, int64_t keep) -> int {
    // factor Y (at y) using the buffer not holding `keep` as the second one
    return thin_qr<PR>(drecs, 1, p, y, other(y, keep), &oQ, &oR, s);
  };
  {
    StageTimer st("rsvd_range", s, 1);
    int rc = product(false, 0, p.oZ, true);
    if (rc != KFB_OK) return rc;
    if ((rc = qr(p.oZ, -1)) != KFB_OK) return rc;
    for (int it = 0; it < power_its; ++it) {
      for (int half = 0; half < 2; ++half) {
        const int64_t y = other(oQ, -1);
        if ((rc = product(half == 0, oQ, y, false)) != KFB_OK) return rc;
        if ((rc = qr(y, -1)) != KFB_OK) return rc;
      }
    }
    // Y' = X^T Q and its R' (Q kept)
    const int64_t Qfin = oQ;
    const int64_t y = other(Qfin, -1);
    if ((rc = product(true, Qfin, y, false)) != KFB_OK) return rc;
    if ((rc = qr(y, Qfin)) != KFB_OK) return rc;
    oQ = Qfin;
  }
  // core: B_jac = R' (assemble_core forms the transpose of its square factor, so
  // it is handed R'^T), V = I
  CoreArgs co;
  co.r = 0; co.n = l; co.N = l; co.Np = p.Np; co.off_P = p.oP; co.off_P2 = -1;
  co.off_R = p.oX1; co.off_B = p.oB; co.off_V = p.oV;
  {
    StageTimer st("core", s, 3);
    KFB_TRY((copy2d<TG, TG>(drecs, 1, op(WS, p.oX1, 1, l), op(WS, oR, l, 1), l, l, s)));
    KFB_TRY((assemble_core<TC, TP, TG, TD>(drecs, 1, co, s)));
    KFB_TRY(zero_words(drecs, 1, WS, p.oCnt, MAX_SWEEPS, s));
  }
  {
    const int rc = core_evd<PR>(drecs, 1, p, s);
    if (rc != KFB_OK) return rc;
  }
  StageTimer st("rsvd_rotate", s, 2);
  KFB_TRY(sqrt_prefix<TD>(drecs, 1, D_BACK, 0, r, s));
  GemmArgs ro;
  ro.A = op(WS, oQ, 1, d); ro.B = op(WS, p.oW, 1, l); ro.C = op(U_BACK, 0, 1, p.ldu);
  ro.m = (int)d; ro.n = r; ro.k = l;
  KFB_TRY((mm<PR, 1, TZ, TW, TU, TU, TA>(drecs, 1, ro, s)));
  return KFB_OK;
}

// Light correction (Algorithm 6) of k modes on the chosen columns:
//   U_c = U[:, idx];  M_S = U_c^T X U_c;  M_S = W L W^T;  U[:, idx] = U_c W,
//   D[idx] = L;  modes re-sorted descending into the back buffers.
// The small symmetric EVD runs as the core eigensolver on the Cholesky factor
// R of M_S (M_S = R^T R), whose square factor's Gram it diagonalises.
struct CorrPlan {
  UpdPlan p;      // n = n_crc: U_c (oZ), X U_c (oZb), M_S (oGram), Cholesky, core
  int64_t oUcw, oIdx, oSrc;
  size_t per_problem;
};

template <int PR>
int run_correct(const Rec* drecs, const CorrPlan& cp, int k, int64_t ldx, hipStream_t s) {
  typedef Ty<PR> T;
  typedef typename T::U TU; typedef typename T::Z TZ; typedef typename T::P TP; typedef typename T::G TG;
  typedef typename T::Core TC; typedef typename T::W TW; typedef typename T::D TD; typedef typename T::Acc TA;
  const UpdPlan& p = cp.p;
  const int64_t d = p.d;
  const int nc = p.n;
  {
    StageTimer st("correct_project", s, 4);
    GatherArgs ga;
    ga.src_slot = U_FRONT; ga.lds = p.ldu; ga.d = d; ga.n = nc; ga.off_idx = cp.oIdx; ga.off_dst = p.oZ;
    KFB_TRY(gather_cols<TU>(drecs, 1, ga, s));
    // X U_c
    GemmArgs g;
    g.A = op(B_X, 0, 1, ldx); g.B = op(WS, p.oZ, 1, d); g.C = op(WS, p.oZb, 1, d);
    g.m = (int)d; g.n = nc; g.k = (int)d;
    KFB_TRY((mm<PR, 1, TU, TU, TZ, TZ, TA>(drecs, 1, g, s)));
    // M_S = U_c^T (X U_c), accumulated in the Gram type
    GemmArgs gs;
    gs.A = op(WS, p.oZ, d, 1); gs.B = op(WS, p.oZb, 1, d); gs.C = op(WS, p.oGram, 1, nc);
    gs.m = nc; gs.n = nc; gs.k = (int)d; gs.ksplit = p.ksG; gs.Part = op(WS, p.oPart, 1, nc);
    KFB_TRY((gemm<TZ, TZ, TG, TG, TG>(drecs, 1, gs, s)));
  }
  {
    StageTimer st("core", s, 4);
    CholArgs ca;
    const double ueps = sizeof(TG) == 4 ? 1.1920929e-07 : 2.220446049250313e-16;
    ca.n = nc; ca.off_gram = p.oGram; ca.off_R = p.oR1; ca.off_Rinv = p.oX2; ca.off_rowbuf = 0;
    ca.tau_rel = 64.0 * ueps; ca.shift_rel = 0.0;
    KFB_TRY(chol_inv<TG>(drecs, 1, ca, s));
    KFB_TRY((copy2d<TG, TG>(drecs, 1, op(WS, p.oX1, 1, nc), op(WS, p.oR1, nc, 1), nc, nc, s)));
    CoreArgs co;
    co.r = 0; co.n = nc; co.N = nc; co.Np = p.Np; co.off_P = p.oP; co.off_P2 = -1;
    co.off_R = p.oX1; co.off_B = p.oB; co.off_V = p.oV;
    KFB_TRY((assemble_core<TC, TP, TG, TD>(drecs, 1, co, s)));
    KFB_TRY(zero_words(drecs, 1, WS, p.oCnt, MAX_SWEEPS, s));
  }
  {
    const int rc = core_evd<PR>(drecs, 1, p, s);
    if (rc != KFB_OK) return rc;
  }
  StageTimer st("correct_write", s, 3);
  // U_c W, then the merged, re-sorted modes into the back buffers
  GemmArgs ro;
  ro.A = op(WS, p.oZ, 1, d); ro.B = op(WS, p.oW, 1, nc); ro.C = op(WS, cp.oUcw, 1, d);
  ro.m = (int)d; ro.n = nc; ro.k = nc;
  KFB_TRY((mm<PR, 1, TZ, TW, TZ, TZ, TA>(drecs, 1, ro, s)));
  MergeArgs ma;
  ma.k = k; ma.n_crc = nc; ma.off_lam = p.oLam; ma.off_idx = cp.oIdx; ma.off_src = cp.oSrc;
  KFB_TRY((correct_merge<TC, TD>(drecs, 1, ma, s)));
  PermuteArgs pa;
  pa.d = d; pa.ldu = p.ldu; pa.k = k; pa.off_src = cp.oSrc; pa.off_ucw = cp.oUcw;
  KFB_TRY(correct_permute<TU>(drecs, 1, pa, s));
  return KFB_OK;
}

// Re-orthonormalisation of a representation whose basis has drifted
// (Rayleigh-Ritz on its own span): U = Q R by CholeskyQR, so that
// U D U^T = Q (R D R^T) Q^T; the k x k core R D R^T, with the square factor
// R diag(sqrt(D)), goes through the core eigensolver, W Lambda W^T, and the
// state becomes (Q W, Lambda): the same matrix on an orthonormal basis.
template <int PR>
int run_reorth(const Rec* drecs, const UpdPlan& p, int64_t oDs, hipStream_t s) {
  typedef Ty<PR> T;
  typedef typename T::U TU; typedef typename T::Z TZ; typedef typename T::P TP; typedef typename T::G TG;
  typedef typename T::Core TC; typedef typename T::W TW; typedef typename T::D TD; typedef typename T::Acc TA;
  const int64_t d = p.d;
  const int k = p.n;
  int64_t oQ, oR;
  {
    StageTimer st("reorth_qr", s, 3 + thin_qr_launches(PR, p.ksG));
    KFB_TRY((copy2d<TZ, TU>(drecs, 1, op(WS, p.oZ, 1, d), op(U_FRONT, 0, 1, p.ldu), (int)d, k, s)));
    const int rc = thin_qr<PR>(drecs, 1, p, p.oZ, p.oZb, &oQ, &oR, s);
    if (rc != KFB_OK) return rc;
    // R <- R diag(sqrt(D))
    KFB_TRY((copy2d<TG, TD>(drecs, 1, op(WS, oDs, 1, k), op(D_FRONT, 0, 1, k), k, 1, s)));
    KFB_TRY(sqrt_prefix<TG>(drecs, 1, WS, oDs, k, s));
    ScaleArgs sc;
    sc.m = k; sc.n = k; sc.X = op(WS, oR, 1, k); sc.row_slot = -1; sc.row_off = 0;
    sc.col_slot = WS; sc.col_off = oDs; sc.extra_mode = 0;
    KFB_TRY((scale2d<TG, TG>(drecs, 1, sc, s)));
  }
  CoreArgs co;
  co.r = 0; co.n = k; co.N = k; co.Np = p.Np; co.off_P = p.oP; co.off_P2 = -1;
  co.off_R = oR; co.off_B = p.oB; co.off_V = p.oV;
  {
    StageTimer st("core", s, 2);
    KFB_TRY((assemble_core<TC, TP, TG, TD>(drecs, 1, co, s)));
    KFB_TRY(zero_words(drecs, 1, WS, p.oCnt, MAX_SWEEPS, s));
  }
  {
    const int rc = core_evd<PR>(drecs, 1, p, s);
    if (rc != KFB_OK) return rc;
  }
  StageTimer st("reorth_rotate", s, 2);
  GemmArgs ro;
  ro.A = op(WS, oQ, 1, d); ro.B = op(WS, p.oW, 1, k); ro.C = op(U_BACK, 0, 1, p.ldu);
  ro.m = (int)d; ro.n = k; ro.k = k;
  KFB_TRY((mm<PR, 1, TZ, TW, TU, TU, TA>(drecs, 1, ro, s)));
  KFB_TRY((ortho_check<TU, TD>(drecs, 1, U_BACK, D_BACK, d, p.ldu, k, drift_tol(PR), s)));
  return KFB_OK;
}

int dispatch_reorth(kfb_state_t st, void* workspace, size_t ws_bytes, hipStream_t s, size_t* need_only) {
  if (!st) return KFB_EINVAL;
  const int k = st->k_valid;
  if (k <= 0) return KFB_EEMPTY;
  if (k > MAX_QR_COLS) return KFB_EINVAL;
  UpdPlan p;
  bool ok = false;
  if (st->prec == KFB_FP64) ok = make_upd_plan<KFB_FP64>(st->d, st->ldu, st->d, 0, k, 1, &p);
  else if (st->prec == KFB_FP32) ok = make_upd_plan<KFB_FP32>(st->d, st->ldu, st->d, 0, k, 1, &p);
  else ok = make_upd_plan<KFB_BF16_MIXED>(st->d, st->ldu, st->d, 0, k, 1, &p);
  if (!ok) return KFB_EINVAL;
  const int64_t oDs = (int64_t)p.per_problem;  // sqrt(D) in the Gram type (8 bytes suffice for all forms)
  const size_t head = align256(sizeof(Rec));
  const size_t need = head + p.per_problem + align256((size_t)k * 8);
  if (need_only) { *need_only = need; return KFB_OK; }
  if (!workspace) return KFB_EINVAL;
  if (ws_bytes < need) return KFB_EWORKSPACE;
  if (((uintptr_t)workspace) & 255) return KFB_EINVAL;
  Rec host;
  memset(&host, 0, sizeof(Rec));
  host.p[U_FRONT] = st->buf + st->off_U[st->front];
  host.p[U_BACK] = st->buf + st->off_U[1 - st->front];
  host.p[WS] = (char*)workspace + head;
  host.p[D_FRONT] = st->buf + st->off_D[st->front];
  host.p[D_BACK] = st->buf + st->off_D[1 - st->front];
  host.p[STATUS] = st->buf + st->off_status;
  host.s[0] = 0.0;  // the core is the square factor alone: no decayed modes,
  host.s[1] = 1.0;  // unit weight
  Rec* dev = (Rec*)workspace;
  if (upload_recs(&host, 1, dev, s) != hipSuccess) return KFB_EHIP;
  int rc;
  if (st->prec == KFB_FP64) rc = run_reorth<KFB_FP64>(dev, p, oDs, s);
  else if (st->prec == KFB_FP32) rc = run_reorth<KFB_FP32>(dev, p, oDs, s);
  else rc = run_reorth<KFB_BF16_MIXED>(dev, p, oDs, s);
  if (rc != KFB_OK) return rc;
  st->front = 1 - st->front;
  return KFB_OK;
}

inline int upd_r_eff(kfb_state_t st) { return st->k_valid < st->r ? st->k_valid : st->r; }

int dispatch_update(int count, kfb_state_t const* sts, const void* const* Ms, int64_t ldm, int32_t n,
                    void* workspace, size_t ws_bytes, hipStream_t s, size_t* need_only,
                    const int32_t* widths = nullptr) {
  if (count <= 0 || !sts) return KFB_EINVAL;
  kfb_state_t s0 = sts[0];
  if (!s0) return KFB_EINVAL;
  const int prec = s0->prec;
  const int r_eff = upd_r_eff(s0);
  if (n <= 0 || n > s0->n_max || ldm < s0->d) return KFB_EINVAL;
  for (int i = 0; i < count; ++i) {
    kfb_state_t st = sts[i];
    if (!st) return KFB_EINVAL;
    if (st->prec != prec || st->d != s0->d || st->r != s0->r || upd_r_eff(st) != r_eff ||
        n > st->n_max || st->ldu != s0->ldu)
      return KFB_ESTATE;
    for (int j = 0; j < i; ++j)
      if (sts[j] == st) return KFB_ESTATE;
  }
  UpdPlan p;
  bool ok = false;
  if (prec == KFB_FP64) ok = make_upd_plan<KFB_FP64>(s0->d, s0->ldu, ldm, r_eff, n, count, &p);
  else if (prec == KFB_FP32) ok = make_upd_plan<KFB_FP32>(s0->d, s0->ldu, ldm, r_eff, n, count, &p);
  else ok = make_upd_plan<KFB_BF16_MIXED>(s0->d, s0->ldu, ldm, r_eff, n, count, &p);
  if (!ok) return KFB_EINVAL;
  const size_t head = align256(sizeof(Rec) * (size_t)count);
  const size_t need = head + p.per_problem * (size_t)count;
  if (need_only) { *need_only = need; return KFB_OK; }
  if (!Ms || !workspace) return KFB_EINVAL;
  if (ws_bytes < need) return KFB_EWORKSPACE;
  if (((uintptr_t)workspace) & 255) return KFB_EINVAL;
  if (widths)
    for (int i = 0; i < count; ++i)
      if (widths[i] < 1 || widths[i] > n) return KFB_EINVAL;
  Rec* host = (Rec*)malloc(sizeof(Rec) * (size_t)count);
  if (!host) return KFB_EINVAL;
  for (int i = 0; i < count; ++i) {
    if (!Ms[i]) { free(host); return KFB_EINVAL; }
    kfb_state_t st = sts[i];
    Rec* rc = &host[i];
    memset(rc, 0, sizeof(Rec));
    rc->p[U_FRONT] = st->buf + st->off_U[st->front];
    rc->p[U_BACK] = st->buf + st->off_U[1 - st->front];
    rc->p[M_IN] = const_cast<void*>(Ms[i]);
    rc->p[WS] = (char*)workspace + head + p.per_problem * (size_t)i;
    rc->p[D_FRONT] = st->buf + st->off_D[st->front];
    rc->p[D_BACK] = st->buf + st->off_D[1 - st->front];
    rc->p[STATUS] = st->buf + st->off_status;
    const int nw = widths ? widths[i] : n;                  // the batch's own width
    rc->s[0] = st->k_valid > 0 ? st->rho : 0.0;           // decay applied to the kept modes
    rc->s[1] = st->k_valid > 0 ? (1.0 - st->rho) / nw : 1.0 / nw;  // batch weight w
    rc->s[2] = widths ? (double)nw : 0.0;                 // columns >= nw are zero padding
  }
  Rec* dev = (Rec*)workspace;
  hipError_t he = upload_recs(host, count, dev, s);
  free(host);
  if (he != hipSuccess) return KFB_EHIP;
  int rc;
  if (prec == KFB_FP64) rc = run_update<KFB_FP64>(dev, count, p, s);
  else if (prec == KFB_FP32) rc = run_update<KFB_FP32>(dev, count, p, s);
  else rc = run_update<KFB_BF16_MIXED>(dev, count, p, s);
  if (rc != KFB_OK) return rc;
  for (int i = 0; i < count; ++i) {
    kfb_state_t st = sts[i];
    st->front = 1 - st->front;
    int64_t kv = (int64_t)r_eff + n;
    if (kv > st->d) kv = st->d;
    st->k_valid = (int32_t)kv;
    st->step += 1;
  }
  return KFB_OK;
}

// Cross-shape grouped update: states of one precision form and one kept rank
// r_eff but different widths d_i, batches of different widths n_i.  Every
// problem runs at the group's shape (dp = max d_i rounded up to 64, n = max
// n_i): its U and batch are copied into zero-padded workspace buffers, the
// update runs on them (zero rows stay zero through every stage: projection,
// residual, CholeskyQR Gram, rotation), and the first d_i rows of the new basis
// are copied into the state's back buffer.  The zero columns of a narrower
// batch are the padding of kfb_brand_update_batched_widths.
template <int PR>
int run_update_cross(const Rec* drecs, int nrec, const UpdPlan& p, hipStream_t s) {
  typedef Ty<PR> T;
  {
    StageTimer st("pad", s, 1);
    KFB_TRY((pad_in<typename T::U, typename T::M>(drecs, nrec, p.d, p.r, p.n, s)));
  }
  const int rc = run_update<PR>(drecs, nrec, p, s);
  if (rc != KFB_OK) return rc;
  StageTimer st("pad", s, 1);
  KFB_TRY((crop_out<typename T::U>(drecs, nrec, p.d, p.N, s)));
  return KFB_OK;
}

int dispatch_update_cross(int count, kfb_state_t const* sts, const void* const* Ms, const int64_t* ldms,
                          const int32_t* widths, void* workspace, size_t ws_bytes, hipStream_t s,
                          size_t* need_only) {
  if (count <= 0 || !sts || !widths || !sts[0]) return KFB_EINVAL;
  const int prec = sts[0]->prec;
  const int r_eff = upd_r_eff(sts[0]);
  int64_t dmax = 0;
  int n = 0, nmax_min = 1 << 30;
  for (int i = 0; i < count; ++i) {
    kfb_state_t st = sts[i];
    if (!st) return KFB_EINVAL;
    if (st->prec != prec || upd_r_eff(st) != r_eff) return KFB_ESTATE;
    for (int j = 0; j < i; ++j)
      if (sts[j] == st) return KFB_ESTATE;
    if (widths[i] < 1 || widths[i] > st->n_max) return KFB_EINVAL;
    if (st->d > dmax) dmax = st->d;
    if (widths[i] > n) n = widths[i];
    if (st->n_max < nmax_min) nmax_min = st->n_max;
  }
  // every state holds r_eff + n modes afterwards: n must fit each state's capacity
  if (n > nmax_min) return KFB_EINVAL;
  const int64_t dp = ((dmax + 63) / 64) * 64;
  UpdPlan p;
  bool ok = false;
  if (prec == KFB_FP64) ok = make_upd_plan<KFB_FP64>(dp, dp, dp, r_eff, n, count, &p);
  else if (prec == KFB_FP32) ok = make_upd_plan<KFB_FP32>(dp, dp, dp, r_eff, n, count, &p);
  else ok = make_upd_plan<KFB_BF16_MIXED>(dp, dp, dp, r_eff, n, count, &p);
  if (!ok) return KFB_EINVAL;
  // the padded copies after the update's own workspace
  const int64_t oUin = (int64_t)p.per_problem;
  const int64_t oMin = oUin + (int64_t)align256((size_t)dp * (r_eff > 0 ? r_eff : 1) * u_elem(prec));
  const int64_t oUout = oMin + (int64_t)align256((size_t)dp * n * m_elem(prec));
  const size_t per = (size_t)oUout + align256((size_t)dp * p.N * u_elem(prec));
  const size_t head = align256(sizeof(Rec) * (size_t)count);
  const size_t need = head + per * (size_t)count;
  if (need_only) { *need_only = need; return KFB_OK; }
  if (!Ms || !ldms || !workspace) return KFB_EINVAL;
  if (ws_bytes < need) return KFB_EWORKSPACE;
  if (((uintptr_t)workspace) & 255) return KFB_EINVAL;
  for (int i = 0; i < count; ++i)
    if (!Ms[i] || ldms[i] < sts[i]->d) return KFB_EINVAL;
  std::vector<Rec> host((size_t)count);
  for (int i = 0; i < count; ++i) {
    kfb_state_t st = sts[i];
    Rec* rc = &host[(size_t)i];
    memset(rc, 0, sizeof(Rec));
    char* ws = (char*)workspace + head + per * (size_t)i;
    rc->p[WS] = ws;
    rc->p[U_FRONT] = ws + oUin;
    rc->p[M_IN] = ws + oMin;
    rc->p[U_BACK] = ws + oUout;
    rc->p[D_FRONT] = st->buf + st->off_D[st->front];
    rc->p[D_BACK] = st->buf + st->off_D[1 - st->front];
    rc->p[STATUS] = st->buf + st->off_status;
    rc->p[X_UF] = st->buf + st->off_U[st->front];
    rc->p[X_M] = const_cast<void*>(Ms[i]);
    rc->p[X_UB] = st->buf + st->off_U[1 - st->front];
    const int nw = widths[i];
    rc->s[0] = st->k_valid > 0 ? st->rho : 0.0;
    rc->s[1] = st->k_valid > 0 ? (1.0 - st->rho) / nw : 1.0 / nw;
    rc->s[2] = (double)nw;
    rc->z[0] = st->d;
    rc->z[1] = st->ldu;
    rc->z[2] = ldms[i];
  }
  Rec* dev = (Rec*)workspace;
  if (upload_recs(host.data(), count, dev, s) != hipSuccess) return KFB_EHIP;
  int rc;
  if (prec == KFB_FP64) rc = run_update_cross<KFB_FP64>(dev, count, p, s);
  else if (prec == KFB_FP32) rc = run_update_cross<KFB_FP32>(dev, count, p, s);
  else rc = run_update_cross<KFB_BF16_MIXED>(dev, count, p, s);
  if (rc != KFB_OK) return rc;
  for (int i = 0; i < count; ++i) {
    kfb_state_t st = sts[i];
    st->front = 1 - st->front;
    st->k_valid = r_eff + n;   // <= r + n_max <= d; the padded modes are empty slots
    st->step += 1;
  }
  return KFB_OK;
}

int pre_modes(kfb_state_t st, uint32_t flags) {
  int k = st->k_valid;
  if ((flags & KFB_TRUNCATE_AFTER) && k > st->r) k = st->r;
  return k;
}

int dispatch_precond(int count, kfb_state_t const* stG, kfb_state_t const* stA, const void* const* G,
                     int64_t ldg, void* const* S, int64_t lds, const double* lamG, const double* lamA,
                     uint32_t flags, void* workspace, size_t ws_bytes, hipStream_t s, size_t* need_only) {
  if (count <= 0 || !stG || !stA) return KFB_EINVAL;
  kfb_state_t g0 = stG[0], a0 = stA[0];
  if (!g0 || !a0) return KFB_EINVAL;
  const int prec = g0->prec;
  const int NG = pre_modes(g0, flags), NA = pre_modes(a0, flags);
  for (int i = 0; i < count; ++i) {
    kfb_state_t g = stG[i], a = stA[i];
    if (!g || !a) return KFB_EINVAL;
    if (g == a) return KFB_ESTATE;
    if (g->prec != prec || a->prec != prec || g->d != g0->d || a->d != a0->d ||
        pre_modes(g, flags) != NG || pre_modes(a, flags) != NA || g->ldu != g0->ldu || a->ldu != a0->ldu)
      return KFB_ESTATE;
  }
  if (NG <= 0 || NA <= 0) return KFB_EEMPTY;
  if (ldg < a0->d || lds < a0->d) return KFB_EINVAL;
  PrePlan p;
  if (prec == KFB_FP64) make_pre_plan<KFB_FP64>(g0->d, a0->d, g0->ldu, a0->ldu, NG, NA, ldg, lds, count, &p);
  else if (prec == KFB_FP32) make_pre_plan<KFB_FP32>(g0->d, a0->d, g0->ldu, a0->ldu, NG, NA, ldg, lds, count, &p);
  else make_pre_plan<KFB_BF16_MIXED>(g0->d, a0->d, g0->ldu, a0->ldu, NG, NA, ldg, lds, count, &p);
  const size_t head = align256(sizeof(Rec) * (size_t)count);
  const size_t need = head + p.per_problem * (size_t)count;
  if (need_only) { *need_only = need; return KFB_OK; }
  if (!G || !S || !workspace || !lamG || !lamA) return KFB_EINVAL;
  if (ws_bytes < need) return KFB_EWORKSPACE;
  if (((uintptr_t)workspace) & 255) return KFB_EINVAL;
  Rec* host = (Rec*)malloc(sizeof(Rec) * (size_t)count);
  if (!host) return KFB_EINVAL;
  p.aligned16 = (ldg % 4 == 0) && (lds % 4 == 0);
  for (int i = 0; i < count; ++i) {
    if (!G[i] || !S[i] || G[i] == S[i] || !(lamG[i] > 0.0) || !(lamA[i] > 0.0)) { free(host); return KFB_EINVAL; }
    if ((((uintptr_t)G[i]) | ((uintptr_t)S[i])) & 15) p.aligned16 = 0;
    kfb_state_t g = stG[i], a = stA[i];
    Rec* rc = &host[i];
    memset(rc, 0, sizeof(Rec));
    rc->p[PU_G] = g->buf + g->off_U[g->front];
    rc->p[PD_G] = g->buf + g->off_D[g->front];
    rc->p[PU_A] = a->buf + a->off_U[a->front];
    rc->p[PD_A] = a->buf + a->off_D[a->front];
    rc->p[P_G] = const_cast<void*>(G[i]);
    rc->p[P_S] = S[i];
    rc->p[PWS] = (char*)workspace + head + p.per_problem * (size_t)i;
    rc->s[0] = lamG[i];
    rc->s[1] = lamA[i];
  }
  Rec* dev = (Rec*)workspace;
  hipError_t he = upload_recs(host, count, dev, s);
  free(host);
  if (he != hipSuccess) return KFB_EHIP;
  if (prec == KFB_FP64) return run_precond<KFB_FP64>(dev, count, p, flags, s);
  if (prec == KFB_FP32) return run_precond<KFB_FP32>(dev, count, p, flags, s);
  return run_precond<KFB_BF16_MIXED>(dev, count, p, flags, s);
}

int dispatch_fac(int count, kfb_state_t const* stG, kfb_state_t const* stA, const void* const* Gk, int64_t ldgk,
                 const void* const* Ak, int64_t ldak, int n, void* const* S, int64_t lds, const double* lamG,
                 const double* lamA, uint32_t flags, void* workspace, size_t ws_bytes, hipStream_t s,
                 size_t* need_only) {
  if (count <= 0 || !stG || !stA || n < 1) return KFB_EINVAL;
  kfb_state_t g0 = stG[0], a0 = stA[0];
  if (!g0 || !a0) return KFB_EINVAL;
  const int prec = g0->prec;
  const int NG = pre_modes(g0, flags), NA = pre_modes(a0, flags);
  for (int i = 0; i < count; ++i) {
    kfb_state_t g = stG[i], a = stA[i];
    if (!g || !a) return KFB_EINVAL;
    if (g == a) return KFB_ESTATE;
    if (g->prec != prec || a->prec != prec || g->d != g0->d || a->d != a0->d ||
        pre_modes(g, flags) != NG || pre_modes(a, flags) != NA || g->ldu != g0->ldu || a->ldu != a0->ldu)
      return KFB_ESTATE;
  }
  if (NG <= 0 || NA <= 0) return KFB_EEMPTY;
  if (ldgk < g0->d || ldak < a0->d || lds < a0->d) return KFB_EINVAL;
  FacPlan p;
  if (prec == KFB_FP64) make_fac_plan<KFB_FP64>(g0->d, a0->d, g0->ldu, a0->ldu, NG, NA, n, &p);
  else if (prec == KFB_FP32) make_fac_plan<KFB_FP32>(g0->d, a0->d, g0->ldu, a0->ldu, NG, NA, n, &p);
  else make_fac_plan<KFB_BF16_MIXED>(g0->d, a0->d, g0->ldu, a0->ldu, NG, NA, n, &p);
  p.ldgk = ldgk; p.ldak = ldak; p.lds = lds;
  const size_t head = align256(sizeof(Rec) * (size_t)count);
  const size_t need = head + p.per_problem * (size_t)count;
  if (need_only) { *need_only = need; return KFB_OK; }
  if (!Gk || !Ak || !S || !workspace || !lamG || !lamA) return KFB_EINVAL;
  if (ws_bytes < need) return KFB_EWORKSPACE;
  if (((uintptr_t)workspace) & 255) return KFB_EINVAL;
  // Y_G and Y_A columns start 16-byte aligned when d_out and d_in are multiples of 4
  p.aligned16 = (lds % 4 == 0) && (g0->d % 4 == 0) && (a0->d % 4 == 0);
  Rec* host = (Rec*)malloc(sizeof(Rec) * (size_t)count);
  if (!host) return KFB_EINVAL;
  const size_t selem = prec == KFB_FP64 ? 8 : 4;
  const size_t sbytes = (size_t)((g0->d - 1) * lds + a0->d) * selem;
  for (int i = 0; i < count; ++i) {
    if (!Gk[i] || !Ak[i] || !S[i] || !(lamG[i] > 0.0) || !(lamA[i] > 0.0)) { free(host); return KFB_EINVAL; }
    const char* sb = (const char*)S[i];
    auto overlaps = [&](const void* x, size_t xb) {
      const char* xc = (const char*)x;
      return sb < xc + xb && xc < sb + sbytes;
    };
    const size_t mel = m_elem(prec);
    if (overlaps(Gk[i], (size_t)((n - 1) * ldgk + g0->d) * mel) || overlaps(Ak[i], (size_t)((n - 1) * ldak + a0->d) * mel)) {
      free(host);
      return KFB_EINVAL;
    }
    if (((uintptr_t)S[i]) & 15) p.aligned16 = 0;
    kfb_state_t g = stG[i], a = stA[i];
    Rec* rc = &host[i];
    memset(rc, 0, sizeof(Rec));
    rc->p[PU_G] = g->buf + g->off_U[g->front];
    rc->p[PD_G] = g->buf + g->off_D[g->front];
    rc->p[PU_A] = a->buf + a->off_U[a->front];
    rc->p[PD_A] = a->buf + a->off_D[a->front];
    rc->p[P_G] = const_cast<void*>(Gk[i]);
    rc->p[P_AK] = const_cast<void*>(Ak[i]);
    rc->p[P_S] = S[i];
    rc->p[PWS] = (char*)workspace + head + p.per_problem * (size_t)i;
    rc->s[0] = lamG[i];
    rc->s[1] = lamA[i];
  }
  Rec* dev = (Rec*)workspace;
  hipError_t he = upload_recs(host, count, dev, s);
  free(host);
  if (he != hipSuccess) return KFB_EHIP;
  if (prec == KFB_FP64) return run_fac<KFB_FP64>(dev, count, p, flags, s);
  if (prec == KFB_FP32) return run_fac<KFB_FP32>(dev, count, p, flags, s);
  return run_fac<KFB_BF16_MIXED>(dev, count, p, flags, s);
}

int dispatch_dense(kfb_state_t st, void* X, int64_t ldx, const void* M, int64_t ldm, int n, int first,
                   void* workspace, size_t ws_bytes, hipStream_t s) {
  if (!st || !X || !M || !workspace || n < 1 || ldx < st->d || ldm < st->d) return KFB_EINVAL;
  if (ws_bytes < 256) return KFB_EWORKSPACE;
  if (((uintptr_t)workspace) & 255) return KFB_EINVAL;
  const size_t xe = st->prec == KFB_FP64 ? 8 : 4;
  const char* xb = (const char*)X;
  const char* mb = (const char*)M;
  const size_t xbytes = (size_t)((st->d - 1) * ldx + st->d) * xe;
  const size_t mbytes = (size_t)((n - 1) * ldm + st->d) * m_elem(st->prec);
  if (xb < mb + mbytes && mb < xb + xbytes) return KFB_EINVAL;
  Rec host;
  memset(&host, 0, sizeof(Rec));
  host.p[M_IN] = const_cast<void*>(M);
  host.p[B_X] = X;
  Rec* dev = (Rec*)workspace;
  if (upload_recs(&host, 1, dev, s) != hipSuccess) return KFB_EHIP;
  const double alpha = first ? 1.0 / n : (1.0 - st->rho) / n;
  const double beta = first ? 0.0 : st->rho;
  if (st->prec == KFB_FP64) return run_dense<KFB_FP64>(dev, st->d, ldx, ldm, n, alpha, beta, s);
  if (st->prec == KFB_FP32) return run_dense<KFB_FP32>(dev, st->d, ldx, ldm, n, alpha, beta, s);
  return run_dense<KFB_BF16_MIXED>(dev, st->d, ldx, ldm, n, alpha, beta, s);
}

constexpr int RSVD_MAX_POWER_ITS = 16;

int dispatch_rsvd(kfb_state_t st, const void* X, int64_t ldx, const void* Omega, int64_t ldo, int oversample,
                  int power_its, void* workspace, size_t ws_bytes, hipStream_t s, size_t* need_only) {
  if (!st || oversample < 0 || power_its < 0 || power_its > RSVD_MAX_POWER_ITS) return KFB_EINVAL;
  const int r = st->r;
  const int64_t l = (int64_t)r + oversample;
  if (r < 1 || l > st->d || l > (int64_t)r + st->n_max || l > 2048) return KFB_EINVAL;
  UpdPlan p;
  bool ok = false;
  if (st->prec == KFB_FP64) ok = make_upd_plan<KFB_FP64>(st->d, st->ldu, st->d, 0, (int)l, 1, &p);
  else if (st->prec == KFB_FP32) ok = make_upd_plan<KFB_FP32>(st->d, st->ldu, st->d, 0, (int)l, 1, &p);
  else ok = make_upd_plan<KFB_BF16_MIXED>(st->d, st->ldu, st->d, 0, (int)l, 1, &p);
  if (!ok) return KFB_EINVAL;
  const size_t ze = st->prec == KFB_FP64 ? 8 : 4;  // Y, Q element size
  const int64_t oZc = (int64_t)p.per_problem;
  const size_t head = align256(sizeof(Rec));
  const size_t need = head + p.per_problem + align256((size_t)st->d * l * ze);
  if (need_only) { *need_only = need; return KFB_OK; }
  if (!X || !Omega || !workspace || ldx < st->d || ldo < st->d) return KFB_EINVAL;
  if (ws_bytes < need) return KFB_EWORKSPACE;
  if (((uintptr_t)workspace) & 255) return KFB_EINVAL;
  Rec host;
  memset(&host, 0, sizeof(Rec));
  host.p[U_FRONT] = st->buf + st->off_U[st->front];
  host.p[U_BACK] = st->buf + st->off_U[1 - st->front];
  host.p[WS] = (char*)workspace + head;
  host.p[D_FRONT] = st->buf + st->off_D[st->front];
  host.p[D_BACK] = st->buf + st->off_D[1 - st->front];
  host.p[STATUS] = st->buf + st->off_status;
  host.p[B_X] = const_cast<void*>(X);
  host.p[B_OMEGA] = const_cast<void*>(Omega);
  host.s[0] = 0.0;  // core of the square factor R' alone: no decayed modes,
  host.s[1] = 1.0;  // unit weight
  Rec* dev = (Rec*)workspace;
  if (upload_recs(&host, 1, dev, s) != hipSuccess) return KFB_EHIP;
  int rc;
  if (st->prec == KFB_FP64) rc = run_rsvd<KFB_FP64>(dev, p, oZc, r, ldx, ldo, power_its, s);
  else if (st->prec == KFB_FP32) rc = run_rsvd<KFB_FP32>(dev, p, oZc, r, ldx, ldo, power_its, s);
  else rc = run_rsvd<KFB_BF16_MIXED>(dev, p, oZc, r, ldx, ldo, power_its, s);
  if (rc != KFB_OK) return rc;
  st->front = 1 - st->front;
  st->k_valid = r;
  return KFB_OK;
}

int dispatch_correct(kfb_state_t st, const void* X, int64_t ldx, const int32_t* col_idx, int n_crc,
                     void* workspace, size_t ws_bytes, hipStream_t s, size_t* need_only) {
  if (!st || n_crc < 1) return KFB_EINVAL;
  const int k = st->k_valid;
  const int rlead = st->r < k ? st->r : k;  // the columns Algorithm 6 draws from
  if (k <= 0) return KFB_EEMPTY;
  if (n_crc > rlead || k > 4096) return KFB_EINVAL;
  CorrPlan cp;
  bool ok = false;
  if (st->prec == KFB_FP64) ok = make_upd_plan<KFB_FP64>(st->d, st->ldu, st->d, 0, n_crc, 1, &cp.p);
  else if (st->prec == KFB_FP32) ok = make_upd_plan<KFB_FP32>(st->d, st->ldu, st->d, 0, n_crc, 1, &cp.p);
  else ok = make_upd_plan<KFB_BF16_MIXED>(st->d, st->ldu, st->d, 0, n_crc, 1, &cp.p);
  if (!ok) return KFB_EINVAL;
  const size_t ze = st->prec == KFB_FP64 ? 8 : 4;
  size_t o = cp.p.per_problem;
  cp.oUcw = (int64_t)o; o = align256(o + (size_t)st->d * n_crc * ze);
  cp.oIdx = (int64_t)o; o = align256(o + (size_t)n_crc * 4);
  cp.oSrc = (int64_t)o; o = align256(o + (size_t)k * 4);
  cp.per_problem = o;
  const size_t head = align256(sizeof(Rec));
  const size_t need = head + cp.per_problem;
  if (need_only) { *need_only = need; return KFB_OK; }
  if (!X || !col_idx || !workspace || ldx < st->d) return KFB_EINVAL;
  if (ws_bytes < need) return KFB_EWORKSPACE;
  if (((uintptr_t)workspace) & 255) return KFB_EINVAL;
  // host-side check of the draw: distinct indices among the leading modes
  std::vector<char> seen((size_t)rlead, 0);
  for (int t = 0; t < n_crc; ++t) {
    const int j = col_idx[t];
    if (j < 0 || j >= rlead || seen[(size_t)j]) return KFB_EINVAL;
    seen[(size_t)j] = 1;
  }
  Rec host;
  memset(&host, 0, sizeof(Rec));
  host.p[U_FRONT] = st->buf + st->off_U[st->front];
  host.p[U_BACK] = st->buf + st->off_U[1 - st->front];
  host.p[WS] = (char*)workspace + head;
  host.p[D_FRONT] = st->buf + st->off_D[st->front];
  host.p[D_BACK] = st->buf + st->off_D[1 - st->front];
  host.p[STATUS] = st->buf + st->off_status;
  host.p[B_X] = const_cast<void*>(X);
  host.s[0] = 0.0;
  host.s[1] = 1.0;
  Rec* dev = (Rec*)workspace;
  if (upload_recs(&host, 1, dev, s) != hipSuccess) return KFB_EHIP;
  if (hipMemcpyAsync((char*)workspace + head + cp.oIdx, col_idx, (size_t)n_crc * 4, hipMemcpyHostToDevice, s) !=
      hipSuccess)
    return KFB_EHIP;
  int rc;
  if (st->prec == KFB_FP64) rc = run_correct<KFB_FP64>(dev, cp, k, ldx, s);
  else if (st->prec == KFB_FP32) rc = run_correct<KFB_FP32>(dev, cp, k, ldx, s);
  else rc = run_correct<KFB_BF16_MIXED>(dev, cp, k, ldx, s);
  if (rc != KFB_OK) return rc;
  st->front = 1 - st->front;
  return KFB_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free update: the workspace is a file-scope device array, one copy
// per GPU, resolved to a device address once per device (the array's name in
// host code is not a device address).
// ---------------------------------------------------------------------------
constexpr size_t SCRATCH_BYTES = size_t(64) << 20;
__device__ __align__(256) char scratch[SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // indexed by device ordinal

int scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return KFB_EHIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
  if (!g_scratch_ptr[(size_t)dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return KFB_EHIP;
    g_scratch_ptr[(size_t)dev] = p;
  }
  *out = g_scratch_ptr[(size_t)dev];
  return KFB_OK;
}

}  // namespace

extern "C" {

size_t kfb_scratch_bytes(void) { return SCRATCH_BYTES; }

int kfb_brand_update_scratch(kfb_state_t st, const void* M, int64_t ldm, int32_t n, kfb_stream_t stream) {
  if (!st || !M) return KFB_EINVAL;
  size_t need = 0;
  int rc = dispatch_update(1, &st, nullptr, ldm, n, nullptr, 0, nullptr, &need);
  if (rc != KFB_OK) return rc;
  if (need > SCRATCH_BYTES) return KFB_EWORKSPACE;
  void* ws = nullptr;
  if ((rc = scratch_address(&ws)) != KFB_OK) return rc;
  const void* Ms[1] = {M};
  return dispatch_update(1, &st, Ms, ldm, n, ws, SCRATCH_BYTES, (hipStream_t)stream, nullptr);
}

size_t kfb_state_bytes(int64_t d, int32_t r, int32_t n_max, int32_t prec) {
  if (d <= 0 || r < 0 || n_max <= 0 || (int64_t)r + n_max > d) return 0;
  if (n_max > MAX_QR_COLS || (int64_t)r + n_max > MAX_CORE) return 0;
  if (prec < KFB_FP64 || prec > KFB_BF16_MIXED) return 0;
  const int64_t cap = (int64_t)r + n_max;
  const size_t ub = align256((size_t)ldu_for(d, prec) * cap * u_elem(prec));
  const size_t db = align256((size_t)cap * d_elem(prec));
  return 2 * ub + 2 * db + 256;
}

int kfb_state_create(kfb_state_t* out, int64_t d, int32_t r, int32_t n_max, double rho, int32_t prec,
                     void* state_buf, size_t state_bytes, kfb_stream_t stream) {
  if (!out || !state_buf) return KFB_EINVAL;
  const size_t need = kfb_state_bytes(d, r, n_max, prec);
  if (need == 0 || !(rho >= 0.0 && rho < 1.0)) return KFB_EINVAL;
  if (state_bytes < need) return KFB_EWORKSPACE;
  if (((uintptr_t)state_buf) & 255) return KFB_EINVAL;
  kfb_state_s* st = new (std::nothrow) kfb_state_s();
  if (!st) return KFB_EINVAL;
  st->d = d; st->r = r; st->n_max = n_max; st->prec = prec; st->rho = rho;
  st->buf = (char*)state_buf; st->bytes = state_bytes;
  st->ldu = ldu_for(d, prec);
  const int64_t cap = (int64_t)r + n_max;
  const size_t ub = align256((size_t)st->ldu * cap * u_elem(prec));
  const size_t db = align256((size_t)cap * d_elem(prec));
  st->off_U[0] = 0; st->off_U[1] = ub;
  st->off_D[0] = 2 * ub; st->off_D[1] = 2 * ub + db;
  st->off_status = 2 * ub + 2 * db;
  if (hipMemsetAsync(st->buf + st->off_status, 0, 4, (hipStream_t)stream) != hipSuccess) {
    delete st;
    return KFB_EHIP;
  }
  *out = st;
  return KFB_OK;
}

int kfb_destroy(kfb_state_t st) {
  if (!st) return KFB_EINVAL;
  delete st;
  return KFB_OK;
}

size_t kfb_update_workspace_bytes(kfb_state_t st, int32_t n) {
  size_t need = 0;
  if (!st) return 0;
  if (dispatch_update(1, &st, nullptr, st->d, n, nullptr, 0, nullptr, &need) != KFB_OK) return 0;
  return need;
}

int kfb_brand_update(kfb_state_t st, const void* M, int64_t ldm, int32_t n, void* workspace,
                     size_t ws_bytes, kfb_stream_t stream) {
  if (!st || !M) return KFB_EINVAL;
  const void* Ms[1] = {M};
  return dispatch_update(1, &st, Ms, ldm, n, workspace, ws_bytes, (hipStream_t)stream, nullptr);
}

size_t kfb_update_batched_workspace_bytes(int32_t count, kfb_state_t const* states, int32_t n) {
  size_t need = 0;
  if (count <= 0 || !states || !states[0]) return 0;
  if (dispatch_update(count, states, nullptr, states[0]->d, n, nullptr, 0, nullptr, &need) != KFB_OK)
    return 0;
  return need;
}

int kfb_brand_update_batched(int32_t count, kfb_state_t const* states, const void* const* Ms,
                             int64_t ldm, int32_t n, void* workspace, size_t ws_bytes,
                             kfb_stream_t stream) {
  return dispatch_update(count, states, Ms, ldm, n, workspace, ws_bytes, (hipStream_t)stream, nullptr);
}

size_t kfb_precondition_workspace_bytes(kfb_state_t st_gamma, kfb_state_t st_a) {
  size_t need = 0;
  if (!st_gamma || !st_a) return 0;
  double l = 1.0;
  if (dispatch_precond(1, &st_gamma, &st_a, nullptr, st_a->d, nullptr, st_a->d, &l, &l, 0, nullptr, 0,
                       nullptr, &need) != KFB_OK)
    return 0;
  return need;
}

int kfb_precondition(kfb_state_t st_gamma, kfb_state_t st_a, const void* G, int64_t ldg, void* S,
                     int64_t lds, double lam_gamma, double lam_a, uint32_t flags, void* workspace,
                     size_t ws_bytes, kfb_stream_t stream) {
  const void* Gs[1] = {G};
  void* Ss[1] = {S};
  return dispatch_precond(1, &st_gamma, &st_a, Gs, ldg, Ss, lds, &lam_gamma, &lam_a, flags, workspace,
                          ws_bytes, (hipStream_t)stream, nullptr);
}

size_t kfb_precondition_batched_workspace_bytes(int32_t count, kfb_state_t const* st_gamma,
                                                kfb_state_t const* st_a) {
  size_t need = 0;
  if (count <= 0 || !st_gamma || !st_a || !st_a[0]) return 0;
  double* l = (double*)malloc(sizeof(double) * (size_t)count);
  if (!l) return 0;
  for (int i = 0; i < count; ++i) l[i] = 1.0;
  const int rc = dispatch_precond(count, st_gamma, st_a, nullptr, st_a[0]->d, nullptr, st_a[0]->d, l, l, 0,
                                  nullptr, 0, nullptr, &need);
  free(l);
  return rc == KFB_OK ? need : 0;
}

int kfb_precondition_batched(int32_t count, kfb_state_t const* st_gamma, kfb_state_t const* st_a,
                             const void* const* G, int64_t ldg, void* const* S, int64_t lds,
                             const double* lam_gamma, const double* lam_a, uint32_t flags,
                             void* workspace, size_t ws_bytes, kfb_stream_t stream) {
  return dispatch_precond(count, st_gamma, st_a, G, ldg, S, lds, lam_gamma, lam_a, flags, workspace,
                          ws_bytes, (hipStream_t)stream, nullptr);
}

size_t kfb_precondition_factored_workspace_bytes(kfb_state_t st_gamma, kfb_state_t st_a, int32_t n) {
  return kfb_precondition_factored_batched_workspace_bytes(1, &st_gamma, &st_a, n);
}

int kfb_precondition_factored(kfb_state_t st_gamma, kfb_state_t st_a, const void* G_k, int64_t ldgk,
                              const void* A_k, int64_t ldak, int32_t n, void* S, int64_t lds,
                              double lam_gamma, double lam_a, uint32_t flags, void* workspace,
                              size_t ws_bytes, kfb_stream_t stream) {
  const void* Gs[1] = {G_k};
  const void* As[1] = {A_k};
  void* Ss[1] = {S};
  return dispatch_fac(1, &st_gamma, &st_a, Gs, ldgk, As, ldak, n, Ss, lds, &lam_gamma, &lam_a, flags,
                      workspace, ws_bytes, (hipStream_t)stream, nullptr);
}

size_t kfb_precondition_factored_batched_workspace_bytes(int32_t count, kfb_state_t const* st_gamma,
                                                         kfb_state_t const* st_a, int32_t n) {
  size_t need = 0;
  if (count <= 0 || !st_gamma || !st_a || !st_gamma[0] || !st_a[0]) return 0;
  double* l = (double*)malloc(sizeof(double) * (size_t)count);
  if (!l) return 0;
  for (int i = 0; i < count; ++i) l[i] = 1.0;
  const int rc = dispatch_fac(count, st_gamma, st_a, nullptr, st_gamma[0]->d, nullptr, st_a[0]->d, n, nullptr,
                              st_a[0]->d, l, l, 0, nullptr, 0, nullptr, &need);
  free(l);
  return rc == KFB_OK ? need : 0;
}

int kfb_precondition_factored_batched(int32_t count, kfb_state_t const* st_gamma,
                                      kfb_state_t const* st_a, const void* const* G_k, int64_t ldgk,
                                      const void* const* A_k, int64_t ldak, int32_t n, void* const* S,
                                      int64_t lds, const double* lam_gamma, const double* lam_a,
                                      uint32_t flags, void* workspace, size_t ws_bytes,
                                      kfb_stream_t stream) {
  return dispatch_fac(count, st_gamma, st_a, G_k, ldgk, A_k, ldak, n, S, lds, lam_gamma, lam_a, flags,
                      workspace, ws_bytes, (hipStream_t)stream, nullptr);
}

size_t kfb_dense_bytes(int64_t d, int64_t ldx, int32_t prec) {
  if (d <= 0 || ldx < d || prec < KFB_FP64 || prec > KFB_BF16_MIXED) return 0;
  return (size_t)ldx * d * (prec == KFB_FP64 ? 8 : 4);
}

size_t kfb_dense_update_workspace_bytes(void) { return 256; }

int kfb_dense_update(kfb_state_t st, void* X, int64_t ldx, const void* M, int64_t ldm, int32_t n,
                     int32_t first, void* workspace, size_t ws_bytes, kfb_stream_t stream) {
  return dispatch_dense(st, X, ldx, M, ldm, n, first, workspace, ws_bytes, (hipStream_t)stream);
}

size_t kfb_rsvd_workspace_bytes(kfb_state_t st, int32_t oversample) {
  size_t need = 0;
  if (dispatch_rsvd(st, nullptr, 0, nullptr, 0, oversample, 0, nullptr, 0, nullptr, &need) != KFB_OK) return 0;
  return need;
}

int kfb_rsvd_overwrite(kfb_state_t st, const void* X, int64_t ldx, const void* Omega, int64_t ldo,
                       int32_t oversample, int32_t power_its, void* workspace, size_t ws_bytes,
                       kfb_stream_t stream) {
  return dispatch_rsvd(st, X, ldx, Omega, ldo, oversample, power_its, workspace, ws_bytes, (hipStream_t)stream,
                       nullptr);
}

size_t kfb_correct_workspace_bytes(kfb_state_t st, int32_t n_crc) {
  size_t need = 0;
  if (dispatch_correct(st, nullptr, 0, nullptr, n_crc, nullptr, 0, nullptr, &need) != KFB_OK) return 0;
  return need;
}

int kfb_light_correction(kfb_state_t st, const void* X, int64_t ldx, const int32_t* col_idx, int32_t n_crc,
                         void* workspace, size_t ws_bytes, kfb_stream_t stream) {
  return dispatch_correct(st, X, ldx, col_idx, n_crc, workspace, ws_bytes, (hipStream_t)stream, nullptr);
}

size_t kfb_update_grouped_workspace_bytes(int32_t count, kfb_state_t const* states, const int32_t* widths) {
  size_t need = 0;
  if (dispatch_update_cross(count, states, nullptr, nullptr, widths, nullptr, 0, nullptr, &need) != KFB_OK) return 0;
  return need;
}

int kfb_brand_update_grouped(int32_t count, kfb_state_t const* states, const void* const* Ms, const int64_t* ldms,
                             const int32_t* widths, void* workspace, size_t ws_bytes, kfb_stream_t stream) {
  return dispatch_update_cross(count, states, Ms, ldms, widths, workspace, ws_bytes, (hipStream_t)stream, nullptr);
}

int kfb_brand_update_batched_widths(int32_t count, kfb_state_t const* states, const void* const* Ms,
                                    int64_t ldm, int32_t n, const int32_t* widths, void* workspace,
                                    size_t ws_bytes, kfb_stream_t stream) {
  if (!widths) return KFB_EINVAL;
  return dispatch_update(count, states, Ms, ldm, n, workspace, ws_bytes, (hipStream_t)stream, nullptr, widths);
}

int kfb_state_info(kfb_state_t st, int32_t* k_valid, int64_t* step, int64_t* d, int32_t* r,
                   int32_t* n_max, int32_t* prec) {
  if (!st) return KFB_EINVAL;
  if (k_valid) *k_valid = st->k_valid;
  if (step) *step = st->step;
  if (d) *d = st->d;
  if (r) *r = st->r;
  if (n_max) *n_max = st->n_max;
  if (prec) *prec = st->prec;
  return KFB_OK;
}

int kfb_state_front(kfb_state_t st, const void** U, int64_t* ldu, const void** D) {
  if (!st) return KFB_EINVAL;
  if (U) *U = st->buf + st->off_U[st->front];
  if (ldu) *ldu = st->ldu;
  if (D) *D = st->buf + st->off_D[st->front];
  return KFB_OK;
}

int kfb_state_load(kfb_state_t st, const void* U, int64_t ldu, const void* D, int32_t k, int64_t step,
                   kfb_stream_t stream) {
  if (!st || !U || !D || k < 0 || k > st->r + st->n_max || k > st->d || ldu < st->d || step < 0)
    return KFB_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const size_t ue = u_elem(st->prec), de = d_elem(st->prec);
  if (k > 0) {
    // the eigenvalues must be finite, non-negative and descending (truncation
    // keeps the leading modes): read back and checked before anything is written
    std::vector<double> h((size_t)k);
    if (de == 8) {
      KFB_TRY(hipMemcpyAsync(h.data(), D, (size_t)k * 8, hipMemcpyDeviceToHost, s));
      KFB_TRY(hipStreamSynchronize(s));
    } else {
      std::vector<float> f((size_t)k);
      KFB_TRY(hipMemcpyAsync(f.data(), D, (size_t)k * 4, hipMemcpyDeviceToHost, s));
      KFB_TRY(hipStreamSynchronize(s));
      for (int i = 0; i < k; ++i) h[(size_t)i] = (double)f[(size_t)i];
    }
    for (int i = 0; i < k; ++i) {
      const double v = h[(size_t)i];
      if (!(v >= 0.0) || !(v <= 1.7976931348623157e308)) return KFB_EINVAL;
      if (i > 0 && v > h[(size_t)i - 1]) return KFB_EINVAL;
    }
    char* Uf = st->buf + st->off_U[st->front];
    char* Df = st->buf + st->off_D[st->front];
    KFB_TRY(hipMemcpy2DAsync(Uf, (size_t)st->ldu * ue, U, (size_t)ldu * ue, (size_t)st->d * ue, (size_t)k,
                             hipMemcpyDeviceToDevice, s));
    KFB_TRY(hipMemcpyAsync(Df, D, (size_t)k * de, hipMemcpyDeviceToDevice, s));
    // unit column norms (the cheap half of orthonormality), as the drift detector
    uint32_t* status = (uint32_t*)(st->buf + st->off_status);
    const double tol = drift_tol(st->prec);
    hipError_t e;
    if (st->prec == KFB_FP64) e = loaded_norms<double, double>((const double*)Uf, st->ldu, st->d, k, (const double*)Df, tol, status, s);
    else if (st->prec == KFB_FP32) e = loaded_norms<float, float>((const float*)Uf, st->ldu, st->d, k, (const float*)Df, tol, status, s);
    else e = loaded_norms<float, double>((const float*)Uf, st->ldu, st->d, k, (const double*)Df, tol, status, s);
    KFB_TRY(e);
  }
  st->k_valid = k;
  st->step = step;
  return KFB_OK;
}

size_t kfb_reorth_workspace_bytes(kfb_state_t st) {
  size_t need = 0;
  if (dispatch_reorth(st, nullptr, 0, nullptr, &need) != KFB_OK) return 0;
  return need;
}

int kfb_reorthonormalize(kfb_state_t st, void* workspace, size_t ws_bytes, kfb_stream_t stream) {
  return dispatch_reorth(st, workspace, ws_bytes, (hipStream_t)stream, nullptr);
}

int kfb_state_status(kfb_state_t st, uint32_t* events, kfb_stream_t stream) {
  if (!st || !events) return KFB_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  uint32_t v = 0;
  KFB_TRY(hipMemcpyAsync(&v, st->buf + st->off_status, 4, hipMemcpyDeviceToHost, s));
  KFB_TRY(hipStreamSynchronize(s));
  KFB_TRY(hipMemsetAsync(st->buf + st->off_status, 0, 4, s));
  KFB_TRY(hipStreamSynchronize(s));
  *events = v;
  return KFB_OK;
}

int kfb_tune_set_jacobi(int32_t prec, int32_t N, int32_t bw) {
  if (prec < KFB_FP64 || prec > KFB_BF16_MIXED || N <= 0) return KFB_EINVAL;
  const int eb = prec == KFB_FP32 ? 4 : 8;
  if (bw & JAC_REFINE) {  // mixed form, 32-column streamed panels only
    if (prec != KFB_BF16_MIXED || (bw & ~JAC_REFINE) != (JAC_STREAMED | 32)) return KFB_EINVAL;
  }
  if (bw != 0 && jacobi_block_fits(N, eb, bw & ~JAC_REFINE) == 0) return KFB_EINVAL;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (size_t i = 0; i < g_tune.size(); ++i)
    if (g_tune[i].prec == prec && g_tune[i].N == N) {
      if (bw == 0) g_tune.erase(g_tune.begin() + i);
      else g_tune[i].bw = bw;
      return KFB_OK;
    }
  if (bw != 0) g_tune.push_back(TuneEntry{prec, N, bw});
  return KFB_OK;
}

int kfb_tune_get_jacobi(int32_t prec, int32_t N, int32_t* bw, int32_t* Np) {
  if (prec < KFB_FP64 || prec > KFB_BF16_MIXED || N <= 0) return KFB_EINVAL;
  const int eb = prec == KFB_FP32 ? 4 : 8;
  int np = 0;
  const int b = pick_jacobi(prec, N, eb, N >= 256, &np, true);  // as a Brand update's main solve
  if (bw) *bw = b;
  if (Np) *Np = np;
  return b ? KFB_OK : KFB_EINVAL;
}

int kfb_tune_set_gemm(int32_t m, int32_t n, int32_t k, int32_t tile) {
  return gemm_tile_set(m, n, k, tile) == 0 ? KFB_OK : KFB_EINVAL;
}

int kfb_tune_get_gemm(int32_t m, int32_t n, int32_t k, int32_t* tile) {
  if (m <= 0 || n <= 0 || k <= 0 || !tile) return KFB_EINVAL;
  const int t = gemm_tile_lookup(m, n, k);
  *tile = t ? t : 128;
  return KFB_OK;
}

int kfb_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.on = on != 0;
  return KFB_OK;
}

int kfb_profile_report(char* buf, size_t len, int reset) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  int rc = KFB_OK;
  for (auto& pe : g_prof.pending) {
    float ms = 0.f;
    if (hipEventSynchronize(pe.b) != hipSuccess || hipEventElapsedTime(&ms, pe.a, pe.b) != hipSuccess) rc = KFB_EHIP;
    g_prof.stages[pe.stage].ms += ms;
    g_prof.pool.push_back(pe.a);
    g_prof.pool.push_back(pe.b);
  }
  g_prof.pending.clear();
  if (buf && len > 0) {
    std::string out = "{";
    char item[256];
    for (size_t i = 0; i < g_prof.stages.size(); ++i) {
      const ProfStage& st = g_prof.stages[i];
      snprintf(item, sizeof(item), "%s\"%s\": {\"calls\": %ld, \"launches\": %ld, \"ms\": %.6f}",
               i ? ", " : "", st.name, st.calls, st.launches, st.ms);
      out += item;
    }
    out += "}";
    const size_t nc = out.size() < len - 1 ? out.size() : len - 1;
    memcpy(buf, out.data(), nc);
    buf[nc] = 0;
  }
  if (reset) {
    for (auto& st : g_prof.stages) { st.calls = 0; st.launches = 0; st.ms = 0.0; }
  }
  return rc;
}

const char* kfb_strerror(int code) {
  switch (code) {
    case KFB_OK: return "ok";
    case KFB_EINVAL: return "invalid argument";
    case KFB_EWORKSPACE: return "buffer or workspace too small";
    case KFB_EHIP: return "HIP runtime error";
    case KFB_ESTATE: return "incompatible states";
    case KFB_EEMPTY: return "state holds no modes";
    default: return "unknown error";
  }
}

#ifndef KFB_SRC_DIGEST
#define KFB_SRC_DIGEST "unknown"
#endif
const char* kfb_build_info(void) { return "kfb gfx950 hip src=" KFB_SRC_DIGEST; }

}  // extern "C"
