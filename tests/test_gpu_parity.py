"""GPU parity of the HIP path against the FP64 CPU oracle (through the C-ABI).

Tolerances: relative reconstruction / preconditioned-gradient error <= 1e-10
(FP64 form), <= 1e-5 (FP32 form), <= 2e-2 (BF16-mixed form).
"""
import numpy as np
import pytest

import oracle
from paper_2210_08494_amd import synth

pytestmark = pytest.mark.gpu

TOL = {0: 1e-10, 1: 1e-5, 2: 2e-2}


def _dev():
    import torch
    return torch.device("cuda:0")


def _to_dev(x, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(device=_dev(), dtype=dtype)


def _front_np(f):
    import torch
    torch.cuda.synchronize()
    U, D = f.front()
    return U.double().cpu().numpy(), D.double().cpu().numpy()


def _batch(cfg, k, side, n, d, bias=False, prec=0):
    x = synth.batch_for(cfg, k, side, n, d, bias=bias)
    if prec == 2:
        x = synth.to_bf16_values(x)  # the exact values a BF16 buffer holds, for both sides
    return x


def _announce(msg):
    print(msg, flush=True)


# ----------------------------------------------------------------------------
# FP64 form: the paper's first workload shape (one FC layer, d = 256)
# ----------------------------------------------------------------------------
def test_fp64_layer_trajectory_vs_dense_definition(kfb):
    import torch
    d, r, n, rho, lam, steps = 256, 32, 32, 0.95, 0.1, 50
    _announce(f"fp64 trajectory d={d} r={r} n={n} steps={steps}")
    fa = kfb.Factor(d, r, n, rho, kfb.KFB_FP64)
    fg = kfb.Factor(d, r, n, rho, kfb.KFB_FP64)
    oa, og = oracle.DenseFactor(d, r, rho), oracle.DenseFactor(d, r, rho)
    worst = dict(rec=0.0, D=0.0, orth=0.0, S=0.0)
    for k in range(steps):
        a, g = _batch(1, k, "A", n, d), _batch(1, k, "G", n, d)
        fa.update(_to_dev(a, torch.float64))
        fg.update(_to_dev(g, torch.float64))
        oa.update(a.T)
        og.update(g.T)
        for f, o in ((fa, oa), (fg, og)):
            U, D = _front_np(f)
            V, lamv = o.modes()
            assert U.shape[1] == o.kept
            worst["rec"] = max(worst["rec"], oracle.e_rec_dense(U, D, o.X))
            worst["D"] = max(worst["D"], oracle.e_D(D, lamv))
            worst["orth"] = max(worst["orth"], oracle.e_orth(U))
        if k % 10 == 9 or k == 0:
            G = synth.grad_for(1, k, d, d)
            Gd = _to_dev(G, torch.float64)
            S = torch.empty_like(Gd)
            kfb.precondition(fg, fa, Gd, S, lam, lam)
            torch.cuda.synchronize()
            S_ref = oracle.precondition_dense(og.X, oa.X, G, lam, lam)
            VG, VA = og.modes()[0], oa.modes()[0]
            worst["S"] = max(worst["S"], oracle.e_S(S.cpu().numpy(), S_ref),
                             oracle.e_S_proj(S.cpu().numpy(), S_ref, VG, VA))
    _announce(f"  worst: {worst}")
    assert worst["rec"] <= 1e-10 and worst["D"] <= 1e-10 and worst["S"] <= 1e-10
    assert worst["orth"] <= 1e-11
    assert fa.status() == 0 and fg.status() == 0


def test_fp64_untruncated_reproduces_ea_factor(kfb):
    # r + n grows to d: truncation never bites, so U D U^T must equal the EA sum exactly
    import torch
    d, n, r, rho = 256, 32, 224, 0.95
    _announce("fp64 untruncated exactness")
    f = kfb.Factor(d, r, n, rho, kfb.KFB_FP64)
    Ms = []
    for k in range(8):
        M = _batch(1, 100 + k, "G", n, d).T
        Ms.append(M)
        f.update(_to_dev(M.T, torch.float64))
        E = sum(((1.0 if i == 0 else 1 - rho) * rho ** (k - i) / n) * (Ms[i] @ Ms[i].T) for i in range(k + 1))
        U, D = _front_np(f)
        assert U.shape[1] == min((k + 1) * n, d)
        e = oracle.e_rec_dense(U, D, E)
        assert e <= 1e-10, (k, e)
        assert oracle.e_orth(U) <= 1e-10


@pytest.mark.parametrize("d,r,n,steps", [(100, 7, 5, 7), (64, 3, 1, 12), (130, 40, 24, 5), (48, 40, 8, 3)])
def test_fp64_ragged_shapes(kfb, d, r, n, steps):
    # ragged tiles, padded Jacobi panels, n = 1, r + n = d
    import torch
    _announce(f"fp64 ragged d={d} r={r} n={n}")
    rho = 0.9
    f = kfb.Factor(d, r, n, rho, kfb.KFB_FP64)
    o = oracle.DenseFactor(d, r, rho)
    for k in range(steps):
        M = _batch(7, k, "A", n, d)
        f.update(_to_dev(M, torch.float64))
        o.update(M.T)
        U, D = _front_np(f)
        V, lamv = o.modes()
        assert oracle.e_rec_dense(U, D, o.X) <= 1e-10
        assert oracle.e_D(D, lamv) <= 1e-10


def test_fp64_rho_zero_and_first_step(kfb):
    import torch
    d, r, n = 128, 16, 16
    f = kfb.Factor(d, r, n, 0.0, kfb.KFB_FP64)
    for k in range(3):
        M = _batch(9, k, "G", n, d)
        f.update(_to_dev(M, torch.float64))
        U, D = _front_np(f)
        s = np.linalg.svd(M.T, compute_uv=False)
        top = np.sort(D)[::-1][:n]
        assert np.allclose(top, s ** 2 / n, rtol=1e-10, atol=1e-12 * s[0] ** 2)


def test_fp64_degenerate_batches(kfb):
    import torch
    d, r, n, rho = 96, 8, 6, 0.9
    _announce("fp64 degenerate batches")
    # duplicate columns: the residual is rank deficient
    f = kfb.Factor(d, r, n, rho, kfb.KFB_FP64)
    o = oracle.DenseFactor(d, r, rho)
    M = _batch(11, 0, "A", n, d)
    M[3] = M[1]
    f.update(_to_dev(M, torch.float64))
    o.update(M.T)
    U, D = _front_np(f)
    assert oracle.e_rec_dense(U, D, o.X) <= 1e-10
    assert f.status() & kfb.KFB_EV_CHOL_DEFICIENT
    # a batch inside span(U): Z_perp = 0
    M2 = (U[:, :3] @ np.random.default_rng(0).standard_normal((3, n))).T.copy()
    f.update(_to_dev(M2, torch.float64))
    o.update(M2.T)
    U, D = _front_np(f)
    assert oracle.e_rec_dense(U, D, o.X) <= 1e-10
    # a zero batch
    Z = np.zeros((n, d))
    f.update(_to_dev(Z, torch.float64))
    o.update(Z.T)
    U, D = _front_np(f)
    assert np.all(np.isfinite(U)) and np.all(np.isfinite(D))
    assert oracle.e_rec_dense(U, D, o.X) <= 1e-10
    # nonfinite input is reported, never crashes
    Mn = _batch(11, 3, "A", n, d)
    Mn[0, 0] = np.nan
    g = kfb.Factor(d, r, n, rho, kfb.KFB_FP64)
    g.update(_to_dev(Mn, torch.float64))
    assert g.status() & kfb.KFB_EV_NONFINITE


def _oracle_state(d, r, n, rho, steps, cfg, side):
    b = oracle.BrandFactor(d, r, rho)
    for k in range(steps):
        b.update(_batch(cfg, k, side, n, d).T)
    return b


@pytest.mark.parametrize("flags", [0, 1, 2, 3, 4, 5, 6, 7])
def test_fp64_precondition_on_loaded_state(kfb, flags):
    # the apply in isolation: both sides start from the same oracle-built state
    import torch
    dG, dA, r, n, rho = 200, 300, 20, 12, 0.95
    _announce(f"fp64 precondition flags={flags}")
    bg = _oracle_state(dG, r, n, rho, 4, 21, "G")
    ba = _oracle_state(dA, r, n, rho, 4, 21, "A")
    fg = kfb.Factor(dG, r, n, rho, kfb.KFB_FP64)
    fa = kfb.Factor(dA, r, n, rho, kfb.KFB_FP64)
    fg.load_state(_to_dev(bg.U, torch.float64), _to_dev(bg.D, torch.float64), step=4)
    fa.load_state(_to_dev(ba.U, torch.float64), _to_dev(ba.D, torch.float64), step=4)
    G = synth.grad_for(21, 0, dG, dA)
    Gd = _to_dev(G, torch.float64)
    S = torch.full_like(Gd, float("nan"))
    lg, la = 0.05, 0.2
    kfb.precondition(fg, fa, Gd, S, lg, la, flags=flags)
    torch.cuda.synchronize()
    UG, DG, UA, DA = bg.U, bg.D, ba.U, ba.D
    if flags & 2:
        UG, DG, UA, DA = UG[:, :r], DG[:r], UA[:, :r], DA[:r]
    lgx, lax = lg, la
    if flags & 4:   # relative damping: lam = phi * lambda_max of the modes used
        lgx, lax = lg * DG.max(), la * DA.max()
    if flags & 1:
        DG, lgx = oracle.spectrum_continuation(DG, lgx)
        DA, lax = oracle.spectrum_continuation(DA, lax)
    XG, XA = (UG * DG) @ UG.T, (UA * DA) @ UA.T
    S_ref = oracle.precondition_dense(XG, XA, G, lgx, lax)
    Sg = S.cpu().numpy()
    assert oracle.e_S(Sg, S_ref) <= 1e-10
    assert oracle.e_S_proj(Sg, S_ref, UG, UA) <= 1e-10
    assert np.max(np.abs(Sg - S_ref)) <= 1e-10 * np.max(np.abs(S_ref))


# ----------------------------------------------------------------------------
# FP32 form
# ----------------------------------------------------------------------------
def test_fp32_trajectory_small(kfb):
    import torch
    d, r, n, rho, steps = 512, 64, 64, 0.95, 20
    _announce(f"fp32 trajectory d={d} r={r} n={n}")
    f = kfb.Factor(d, r, n, rho, kfb.KFB_FP32)
    o = oracle.DenseFactor(d, r, rho)
    worst = 0.0
    for k in range(steps):
        M = _batch(2, k, "A", n, d)
        Mf = M.astype(np.float32).astype(np.float64)
        f.update(_to_dev(Mf, torch.float32))
        o.update(Mf.T)
        U, D = _front_np(f)
        worst = max(worst, oracle.e_rec_dense(U, D, o.X))
    _announce(f"  worst e_rec {worst:.3e}")
    assert worst <= TOL[1]


# ----------------------------------------------------------------------------
# BF16-mixed form
# ----------------------------------------------------------------------------
def test_mixed_trajectory_small(kfb):
    import torch
    d, r, n, rho, steps = 1024, 128, 128, 0.95, 12
    _announce(f"mixed trajectory d={d} r={r} n={n}")
    f = kfb.Factor(d, r, n, rho, kfb.KFB_BF16_MIXED)
    o = oracle.BrandFactor(d, r, rho)
    worst = 0.0
    for k in range(steps):
        M = _batch(3, k, "A", n, d, prec=2)
        f.update(_to_dev(M, torch.bfloat16))
        o.update(M.T)
        U, D = _front_np(f)
        worst = max(worst, oracle.e_rec_lowrank(U, D, o.U, o.D))
    _announce(f"  worst e_rec {worst:.3e} orth {oracle.e_orth(U):.3e}")
    assert worst <= TOL[2]


def test_mixed_long_run_stability(kfb):
    # 150 consecutive BF16-mixed updates: the re-projection and CholeskyQR2 keep
    # U orthonormal (no accumulation of the BF16 rounding across steps) and the
    # state tracks the FP64 oracle throughout
    import torch
    d, r, n, steps = 1024, 64, 64, 150
    _announce(f"mixed long run d={d} r={r} n={n} steps={steps}")
    f = kfb.Factor(d, r, n, 0.95, kfb.KFB_BF16_MIXED)
    o = oracle.BrandFactor(d, r, 0.95)
    errs, orths = [], []
    for k in range(steps):
        M = _batch(18, k, "A", n, d, prec=2)
        f.update(_to_dev(M, torch.bfloat16))
        o.update(M.T)
        if k % 10 == 9:
            U, D = _front_np(f)
            errs.append(oracle.e_rec_lowrank(U, D, o.U, o.D))
            orths.append(oracle.e_orth(U))
    _announce(f"  e_rec first {errs[0]:.3e} last {errs[-1]:.3e} max {max(errs):.3e}; "
              f"orth first {orths[0]:.3e} last {orths[-1]:.3e} max {max(orths):.3e}")
    assert max(errs) <= TOL[2]
    assert max(orths) <= 1e-3            # the drift detector's threshold for this form
    assert orths[-1] <= 10 * orths[0] + 1e-6   # no growth over the run
    assert f.status() == 0


@pytest.mark.parametrize("d,r,n", [(1056, 64, 64), (1000, 36, 20), (4100, 40, 36)])
def test_mixed_ragged_products(kfb, d, r, n):
    # shapes off the MFMA GEMMs' tile grid: split-K with a short last chunk
    # (d = 1056: chunks of 288), d not a multiple of 32 (element-wise fallback),
    # ranks and widths that are not multiples of 32
    import torch
    _announce(f"mixed ragged d={d} r={r} n={n}")
    f = kfb.Factor(d, r, n, 0.95, kfb.KFB_BF16_MIXED)
    o = oracle.BrandFactor(d, r, 0.95)
    worst = 0.0
    for k in range(5):
        M = _batch(17, k, "G", n, d, prec=2)
        f.update(_to_dev(M, torch.bfloat16))
        o.update(M.T)
        U, D = _front_np(f)
        worst = max(worst, oracle.e_rec_lowrank(U, D, o.U, o.D))
    _announce(f"  worst e_rec {worst:.3e} orth {oracle.e_orth(U):.3e}")
    assert worst <= TOL[2] and oracle.e_orth(U) <= TOL[2]
    assert f.status() == 0


def test_batched_equals_single(kfb):
    import torch
    d, r, n, rho = 384, 32, 32, 0.95
    for prec, dt in ((kfb.KFB_FP64, torch.float64), (kfb.KFB_FP32, torch.float32),
                     (kfb.KFB_BF16_MIXED, torch.bfloat16)):
        _announce(f"batched == single, prec={prec}")
        single = [kfb.Factor(d, r, n, rho, prec) for _ in range(3)]
        grouped = [kfb.Factor(d, r, n, rho, prec) for _ in range(3)]
        ws = kfb.Workspace()
        for k in range(3):
            Ms = [_to_dev(_batch(4, k, "A" if i % 2 else "G", n, d, prec=prec), dt) for i in range(3)]
            for f, M in zip(single, Ms):
                f.update(M)
            kfb.update_batched(grouped, Ms, ws)
        torch.cuda.synchronize()
        for a, b in zip(single, grouped):
            Ua, Da = a.front()
            Ub, Db = b.front()
            assert torch.equal(Ua, Ub) and torch.equal(Da, Db)


@pytest.mark.parametrize("dG,dA,rG,nG,rA,nA", [(768, 1024, 64, 64, 64, 64), (770, 1001, 64, 64, 64, 64),
                                                (768, 1024, 64, 64, 48, 32)])
@pytest.mark.parametrize("flags", [0, 1])
def test_mixed_precondition_on_loaded_state(kfb, flags, dG, dA, rG, nG, rA, nA):
    # BF16-MFMA apply on an oracle-built state (U in FP32, D in FP64), G FP32;
    # widths that are not multiples of 4 / 32 take the general BF16 kernel
    # (unaligned G rows, k not a whole number of tiles) with the coefficient
    # scalings in its epilogue; the last case has a different number of modes
    # on the two sides (the row and column coefficient vectors differ in length)
    import torch
    rho = 0.95
    _announce(f"mixed precondition flags={flags} dG={dG} dA={dA} ranks G {rG}+{nG} A {rA}+{nA}")
    bg = _oracle_state(dG, rG, nG, rho, 4, 31, "G")
    ba = _oracle_state(dA, rA, nA, rho, 4, 31, "A")
    fg = kfb.Factor(dG, rG, nG, rho, kfb.KFB_BF16_MIXED)
    fa = kfb.Factor(dA, rA, nA, rho, kfb.KFB_BF16_MIXED)
    UG32, UA32 = bg.U.astype(np.float32), ba.U.astype(np.float32)
    fg.load_state(_to_dev(UG32, torch.float32), _to_dev(bg.D, torch.float64), step=4)
    fa.load_state(_to_dev(UA32, torch.float32), _to_dev(ba.D, torch.float64), step=4)
    G = synth.grad_for(31, 0, dG, dA).astype(np.float32)
    Gd = _to_dev(G, torch.float32)
    S = torch.empty_like(Gd)
    lg, la = 0.01, 0.01
    kfb.precondition(fg, fa, Gd, S, lg, la, flags=flags)
    torch.cuda.synchronize()
    DG, DA, lgx, lax = bg.D, ba.D, lg, la
    if flags & 1:
        DG, lgx = oracle.spectrum_continuation(DG, lg)
        DA, lax = oracle.spectrum_continuation(DA, la)
    S_ref = oracle.precondition_lowrank(UG32.astype(np.float64), DG, UA32.astype(np.float64), DA,
                                        G.astype(np.float64), lgx, lax)
    es = oracle.e_S(S.cpu().numpy(), S_ref)
    ep = oracle.e_S_proj(S.cpu().numpy(), S_ref, bg.U, ba.U)
    _announce(f"  e_S {es:.3e} e_S_proj {ep:.3e}")
    assert es <= TOL[2] and ep <= TOL[2]


# ----------------------------------------------------------------------------
# FP64 core eigensolver with panels read from global memory (streamed
# configurations of the tuning table: 16- and 32-column blocks)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("bw", [16, 32])
@pytest.mark.parametrize("d,r,n,steps", [(300, 80, 70, 4), (400, 96, 96, 4), (1024, 256, 256, 3), (90, 40, 24, 3)])
def test_fp64_streamed_panel_eigensolver(kfb, d, r, n, steps, bw):
    import torch
    N = r + n
    if N < 4 * bw:
        pytest.skip("fewer than four blocks")
    kfb.tune_set_jacobi(kfb.KFB_FP64, N, kfb.KFB_JAC_STREAMED | bw)
    try:
        _announce(f"fp64 streamed-panel Jacobi bw={bw} d={d} r={r} n={n} N={N}")
        rho = 0.95
        f = kfb.Factor(d, r, n, rho, kfb.KFB_FP64)
        o = oracle.DenseFactor(d, r, rho)
        for k in range(steps):
            M = _batch(11, k, "A", n, d)
            f.update(_to_dev(M, torch.float64))
            o.update(M.T)
            U, D = _front_np(f)
            V, lamv = o.modes()
            er, ed, eo = oracle.e_rec_dense(U, D, o.X), oracle.e_D(D, lamv), oracle.e_orth(U)
            _announce(f"  step {k} e_rec {er:.3e} e_D {ed:.3e} orth {eo:.2e}")
            assert er <= 1e-10 and ed <= 1e-10 and eo <= 1e-11
        assert f.status() == 0
    finally:
        kfb.tune_set_jacobi(kfb.KFB_FP64, N, 0)


@pytest.mark.parametrize("d,r,n,steps", [(400, 96, 96, 5), (1024, 256, 256, 4), (700, 200, 150, 4)])
def test_fp32_streamed_panel_eigensolver(kfb, d, r, n, steps):
    # the FP32 form's core through the 32-column streamed-panel eigensolver on FP32
    # MFMA (main iteration, and the new-direction block's when n admits it), vs the
    # dense definition on the same FP32-rounded batches
    import torch
    N = r + n
    cfg = kfb.KFB_JAC_STREAMED | 32
    kfb.tune_set_jacobi(kfb.KFB_FP32, N, cfg)
    if n >= 128:
        kfb.tune_set_jacobi(kfb.KFB_FP32, n, cfg)
    try:
        _announce(f"fp32 streamed-panel Jacobi d={d} r={r} n={n} N={N}")
        rho = 0.95
        f = kfb.Factor(d, r, n, rho, kfb.KFB_FP32)
        o = oracle.DenseFactor(d, r, rho)
        for k in range(steps):
            M = _batch(12, k, "A" if k % 2 else "G", n, d)
            Mf = M.astype(np.float32).astype(np.float64)
            f.update(_to_dev(Mf, torch.float32))
            o.update(Mf.T)
            U, D = _front_np(f)
            V, lamv = o.modes()
            er, ed, eo = oracle.e_rec_dense(U, D, o.X), oracle.e_D(D, lamv), oracle.e_orth(U, D, rel_floor=1e-6)
            _announce(f"  step {k} e_rec {er:.3e} e_D {ed:.3e} orth {eo:.2e}")
            assert er <= TOL[1] and ed <= TOL[1] and eo <= 1e-4
        assert f.status() & kfb.KFB_EV_JACOBI_MAXSWEEPS == 0
    finally:
        kfb.tune_set_jacobi(kfb.KFB_FP32, N, 0)
        if n >= 128:
            kfb.tune_set_jacobi(kfb.KFB_FP32, n, 0)


@pytest.mark.parametrize("bw", [16, 32, 32 | 0x200])
def test_mixed_streamed_panel_headline_core(kfb, bw):
    # the headline shape's core (N = 512) through the streamed-panel eigensolvers (FP64
    # iteration; or, with KFB_JAC_REFINE, the FP32 iteration and the FP64 refinement), vs Oracle-B
    import torch
    d, r, n, rho, steps = 4096, 256, 256, 0.95, 3
    kfb.tune_set_jacobi(kfb.KFB_BF16_MIXED, r + n, kfb.KFB_JAC_STREAMED | bw)
    try:
        _announce(f"mixed streamed-panel bw={bw} d={d} r={r} n={n}")
        f = kfb.Factor(d, r, n, rho, kfb.KFB_BF16_MIXED)
        o = oracle.BrandFactor(d, r, rho)
        for k in range(steps):
            M = _batch(3, 200 + k, "A", n, d, prec=2)
            f.update(_to_dev(M, torch.bfloat16))
            o.update(M.T)
            U, D = _front_np(f)
            e = oracle.e_rec_lowrank(U, D, o.U, o.D)
            _announce(f"  step {k} e_rec {e:.3e} orth {oracle.e_orth(U):.2e}")
            assert e <= TOL[2]
        assert f.status() & kfb.KFB_EV_JACOBI_MAXSWEEPS == 0
    finally:
        kfb.tune_set_jacobi(kfb.KFB_BF16_MIXED, r + n, 0)


@pytest.mark.parametrize("dup", [False, True])
def test_mixed_refined_core_ragged_and_clustered(kfb, dup):
    # the mixed form's FP32 iteration + FP64 refinement at a core whose size is no
    # multiple of the panel (N = 350, new-direction block n = 150), and with every
    # batch column duplicated (a cluster of 75 zero eigenvalues that the refinement
    # only re-orthonormalises): vs Oracle-B, and vs the FP64 iteration on the same inputs
    import torch
    d, r, n, rho, steps = 700, 200, 150, 0.95, 4
    N = r + n
    res = {}
    for cfg in (kfb.KFB_JAC_STREAMED | kfb.KFB_JAC_REFINE | 32, kfb.KFB_JAC_STREAMED | 32):
        kfb.tune_set_jacobi(kfb.KFB_BF16_MIXED, N, cfg)
        try:
            _announce(f"mixed core cfg={cfg:#x} d={d} r={r} n={n} dup={dup}")
            f = kfb.Factor(d, r, n, rho, kfb.KFB_BF16_MIXED)
            o = oracle.BrandFactor(d, r, rho)
            out = []
            for k in range(steps):
                M = _batch(14, k, "G", n, d, prec=2)
                if dup:
                    M = np.concatenate([M[: n // 2], M[: n // 2]], axis=0)
                f.update(_to_dev(M, torch.bfloat16))
                o.update(M.T)
                U, D = _front_np(f)
                e, eo = oracle.e_rec_lowrank(U, D, o.U, o.D), oracle.e_orth(U, D, rel_floor=1e-6)
                _announce(f"  step {k} e_rec {e:.3e} orth {eo:.2e}")
                assert e <= TOL[2] and eo <= 1e-3
                out.append((U, D))
            assert f.status() & kfb.KFB_EV_JACOBI_MAXSWEEPS == 0
            res[cfg] = out
        finally:
            kfb.tune_set_jacobi(kfb.KFB_BF16_MIXED, N, 0)
    a_, b_ = res.values()
    for k, ((Ua, Da), (Ub, Db)) in enumerate(zip(a_, b_)):
        e = oracle.e_rec_lowrank(Ua, Da, Ub, Db)
        _announce(f"  step {k}: refined vs FP64 iteration {e:.3e}")
        assert e <= 1e-4


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_ortho_drift_is_reported(kfb, prec):
    # a clean trajectory never sets the drift bit; a basis loaded with columns scaled by
    # 1.01 (squared norms off by 0.02) carries the defect into the next update's basis
    import torch
    d, r, n, rho = 192, 16, 16, 0.95
    mdt = {0: torch.float64, 1: torch.float32, 2: torch.bfloat16}[prec]
    udt = torch.float64 if prec == 0 else torch.float32
    ddt = torch.float32 if prec == 1 else torch.float64
    _announce(f"ortho drift prec={prec}")
    f = kfb.Factor(d, r, n, rho, prec)
    for k in range(6):
        f.update(_to_dev(_batch(12, k, "A", n, d, prec=prec), mdt))
    assert f.status() & kfb.KFB_EV_ORTHO_DRIFT == 0
    b = _oracle_state(d, r, n, rho, 3, 13, "A")
    g = kfb.Factor(d, r, n, rho, prec)
    g.load_state(_to_dev(1.01 * b.U, udt), _to_dev(b.D, ddt), step=3)
    assert g.status() & kfb.KFB_EV_ORTHO_DRIFT          # the load's own column-norm check
    g.update(_to_dev(_batch(13, 3, "A", n, d, prec=prec), mdt))
    assert g.status() & kfb.KFB_EV_ORTHO_DRIFT          # carried into the updated basis


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_drift_recovery(kfb, prec):
    # a drifted basis (columns off unit norm and slightly mixed) is re-orthonormalised
    # without changing the matrix it stands for: against the oracle's Rayleigh-Ritz
    # of the same representation, orthonormal to the form's precision, and the next
    # update tracks Oracle-B started from the recovered state
    import torch
    d, r, n, rho = 320, 48, 32, 0.95
    mdt = {0: torch.float64, 1: torch.float32, 2: torch.bfloat16}[prec]
    udt = torch.float64 if prec == 0 else torch.float32
    ddt = torch.float32 if prec == 1 else torch.float64
    orth_tol = {0: 1e-13, 1: 1e-5, 2: 1e-4}[prec]
    _announce(f"drift recovery prec={prec}")
    b = _oracle_state(d, r, n, rho, 3, 15, "A")
    k = b.U.shape[1]
    mix = np.eye(k) + 0.01 * np.random.default_rng(16).standard_normal((k, k))
    Ud = (b.U @ mix).astype(np.float32 if prec else np.float64).astype(np.float64)
    Dd = b.D.astype(np.float32).astype(np.float64) if prec == 1 else b.D
    g = kfb.Factor(d, r, n, rho, prec)
    g.load_state(_to_dev(Ud, udt), _to_dev(Dd, ddt), step=3)
    assert g.status() & kfb.KFB_EV_ORTHO_DRIFT
    g.reorthonormalize()
    U, D = _front_np(g)
    Uo, Do = oracle.reorthonormalize(Ud, Dd)
    e = oracle.e_rec_lowrank(U, D, Uo, Do)
    _announce(f"  e_rec {e:.3e} e_D {oracle.e_D(D, Do):.3e} orth {oracle.e_orth(U):.3e}")
    assert e <= TOL[prec] and oracle.e_D(D, Do) <= TOL[prec]
    assert oracle.e_orth(U) <= orth_tol
    assert g.status() == 0
    assert g.info()["k_valid"] == k and g.info()["step"] == 3
    o = oracle.BrandFactor(d, r, rho)
    o.U, o.D, o.k = Uo, Do, 3
    M = _batch(15, 3, "A", n, d, prec=prec)
    g.update(_to_dev(M, mdt))
    o.update(M.T)
    U, D = _front_np(g)
    assert oracle.e_rec_lowrank(U, D, o.U, o.D) <= TOL[prec]
    assert g.status() == 0


def test_state_load_rejects_bad_eigenvalues(kfb):
    import torch
    d, r, n = 128, 8, 8
    f = kfb.Factor(d, r, n, 0.95, kfb.KFB_FP64)
    f.update(_to_dev(_batch(17, 0, "A", n, d), torch.float64))
    torch.cuda.synchronize()
    U0, D0 = _front_np(f)
    Q = np.linalg.qr(np.random.default_rng(3).standard_normal((d, 4)))[0]
    for bad in ([1.0, 2.0, 0.5, 0.1], [2.0, 1.0, -0.5, -1.0], [2.0, np.nan, 1.0, 0.5], [np.inf, 1.0, 0.5, 0.1]):
        with pytest.raises(kfb.KfbError):
            f.load_state(_to_dev(Q, torch.float64), _to_dev(np.array(bad), torch.float64), step=9)
    # the state is untouched by a rejected load
    U1, D1 = _front_np(f)
    assert f.info()["k_valid"] == n and f.info()["step"] == 1
    assert np.array_equal(U0, U1) and np.array_equal(D0, D1)
    f.load_state(_to_dev(Q, torch.float64), _to_dev(np.array([2.0, 1.0, 1.0, 0.0]), torch.float64), step=9)
    assert f.info()["k_valid"] == 4 and f.status() == 0


def test_batched_widths_argument_errors(kfb):
    import torch
    d, r, n = 128, 8, 16
    fs = [kfb.Factor(d, r, n, 0.95, kfb.KFB_FP64) for _ in range(2)]
    ws = kfb.Workspace()
    Ms = [torch.zeros((n, d), dtype=torch.float64, device=_dev()) for _ in range(2)]
    for bad in ([0, 4], [4, n + 1], [-3, 4]):
        with pytest.raises(kfb.KfbError):
            kfb.update_batched_widths(fs, Ms, bad, ws)
    kfb.update_batched_widths(fs, Ms, [n, 1], ws)   # zero batches: valid, state stays empty of energy
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec", [0, 2])
def test_batched_uneven_widths_equal_unpadded(kfb, prec):
    # batches of widths 40, 64, 25 zero-padded to 64 in one grouped call equal the
    # same updates run alone at their own widths (the padded modes carry eigenvalue 0)
    import torch
    d, r, nmax, rho = 256, 32, 64, 0.95
    widths = [40, 64, 25]
    mdt = torch.float64 if prec == 0 else torch.bfloat16
    tol = 1e-10 if prec == 0 else 1e-5
    _announce(f"uneven widths prec={prec}")
    padded = [kfb.Factor(d, r, nmax, rho, prec) for _ in widths]
    alone = [kfb.Factor(d, r, nmax, rho, prec) for _ in widths]
    ws = kfb.Workspace()
    worst = 0.0
    for k in range(4):
        Ms, Mp = [], []
        for i, w in enumerate(widths):
            M = _batch(14, 4 * k + i, "A" if i % 2 else "G", w, d, prec=prec)
            Md = _to_dev(M, mdt)
            P = torch.zeros((nmax, d), dtype=mdt, device=_dev())
            P[:w] = Md
            Ms.append(Md)
            Mp.append(P)
        kfb.update_batched_widths(padded, Mp, widths, ws)
        for f, Md in zip(alone, Ms):
            f.update(Md)
        for a, b in zip(padded, alone):
            Ua, Da = _front_np(a)
            Ub, Db = _front_np(b)
            worst = max(worst, oracle.e_rec_lowrank(Ua, Da, Ub, Db))
    _announce(f"  worst e_rec {worst:.3e}")
    assert worst <= tol
    for f in padded:
        assert f.status() & kfb.KFB_EV_CHOL_DEFICIENT == 0
        assert f.info()["k_valid"] == r + nmax     # the padded slots stay until the next truncation


@pytest.mark.parametrize("prec", [0, 2])
def test_cross_shape_grouped_update(kfb, prec):
    # factors of widths 512 / 1536 / 2048 / 1000 and ranks 128 / 128 / 200 / 96 in one
    # grouped call per step (batches of widths 128, 64, 100, 32), against the same
    # updates run one by one and against Oracle-B; the group's kept rank agrees at
    # every step (r_eff = min(k_valid, r)), the widths and batch widths do not
    import torch
    rho = 0.95
    shapes = [(512, 128, 128), (1536, 128, 128), (2048, 128, 128), (1000, 96, 128)]   # (d, r, n_max)
    widths = [128, 64, 100, 32]
    mdt = torch.float64 if prec == 0 else torch.bfloat16
    _announce(f"cross-shape grouped update prec={prec}")
    grouped = [kfb.Factor(d, r, nm, rho, prec) for d, r, nm in shapes]
    alone = [kfb.Factor(d, r, nm, rho, prec) for d, r, nm in shapes]
    orc = [oracle.BrandFactor(d, r, rho) for d, r, nm in shapes]
    ws = kfb.Workspace()
    worst = dict(alone=0.0, oracle=0.0)
    for k in range(4):
        # one grouped call per kept rank r_eff = min(k_valid, r): the three rank-128
        # factors of different widths share it from the second step on
        Ms, Md = [], []
        for i, (d, r, nm) in enumerate(shapes):
            M = _batch(19, 10 * k + i, "A" if i % 2 else "G", widths[i], d, prec=prec)
            Ms.append(M)
            Md.append(_to_dev(M, mdt))
        buckets = {}
        for i, f in enumerate(grouped):
            buckets.setdefault(min(f.info()["k_valid"], f.r), []).append(i)
        if k > 0:
            assert sorted(len(v) for v in buckets.values()) == [1, 3]
        for idx in buckets.values():
            kfb.update_grouped([grouped[i] for i in idx], [Md[i] for i in idx], ws)
        for f, o, M, Mh in zip(alone, orc, Md, Ms):
            f.update(M)
            o.update(Mh.T)
        for g, a, o in zip(grouped, alone, orc):
            Ug, Dg = _front_np(g)
            Ua, Da = _front_np(a)
            worst["alone"] = max(worst["alone"], oracle.e_rec_lowrank(Ug, Dg, Ua, Da))
            worst["oracle"] = max(worst["oracle"], oracle.e_rec_lowrank(Ug, Dg, o.U, o.D))
            keep = Dg > 0
            assert oracle.e_orth(Ug[:, keep]) <= TOL[prec]
    _announce(f"  {worst}")
    assert worst["oracle"] <= TOL[prec]
    assert worst["alone"] <= (1e-10 if prec == 0 else 1e-4)
    for g in grouped:
        assert g.status() & (kfb.KFB_EV_CHOL_DEFICIENT | kfb.KFB_EV_NONFINITE | kfb.KFB_EV_ORTHO_DRIFT) == 0


def test_gemm_tile_choice_does_not_change_results(kfb):
    # the BF16 products of the mixed apply with 128 or 256 output tiles (the
    # autotuner's two candidates): the k order of every sum is the same, so the
    # results are bit-identical; grouped two-sided and factored applications
    import torch
    from paper_2210_08494_amd import tune
    dG, dA, r, n, rho, lam = 1024, 1280, 128, 128, 0.95, 0.01
    _announce("gemm tile 128 vs 256")
    fgs, fas = [], []
    for i in range(3):
        bg = _oracle_state(dG, r, n, rho, 3, 50 + i, "G")
        ba = _oracle_state(dA, r, n, rho, 3, 60 + i, "A")
        fg = kfb.Factor(dG, r, n, rho, kfb.KFB_BF16_MIXED)
        fa = kfb.Factor(dA, r, n, rho, kfb.KFB_BF16_MIXED)
        fg.load_state(_to_dev(bg.U.astype(np.float32), torch.float32), _to_dev(bg.D, torch.float64), step=3)
        fa.load_state(_to_dev(ba.U.astype(np.float32), torch.float32), _to_dev(ba.D, torch.float64), step=3)
        fgs.append(fg)
        fas.append(fa)
    NG, NA = fgs[0].info()["k_valid"], fas[0].info()["k_valid"]
    Gs = [_to_dev(synth.grad_for(70 + i, 0, dG, dA).astype(np.float32), torch.float32) for i in range(3)]
    Gk = [_to_dev(synth.to_bf16_values(synth.batch_for(71, i, "G", n, dG)), torch.bfloat16) for i in range(3)]
    Ak = [_to_dev(synth.to_bf16_values(synth.batch_for(71, i, "A", n, dA)), torch.bfloat16) for i in range(3)]
    shapes = tune.precond_product_shapes(dG, dA, NG, NA) + tune.factored_product_shapes(dG, dA, n)
    ws = kfb.Workspace()
    out = {}
    try:
        for tile in (128, 256):
            for (m, nn, k) in shapes:
                kfb.tune_set_gemm(m, nn, k, tile)
                assert kfb.tune_get_gemm(m, nn, k) == tile
            S2 = [torch.empty_like(G) for G in Gs]
            SF = [torch.empty_like(G) for G in Gs]
            kfb.precondition_batched(fgs, fas, Gs, S2, [lam] * 3, [lam] * 3, 1, ws)
            kfb.precondition_factored_batched(fgs, fas, Gk, Ak, SF, [lam] * 3, [lam] * 3, 0, ws)
            torch.cuda.synchronize()
            out[tile] = (S2, SF)
    finally:
        for (m, nn, k) in shapes:
            kfb.tune_set_gemm(m, nn, k, 0)
    for a, b in zip(out[128][0] + out[128][1], out[256][0] + out[256][1]):
        assert torch.equal(a, b)
    with pytest.raises(kfb.KfbError):
        kfb.tune_set_gemm(64, 64, 64, 192)
