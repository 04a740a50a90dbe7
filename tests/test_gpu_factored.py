"""GPU parity of the factored (linear-cost) preconditioner, Algorithm 8.

The step for a layer gradient G_k A_k^T is formed from the two thin factors
without the gradient itself.  The FP64 form is checked against the dense
definition (Cholesky solves with the d x d regularised factors applied to the
explicit product G_k A_k^T, Section 2.1), the FP32 and BF16-mixed forms
against the oracle's factored form on the same (rounded) states; tolerances
1e-10 / 1e-5 / 2e-2 relative.  States come from the oracle and are loaded
through kfb_state_load, so the apply is tested in isolation.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2210_08494_amd import synth

pytestmark = pytest.mark.gpu


def _dev():
    import torch
    return torch.device("cuda:0")


def _to_dev(x, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(device=_dev(), dtype=dtype)


def _oracle_state(d, r, n, rho, steps, cfg, side, bias=False):
    b = oracle.BrandFactor(d, r, rho)
    for k in range(steps):
        b.update(synth.batch_for(cfg, k, side, n, d, bias=bias).T)
    return b


def _loaded(kfb, b, r, n, prec, udt, ddt):
    import torch
    f = kfb.Factor(b.U.shape[0], r, n, 0.95, prec)
    f.load_state(_to_dev(b.U, udt), _to_dev(b.D, ddt), step=3)
    return f


@pytest.mark.parametrize("flags", [0, 1, 2, 3, 5])
@pytest.mark.parametrize("nk", [12, 1, 37])
def test_fp64_factored_equals_dense_definition(kfb, flags, nk):
    import torch
    dG, dA, r, n, rho = 200, 300, 20, 12, 0.95
    print(f"fp64 factored flags={flags} n={nk}", flush=True)
    bg = _oracle_state(dG, r, n, rho, 4, 41, "G")
    ba = _oracle_state(dA, r, n, rho, 4, 41, "A")
    fg = _loaded(kfb, bg, r, n, kfb.KFB_FP64, torch.float64, torch.float64)
    fa = _loaded(kfb, ba, r, n, kfb.KFB_FP64, torch.float64, torch.float64)
    Gk = synth.batch_for(41, 9, "G", nk, dG)   # (n, d) rows = columns of G_k
    Ak = synth.batch_for(41, 9, "A", nk, dA)
    S = torch.full((dG, dA), float("nan"), device=_dev(), dtype=torch.float64)
    lg, la = 0.05, 0.2
    kfb.precondition_factored(fg, fa, _to_dev(Gk, torch.float64), _to_dev(Ak, torch.float64), S, lg, la,
                              flags=flags)
    # the two-sided apply of the explicit gradient on the same states
    J = Gk.T @ Ak
    S2 = torch.full_like(S, float("nan"))
    kfb.precondition(fg, fa, _to_dev(J, torch.float64), S2, lg, la, flags=flags)
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
    S_ref = oracle.precondition_dense(XG, XA, J, lgx, lax)
    Sg = S.cpu().numpy()
    assert oracle.e_S(Sg, S_ref) <= 1e-10
    assert oracle.e_S_proj(Sg, S_ref, UG, UA) <= 1e-10
    assert np.max(np.abs(Sg - S_ref)) <= 1e-10 * np.max(np.abs(S_ref))
    assert oracle.e_S(Sg, S2.cpu().numpy()) <= 1e-10


def test_fp32_factored_realistic_width(kfb):
    # d_in = 4097 (bias row), d_out = 4096, r = n = 256: N = 512 modes per side
    import torch
    dA, dG, r, n, rho, lam = 4097, 4096, 256, 256, 0.95, 0.01
    print(f"fp32 factored dA={dA} dG={dG}", flush=True)
    bg = _oracle_state(dG, r, n, rho, 3, 42, "G")
    ba = _oracle_state(dA, r, n, rho, 3, 42, "A", bias=True)
    UG, UA = bg.U.astype(np.float32), ba.U.astype(np.float32)
    DG, DA = bg.D.astype(np.float32), ba.D.astype(np.float32)
    fg = kfb.Factor(dG, r, n, rho, kfb.KFB_FP32)
    fa = kfb.Factor(dA, r, n, rho, kfb.KFB_FP32)
    fg.load_state(_to_dev(UG, torch.float32), _to_dev(DG, torch.float32), step=3)
    fa.load_state(_to_dev(UA, torch.float32), _to_dev(DA, torch.float32), step=3)
    # the factors of the last step's gradient: the batches the states were built from
    Gk = synth.batch_for(42, 2, "G", n, dG).astype(np.float32)
    Ak = synth.batch_for(42, 2, "A", n, dA, bias=True).astype(np.float32)
    S = torch.empty((dG, dA), device=_dev(), dtype=torch.float32)
    kfb.precondition_factored(fg, fa, _to_dev(Gk, torch.float32), _to_dev(Ak, torch.float32), S, lam, lam)
    torch.cuda.synchronize()
    S_ref = oracle.precondition_factored(UG.astype(np.float64), DG.astype(np.float64), UA.astype(np.float64),
                                         DA.astype(np.float64), Gk.T.astype(np.float64), Ak.T.astype(np.float64),
                                         lam, lam)
    es = oracle.e_S(S.cpu().numpy(), S_ref)
    ep = oracle.e_S_proj(S.cpu().numpy(), S_ref, bg.U, ba.U)
    print(f"  e_S {es:.3e} e_S_proj {ep:.3e}", flush=True)
    assert es <= 1e-5 and ep <= 1e-5


@pytest.mark.parametrize("flags", [0, 1])
def test_mixed_factored_headline_shape(kfb, flags):
    # d = 4096 both sides, r = n = 256; U FP32, D FP64, G_k and A_k BF16
    import torch
    d, r, n, rho, lam = 4096, 256, 256, 0.95, 0.01
    print(f"mixed factored d={d} flags={flags}", flush=True)
    bg = _oracle_state(d, r, n, rho, 3, 43, "G")
    ba = _oracle_state(d, r, n, rho, 3, 43, "A")
    UG, UA = bg.U.astype(np.float32), ba.U.astype(np.float32)
    fg = kfb.Factor(d, r, n, rho, kfb.KFB_BF16_MIXED)
    fa = kfb.Factor(d, r, n, rho, kfb.KFB_BF16_MIXED)
    fg.load_state(_to_dev(UG, torch.float32), _to_dev(bg.D, torch.float64), step=3)
    fa.load_state(_to_dev(UA, torch.float32), _to_dev(ba.D, torch.float64), step=3)
    Gk = synth.to_bf16_values(synth.batch_for(43, 2, "G", n, d))
    Ak = synth.to_bf16_values(synth.batch_for(43, 2, "A", n, d))
    S = torch.empty((d, d), device=_dev(), dtype=torch.float32)
    kfb.precondition_factored(fg, fa, _to_dev(Gk, torch.bfloat16), _to_dev(Ak, torch.bfloat16), S, lam, lam,
                              flags=flags)
    torch.cuda.synchronize()
    DG, DA, lgx, lax = bg.D, ba.D, lam, lam
    if flags & 1:
        DG, lgx = oracle.spectrum_continuation(DG, lam)
        DA, lax = oracle.spectrum_continuation(DA, lam)
    S_ref = oracle.precondition_factored(UG.astype(np.float64), DG, UA.astype(np.float64), DA, Gk.T, Ak.T,
                                         lgx, lax)
    es = oracle.e_S(S.cpu().numpy(), S_ref)
    ep = oracle.e_S_proj(S.cpu().numpy(), S_ref, bg.U, ba.U)
    print(f"  e_S {es:.3e} e_S_proj {ep:.3e}", flush=True)
    assert es <= 2e-2 and ep <= 2e-2


def test_factored_batched_equals_single(kfb):
    import torch
    dG, dA, r, n, nk = 256, 320, 24, 16, 20
    for prec, mdt, udt, ddt in ((kfb.KFB_FP64, torch.float64, torch.float64, torch.float64),
                                (kfb.KFB_FP32, torch.float32, torch.float32, torch.float32),
                                (kfb.KFB_BF16_MIXED, torch.bfloat16, torch.float32, torch.float64)):
        print(f"factored batched == single, prec={prec}", flush=True)
        fgs, fas, Gks, Aks = [], [], [], []
        for i in range(3):
            bg = _oracle_state(dG, r, n, 0.95, 3, 50 + i, "G")
            ba = _oracle_state(dA, r, n, 0.95, 3, 50 + i, "A")
            fgs.append(_loaded(kfb, bg, r, n, prec, udt, ddt))
            fas.append(_loaded(kfb, ba, r, n, prec, udt, ddt))
            Gks.append(_to_dev(synth.batch_for(60 + i, 0, "G", nk, dG), mdt))
            Aks.append(_to_dev(synth.batch_for(60 + i, 0, "A", nk, dA), mdt))
        sdt = torch.float64 if prec == kfb.KFB_FP64 else torch.float32
        single = [torch.empty((dG, dA), device=_dev(), dtype=sdt) for _ in range(3)]
        grouped = [torch.empty((dG, dA), device=_dev(), dtype=sdt) for _ in range(3)]
        lg, la = [0.01, 0.02, 0.05], [0.03, 0.01, 0.1]
        for i in range(3):
            kfb.precondition_factored(fgs[i], fas[i], Gks[i], Aks[i], single[i], lg[i], la[i])
        kfb.precondition_factored_batched(fgs, fas, Gks, Aks, grouped, lg, la, 0, kfb.Workspace())
        torch.cuda.synchronize()
        for a, b in zip(single, grouped):
            assert torch.equal(a, b)


def test_factored_argument_errors(kfb):
    import torch
    lib = kfb.load()
    d, r, n = 64, 8, 8
    fg = kfb.Factor(d, r, n, 0.95, kfb.KFB_FP64)
    fa = kfb.Factor(d, r, n, 0.95, kfb.KFB_FP64)
    X = torch.zeros((n, d), device=_dev(), dtype=torch.float64)
    S = torch.zeros((d, d), device=_dev(), dtype=torch.float64)
    ws = torch.zeros(1 << 20, device=_dev(), dtype=torch.uint8)
    p = ctypes.c_void_p

    def call(h1, h2, nk, Sp=S.data_ptr(), lam=0.1, ld=d):
        return lib.kfb_precondition_factored(h1, h2, p(X.data_ptr()), ld, p(X.data_ptr()), ld, nk, p(Sp), d,
                                             lam, lam, 0, p(ws.data_ptr()), ws.numel(), None)
    assert lib.kfb_precondition_factored_workspace_bytes(fg.handle, fa.handle, 0) == 0
    assert call(fg.handle, fa.handle, n) == 5            # KFB_EEMPTY: no modes yet
    b = _oracle_state(d, r, n, 0.95, 2, 70, "A")
    fg.load_state(_to_dev(b.U, torch.float64), _to_dev(b.D, torch.float64), step=2)
    fa.load_state(_to_dev(b.U, torch.float64), _to_dev(b.D, torch.float64), step=2)
    assert call(fg.handle, fa.handle, 0) == 1            # n < 1
    assert call(fg.handle, fa.handle, n, lam=0.0) == 1   # lam <= 0
    assert call(fg.handle, fa.handle, n, ld=d - 1) == 1  # leading dimension below d
    assert call(fg.handle, fa.handle, n, Sp=X.data_ptr()) == 1  # S aliases the factors
    assert call(fg.handle, fg.handle, n) == 4            # the same state on both sides
    assert call(fg.handle, fa.handle, n) == 0
    torch.cuda.synchronize()
