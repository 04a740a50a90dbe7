"""Thin ctypes binding of the kfb C-ABI (include/kfb.h).

Argument marshalling only: every step of the Brand update and of the inverse
application runs in the HIP kernels of libkfb.so.  PyTorch supplies device
memory (caller-owned state buffers and workspaces) and the current stream.
There is no CPU fallback: if the library is missing, load() raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkfb.so")

KFB_FP64, KFB_FP32, KFB_BF16_MIXED = 0, 1, 2
KFB_SPECTRUM_CONTINUATION, KFB_TRUNCATE_AFTER, KFB_RELATIVE_DAMPING = 1, 2, 4
KFB_EV_NONFINITE, KFB_EV_CHOL_DEFICIENT, KFB_EV_JACOBI_MAXSWEEPS, KFB_EV_ORTHO_DRIFT = 1, 2, 4, 8
KFB_JAC_STREAMED = 0x100
KFB_JAC_REFINE = 0x200
ERRORS = {0: "KFB_OK", 1: "KFB_EINVAL", 2: "KFB_EWORKSPACE", 3: "KFB_EHIP", 4: "KFB_ESTATE",
          5: "KFB_EEMPTY"}

_lib = None
_vp, _sz, _i32, _i64, _u32, _dbl = (ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64,
                                    ctypes.c_uint32, ctypes.c_double)

_SIGS = {
    "kfb_state_bytes": (_sz, [_i64, _i32, _i32, _i32]),
    "kfb_state_create": (ctypes.c_int, [ctypes.POINTER(_vp), _i64, _i32, _i32, _dbl, _i32, _vp, _sz, _vp]),
    "kfb_destroy": (ctypes.c_int, [_vp]),
    "kfb_update_workspace_bytes": (_sz, [_vp, _i32]),
    "kfb_brand_update": (ctypes.c_int, [_vp, _vp, _i64, _i32, _vp, _sz, _vp]),
    "kfb_scratch_bytes": (_sz, []),
    "kfb_brand_update_scratch": (ctypes.c_int, [_vp, _vp, _i64, _i32, _vp]),
    "kfb_update_batched_workspace_bytes": (_sz, [_i32, ctypes.POINTER(_vp), _i32]),
    "kfb_brand_update_batched": (ctypes.c_int, [_i32, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _i64, _i32,
                                                _vp, _sz, _vp]),
    "kfb_brand_update_batched_widths": (ctypes.c_int, [_i32, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _i64, _i32,
                                                       ctypes.POINTER(_i32), _vp, _sz, _vp]),
    "kfb_update_grouped_workspace_bytes": (_sz, [_i32, ctypes.POINTER(_vp), ctypes.POINTER(_i32)]),
    "kfb_brand_update_grouped": (ctypes.c_int, [_i32, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                                ctypes.POINTER(_i64), ctypes.POINTER(_i32), _vp, _sz, _vp]),
    "kfb_precondition_workspace_bytes": (_sz, [_vp, _vp]),
    "kfb_precondition": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _i64, _dbl, _dbl, _u32, _vp, _sz, _vp]),
    "kfb_precondition_batched_workspace_bytes": (_sz, [_i32, ctypes.POINTER(_vp), ctypes.POINTER(_vp)]),
    "kfb_precondition_batched": (ctypes.c_int, [_i32, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                                ctypes.POINTER(_vp), _i64, ctypes.POINTER(_vp), _i64,
                                                ctypes.POINTER(_dbl), ctypes.POINTER(_dbl), _u32, _vp, _sz,
                                                _vp]),
    "kfb_precondition_factored_workspace_bytes": (_sz, [_vp, _vp, _i32]),
    "kfb_precondition_factored": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _i64, _i32, _vp, _i64, _dbl, _dbl,
                                                 _u32, _vp, _sz, _vp]),
    "kfb_precondition_factored_batched_workspace_bytes": (_sz, [_i32, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                                                _i32]),
    "kfb_precondition_factored_batched": (ctypes.c_int, [_i32, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                                         ctypes.POINTER(_vp), _i64, ctypes.POINTER(_vp), _i64,
                                                         _i32, ctypes.POINTER(_vp), _i64, ctypes.POINTER(_dbl),
                                                         ctypes.POINTER(_dbl), _u32, _vp, _sz, _vp]),
    "kfb_dense_bytes": (_sz, [_i64, _i64, _i32]),
    "kfb_dense_update_workspace_bytes": (_sz, []),
    "kfb_dense_update": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _i32, _i32, _vp, _sz, _vp]),
    "kfb_rsvd_workspace_bytes": (_sz, [_vp, _i32]),
    "kfb_rsvd_overwrite": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _i32, _i32, _vp, _sz, _vp]),
    "kfb_correct_workspace_bytes": (_sz, [_vp, _i32]),
    "kfb_light_correction": (ctypes.c_int, [_vp, _vp, _i64, ctypes.POINTER(_i32), _i32, _vp, _sz, _vp]),
    "kfb_state_info": (ctypes.c_int, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                                      ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "kfb_state_front": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_i64), ctypes.POINTER(_vp)]),
    "kfb_state_load": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i32, _i64, _vp]),
    "kfb_state_status": (ctypes.c_int, [_vp, ctypes.POINTER(_u32), _vp]),
    "kfb_reorth_workspace_bytes": (_sz, [_vp]),
    "kfb_reorthonormalize": (ctypes.c_int, [_vp, _vp, _sz, _vp]),
    "kfb_tune_set_jacobi": (ctypes.c_int, [_i32, _i32, _i32]),
    "kfb_tune_get_jacobi": (ctypes.c_int, [_i32, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "kfb_tune_set_gemm": (ctypes.c_int, [_i32, _i32, _i32, _i32]),
    "kfb_tune_get_gemm": (ctypes.c_int, [_i32, _i32, _i32, ctypes.POINTER(_i32)]),
    "kfb_profile_enable": (ctypes.c_int, [ctypes.c_int]),
    "kfb_profile_report": (ctypes.c_int, [ctypes.c_char_p, _sz, ctypes.c_int]),
    "kfb_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "kfb_build_info": (ctypes.c_char_p, []),
}
EXPORTS = tuple(_SIGS)


class KfbError(RuntimeError):
    pass


def load(path: str | None = None):
    """Load libkfb.so (built in-tree by __graft_entry__.build()); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise KfbError(f"{p} not found: the HIP library must be built (python -c "
                       "'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(p)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(rc: int, what: str):
    if rc != 0:
        raise KfbError(f"{what} failed: {ERRORS.get(rc, rc)} ({load().kfb_strerror(rc).decode()})")


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------
# Same-named wrappers of the C-ABI (pointers are ints or tensors)
# ---------------------------------------------------------------------------
def kfb_state_bytes(d, r, n_max, prec) -> int:
    return int(load().kfb_state_bytes(d, r, n_max, prec))


class Workspace:
    """A growable device byte buffer (256-byte aligned by the PyTorch allocator)."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf = None

    def get(self, nbytes: int):
        import torch
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.device)
        return self.buf


def _dtype_of(prec):
    import torch
    return torch.float64 if prec == KFB_FP64 else torch.float32


def _ddtype_of(prec):
    import torch
    return torch.float32 if prec == KFB_FP32 else torch.float64


def _mdtype_of(prec):
    import torch
    return {KFB_FP64: torch.float64, KFB_FP32: torch.float32, KFB_BF16_MIXED: torch.bfloat16}[prec]


class Factor:
    """One K-factor state (caller-owned buffer) behind a kfb handle."""

    def __init__(self, d: int, r: int, n_max: int, rho: float, prec: int, device="cuda"):
        import torch
        lib = load()
        self.d, self.r, self.n_max, self.rho, self.prec = int(d), int(r), int(n_max), float(rho), int(prec)
        nbytes = lib.kfb_state_bytes(self.d, self.r, self.n_max, self.prec)
        if nbytes == 0:
            raise KfbError(f"invalid state sizes d={d} r={r} n_max={n_max}")
        self.buf = torch.zeros(int(nbytes), dtype=torch.uint8, device=device)
        self.handle = ctypes.c_void_p()
        _check(lib.kfb_state_create(ctypes.byref(self.handle), self.d, self.r, self.n_max, self.rho,
                                    self.prec, _ptr(self.buf), int(nbytes), _stream()), "kfb_state_create")
        self.ws = Workspace(device)

    def __del__(self):
        try:
            if getattr(self, "handle", None) and _lib is not None:
                _lib.kfb_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    @property
    def mdtype(self):
        return _mdtype_of(self.prec)

    def info(self):
        k, s, d, r, nm, pr = _i32(), _i64(), _i64(), _i32(), _i32(), _i32()
        _check(load().kfb_state_info(self.handle, ctypes.byref(k), ctypes.byref(s), ctypes.byref(d),
                                     ctypes.byref(r), ctypes.byref(nm), ctypes.byref(pr)), "kfb_state_info")
        return dict(k_valid=k.value, step=s.value, d=d.value, r=r.value, n_max=nm.value, prec=pr.value)

    def update(self, M, ws: Workspace | None = None):
        """M: device tensor of shape (n, d) (= column-major d x n), dtype per precision."""
        lib = load()
        _batch_check(M, self, "update")
        n = int(M.shape[0])
        need = lib.kfb_update_workspace_bytes(self.handle, n)
        if need == 0:
            raise KfbError("kfb_update_workspace_bytes rejected the shape")
        w = (ws or self.ws).get(need)
        _check(lib.kfb_brand_update(self.handle, _ptr(M), int(M.stride(0)), n, _ptr(w), int(w.numel()),
                                    _stream()), "kfb_brand_update")

    def front(self):
        """(U, D) device views of the current modes: U (d x k), D (k,)."""
        import torch
        lib = load()
        up, ld, dp = _vp(), _i64(), _vp()
        _check(lib.kfb_state_front(self.handle, ctypes.byref(up), ctypes.byref(ld), ctypes.byref(dp)),
               "kfb_state_front")
        k = self.info()["k_valid"]
        base = self.buf.data_ptr()
        dt, ddt = _dtype_of(self.prec), _ddtype_of(self.prec)
        es, des = torch.tensor([], dtype=dt).element_size(), torch.tensor([], dtype=ddt).element_size()
        uoff, doff = up.value - base, dp.value - base
        ldu = ld.value
        Ucols = self.buf[uoff:uoff + max(k, 1) * ldu * es].view(dt).view(max(k, 1), ldu)[:k, :self.d]
        D = self.buf[doff:doff + max(k, 1) * des].view(ddt)[:k]
        return Ucols.t(), D

    def load_state(self, U, D, step: int = 1):
        """Overwrite with (U: d x k device tensor in the state's dtype, D: k)."""
        lib = load()
        if not (U.is_cuda and D.is_cuda and U.dim() == 2 and U.shape[0] == self.d and D.dim() == 1
                and D.shape[0] == U.shape[1] and U.dtype == _dtype_of(self.prec) and D.dtype == _ddtype_of(self.prec)):
            raise KfbError(f"load_state: expected U ({self.d}, k) {_dtype_of(self.prec)} and D (k,) "
                           f"{_ddtype_of(self.prec)} device tensors")
        Uc = U.t().contiguous()  # k x d rows = columns of U
        k = int(Uc.shape[0])
        Dc = D.contiguous()
        _check(lib.kfb_state_load(self.handle, _ptr(Uc), int(Uc.stride(0)), _ptr(Dc), k, int(step), _stream()),
               "kfb_state_load")
        import torch
        torch.cuda.current_stream().synchronize()

    def reorthonormalize(self, ws: Workspace | None = None):
        """Drift recovery: the same matrix on an orthonormal basis (Rayleigh-Ritz on span(U))."""
        lib = load()
        need = lib.kfb_reorth_workspace_bytes(self.handle)
        if need == 0:
            raise KfbError("kfb_reorth_workspace_bytes rejected the state (no modes, or more than 2048)")
        w = (ws or self.ws).get(need)
        _check(lib.kfb_reorthonormalize(self.handle, _ptr(w), int(w.numel()), _stream()), "kfb_reorthonormalize")

    def status(self) -> int:
        ev = _u32()
        _check(load().kfb_state_status(self.handle, ctypes.byref(ev), _stream()), "kfb_state_status")
        return ev.value


def _batch_check(M, f: "Factor", what: str):
    """A batch (or gradient factor) of the state f: (n, d) on f's device (the device of its state
    buffer), f's batch dtype, rows contiguous."""
    if not (M.dim() == 2 and M.shape[1] == f.d and M.dtype == f.mdtype and M.stride(1) == 1
            and M.shape[0] >= 1 and M.device == f.buf.device):
        raise KfbError(f"{what}: expected a ({'n'}, {f.d}) {f.mdtype} tensor with unit column stride on "
                       f"{f.buf.device}, got {tuple(M.shape)} {M.dtype} strides {tuple(M.stride())} on {M.device}")


def _grad_check(X, fg: "Factor", fa: "Factor", what: str):
    """A layer gradient or step: (d_out, d_in) = (fg.d, fa.d), rows contiguous, on the states'
    device, double in the FP64 form and float otherwise."""
    dt = _dtype_of(fg.prec)
    if not (X.dim() == 2 and tuple(X.shape) == (fg.d, fa.d) and X.stride(1) == 1
            and X.stride(0) >= fa.d and X.dtype == dt and X.device == fg.buf.device):
        raise KfbError(f"{what}: expected a ({fg.d}, {fa.d}) {dt} tensor with unit column stride on "
                       f"{fg.buf.device}, got {tuple(X.shape)} {X.dtype} strides {tuple(X.stride())} on {X.device}")


def _pair_check(fg: "Factor", fa: "Factor", what: str):
    if fg is fa or fg.prec != fa.prec or fg.buf.device != fa.buf.device:
        raise KfbError(f"{what}: the two sides must be distinct states of one precision form on one device")


def precondition(fg: Factor, fa: Factor, G, S, lam_g: float, lam_a: float, flags: int = 0,
                 ws: Workspace | None = None):
    """S = (Gamma~ + lam_g I)^{-1} G (A~ + lam_a I)^{-1}; G, S row-major (d_out, d_in) device tensors."""
    lib = load()
    _pair_check(fg, fa, "precondition")
    _grad_check(G, fg, fa, "precondition (G)")
    _grad_check(S, fg, fa, "precondition (S)")
    need = lib.kfb_precondition_workspace_bytes(fg.handle, fa.handle)
    if need == 0:
        raise KfbError("kfb_precondition_workspace_bytes rejected the states")
    w = (ws or fg.ws).get(need)
    _check(lib.kfb_precondition(fg.handle, fa.handle, _ptr(G), int(G.stride(0)), _ptr(S), int(S.stride(0)),
                                float(lam_g), float(lam_a), int(flags), _ptr(w), int(w.numel()), _stream()),
           "kfb_precondition")


def _same_layout(ts, what: str, count: int):
    """The grouped calls take one shape and leading dimension for all problems:
    check every tensor against the first before any pointer reaches the library."""
    if len(ts) != count:
        raise KfbError(f"{what}: {len(ts)} tensors for {count} problems")
    t0 = ts[0]
    for t in ts:
        if t.dim() != 2 or t.shape != t0.shape or t.stride() != t0.stride() or t.dtype != t0.dtype \
                or t.stride(1) != 1:
            raise KfbError(f"{what}: every tensor must be 2-D, row-contiguous and share shape, strides and dtype")


def update_batched(factors, Ms, ws: Workspace):
    """One grouped launch sequence updating every factor with its batch (same shape bucket)."""
    lib = load()
    cnt = len(factors)
    _same_layout(Ms, "update_batched", cnt)
    for f, M in zip(factors, Ms):
        _batch_check(M, f, "update_batched")
    hs = (_vp * cnt)(*[f.handle.value for f in factors])
    ms = (_vp * cnt)(*[m.data_ptr() for m in Ms])
    n = int(Ms[0].shape[0])
    need = lib.kfb_update_batched_workspace_bytes(cnt, hs, n)
    if need == 0:
        raise KfbError("kfb_update_batched_workspace_bytes rejected the bucket")
    w = ws.get(need)
    _check(lib.kfb_brand_update_batched(cnt, hs, ms, int(Ms[0].stride(0)), n, _ptr(w), int(w.numel()),
                                        _stream()), "kfb_brand_update_batched")


def update_batched_widths(factors, Ms, widths, ws: Workspace):
    """Grouped update of batches padded with zero columns to a common n; widths[i] = real columns of Ms[i]."""
    lib = load()
    cnt = len(factors)
    _same_layout(Ms, "update_batched_widths", cnt)
    for f, M in zip(factors, Ms):
        _batch_check(M, f, "update_batched_widths")
    if len(widths) != cnt:
        raise KfbError(f"update_batched_widths: {len(widths)} widths for {cnt} problems")
    hs = (_vp * cnt)(*[f.handle.value for f in factors])
    ms = (_vp * cnt)(*[m.data_ptr() for m in Ms])
    ws_ = (_i32 * cnt)(*[int(x) for x in widths])
    n = int(Ms[0].shape[0])
    need = lib.kfb_update_batched_workspace_bytes(cnt, hs, n)
    if need == 0:
        raise KfbError("kfb_update_batched_workspace_bytes rejected the bucket")
    w = ws.get(need)
    _check(lib.kfb_brand_update_batched_widths(cnt, hs, ms, int(Ms[0].stride(0)), n, ws_, _ptr(w), int(w.numel()),
                                               _stream()), "kfb_brand_update_batched_widths")


def update_grouped(factors, Ms, ws: Workspace):
    """One grouped launch sequence over factors of different widths (same precision form and
    kept rank); Ms[i]: (n_i, d_i) batch of factors[i] in its dtype, rows contiguous."""
    lib = load()
    cnt = len(factors)
    if len(Ms) != cnt or cnt < 1:
        raise KfbError(f"update_grouped: {len(Ms)} batches for {cnt} problems")
    for f, M in zip(factors, Ms):
        _batch_check(M, f, "update_grouped")
    hs = (_vp * cnt)(*[f.handle.value for f in factors])
    ms = (_vp * cnt)(*[m.data_ptr() for m in Ms])
    lds = (_i64 * cnt)(*[int(m.stride(0)) for m in Ms])
    wd = (_i32 * cnt)(*[int(m.shape[0]) for m in Ms])
    need = lib.kfb_update_grouped_workspace_bytes(cnt, hs, wd)
    if need == 0:
        raise KfbError("kfb_update_grouped_workspace_bytes rejected the group")
    w = ws.get(need)
    _check(lib.kfb_brand_update_grouped(cnt, hs, ms, lds, wd, _ptr(w), int(w.numel()), _stream()),
           "kfb_brand_update_grouped")


def precondition_batched(fgs, fas, Gs, Ss, lam_g, lam_a, flags, ws: Workspace):
    lib = load()
    cnt = len(fgs)
    _same_layout(Gs, "precondition_batched (G)", cnt)
    _same_layout(Ss, "precondition_batched (S)", cnt)
    if len(fas) != cnt or len(lam_g) != cnt or len(lam_a) != cnt:
        raise KfbError("precondition_batched: one A state and one lambda per side for every layer")
    for fg, fa, G, S in zip(fgs, fas, Gs, Ss):
        _pair_check(fg, fa, "precondition_batched")
        _grad_check(G, fg, fa, "precondition_batched (G)")
        _grad_check(S, fg, fa, "precondition_batched (S)")
    hg = (_vp * cnt)(*[f.handle.value for f in fgs])
    ha = (_vp * cnt)(*[f.handle.value for f in fas])
    gp = (_vp * cnt)(*[g.data_ptr() for g in Gs])
    sp = (_vp * cnt)(*[s.data_ptr() for s in Ss])
    lg = (_dbl * cnt)(*[float(x) for x in lam_g])
    la = (_dbl * cnt)(*[float(x) for x in lam_a])
    need = lib.kfb_precondition_batched_workspace_bytes(cnt, hg, ha)
    if need == 0:
        raise KfbError("kfb_precondition_batched_workspace_bytes rejected the bucket")
    w = ws.get(need)
    _check(lib.kfb_precondition_batched(cnt, hg, ha, gp, int(Gs[0].stride(0)), sp, int(Ss[0].stride(0)), lg, la,
                                        int(flags), _ptr(w), int(w.numel()), _stream()),
           "kfb_precondition_batched")


def _factor_arg(X, f: "Factor", what: str = "gradient factor"):
    _batch_check(X, f, what)
    return int(X.shape[0]), int(X.stride(0))


def precondition_factored(fg: Factor, fa: Factor, Gk, Ak, S, lam_g: float, lam_a: float, flags: int = 0,
                          ws: Workspace | None = None):
    """S = [(Gamma~ + lam_g I)^{-1} G_k] [(A~ + lam_a I)^{-1} A_k]^T (Algorithm 8).

    Gk: (n, d_out) and Ak: (n, d_in) device tensors (= d x n column-major), the
    state's batch dtype; S row-major (d_out, d_in)."""
    lib = load()
    _pair_check(fg, fa, "precondition_factored")
    n, ldgk = _factor_arg(Gk, fg, "precondition_factored (G_k)")
    n2, ldak = _factor_arg(Ak, fa, "precondition_factored (A_k)")
    if n != n2:
        raise KfbError(f"precondition_factored: G_k has {n} columns, A_k {n2}")
    _grad_check(S, fg, fa, "precondition_factored (S)")
    need = lib.kfb_precondition_factored_workspace_bytes(fg.handle, fa.handle, n)
    if need == 0:
        raise KfbError("kfb_precondition_factored_workspace_bytes rejected the states")
    w = (ws or fg.ws).get(need)
    _check(lib.kfb_precondition_factored(fg.handle, fa.handle, _ptr(Gk), ldgk, _ptr(Ak), ldak, n, _ptr(S),
                                         int(S.stride(0)), float(lam_g), float(lam_a), int(flags), _ptr(w),
                                         int(w.numel()), _stream()), "kfb_precondition_factored")


def precondition_factored_batched(fgs, fas, Gks, Aks, Ss, lam_g, lam_a, flags, ws: Workspace):
    lib = load()
    cnt = len(fgs)
    _same_layout(Gks, "precondition_factored_batched (G_k)", cnt)
    _same_layout(Aks, "precondition_factored_batched (A_k)", cnt)
    _same_layout(Ss, "precondition_factored_batched (S)", cnt)
    if len(fas) != cnt or len(lam_g) != cnt or len(lam_a) != cnt:
        raise KfbError("precondition_factored_batched: one A state and one lambda per side for every layer")
    for fg, fa, Gk, Ak, S in zip(fgs, fas, Gks, Aks, Ss):
        _pair_check(fg, fa, "precondition_factored_batched")
        _batch_check(Gk, fg, "precondition_factored_batched (G_k)")
        _batch_check(Ak, fa, "precondition_factored_batched (A_k)")
        _grad_check(S, fg, fa, "precondition_factored_batched (S)")
    n, ldgk = _factor_arg(Gks[0], fgs[0])
    n2, ldak = _factor_arg(Aks[0], fas[0])
    if n != n2:
        raise KfbError(f"precondition_factored_batched: G_k has {n} columns, A_k {n2}")
    hg = (_vp * cnt)(*[f.handle.value for f in fgs])
    ha = (_vp * cnt)(*[f.handle.value for f in fas])
    gp = (_vp * cnt)(*[g.data_ptr() for g in Gks])
    ap = (_vp * cnt)(*[a.data_ptr() for a in Aks])
    sp = (_vp * cnt)(*[s.data_ptr() for s in Ss])
    lg = (_dbl * cnt)(*[float(x) for x in lam_g])
    la = (_dbl * cnt)(*[float(x) for x in lam_a])
    need = lib.kfb_precondition_factored_batched_workspace_bytes(cnt, hg, ha, n)
    if need == 0:
        raise KfbError("kfb_precondition_factored_batched_workspace_bytes rejected the bucket")
    w = ws.get(need)
    _check(lib.kfb_precondition_factored_batched(cnt, hg, ha, gp, ldgk, ap, ldak, n, sp, int(Ss[0].stride(0)),
                                                 lg, la, int(flags), _ptr(w), int(w.numel()), _stream()),
           "kfb_precondition_factored_batched")


def _dense_check(X, f: "Factor", what: str):
    dt = _dtype_of(f.prec)
    if not (X.dim() == 2 and tuple(X.shape) == (f.d, f.d) and X.stride(1) == 1
            and X.stride(0) >= f.d and X.dtype == dt and X.device == f.buf.device):
        raise KfbError(f"{what}: expected a ({f.d}, {f.d}) {dt} dense factor on {f.buf.device}, got "
                       f"{tuple(X.shape)} {X.dtype} on {X.device}")


def dense_factor(f: Factor, device="cuda"):
    """A zeroed dense EA factor for the state f (d x d; row j of the tensor is column j)."""
    import torch
    return torch.zeros((f.d, f.d), dtype=_dtype_of(f.prec), device=device)


def dense_update(f: Factor, X, M, first: bool, ws: Workspace | None = None):
    """X <- rho X + (1 - rho)/n M M^T (first: M M^T / n), B-R-KFAC's dense EA factor of f."""
    lib = load()
    _dense_check(X, f, "dense_update")
    n, ldm = _factor_arg(M, f, "dense_update (M)")
    w = (ws or f.ws).get(lib.kfb_dense_update_workspace_bytes())
    _check(lib.kfb_dense_update(f.handle, _ptr(X), int(X.stride(0)), _ptr(M), ldm, n, 1 if first else 0, _ptr(w),
                                int(w.numel()), _stream()), "kfb_dense_update")


def rsvd_overwrite(f: Factor, X, Omega, oversample: int, power_its: int, ws: Workspace | None = None):
    """(U, D) of f <- the rank-r randomized SVD of X with the sketch Omega ((r + oversample, d) tensor)."""
    lib = load()
    _dense_check(X, f, "rsvd_overwrite")
    if not (Omega.is_cuda and Omega.dim() == 2 and tuple(Omega.shape) == (f.r + oversample, f.d)
            and Omega.stride(1) == 1 and Omega.dtype == X.dtype and Omega.device == X.device):
        raise KfbError(f"rsvd_overwrite: Omega must be a ({f.r + oversample}, {f.d}) {X.dtype} tensor "
                       f"with unit column stride on {X.device}")
    need = lib.kfb_rsvd_workspace_bytes(f.handle, int(oversample))
    if need == 0:
        raise KfbError("kfb_rsvd_workspace_bytes rejected the sizes")
    w = (ws or f.ws).get(need)
    _check(lib.kfb_rsvd_overwrite(f.handle, _ptr(X), int(X.stride(0)), _ptr(Omega), int(Omega.stride(0)),
                                  int(oversample), int(power_its), _ptr(w), int(w.numel()), _stream()),
           "kfb_rsvd_overwrite")


def light_correction(f: Factor, X, col_idx, ws: Workspace | None = None):
    """B-KFAC-C (Algorithm 6): correct the modes col_idx (host ints) of f against the dense EA factor X."""
    lib = load()
    _dense_check(X, f, "light_correction")
    idx = [int(i) for i in col_idx]
    arr = (_i32 * len(idx))(*idx)
    need = lib.kfb_correct_workspace_bytes(f.handle, len(idx))
    if need == 0:
        raise KfbError("kfb_correct_workspace_bytes rejected the sizes")
    w = (ws or f.ws).get(need)
    _check(lib.kfb_light_correction(f.handle, _ptr(X), int(X.stride(0)), arr, len(idx), _ptr(w), int(w.numel()),
                                    _stream()), "kfb_light_correction")


def profile_enable(on: bool = True):
    _check(load().kfb_profile_enable(1 if on else 0), "kfb_profile_enable")


def profile_report(reset: bool = True) -> dict:
    """Stage timings recorded while profiling was enabled: {stage: {calls, launches, ms}}."""
    import json
    buf = ctypes.create_string_buffer(1 << 16)
    _check(load().kfb_profile_report(buf, len(buf), 1 if reset else 0), "kfb_profile_report")
    return json.loads(buf.value.decode() or "{}")


def tune_set_jacobi(prec: int, N: int, bw: int):
    _check(load().kfb_tune_set_jacobi(int(prec), int(N), int(bw)), "kfb_tune_set_jacobi")


def tune_get_jacobi(prec: int, N: int):
    bw, Np = _i32(), _i32()
    _check(load().kfb_tune_get_jacobi(int(prec), int(N), ctypes.byref(bw), ctypes.byref(Np)), "kfb_tune_get_jacobi")
    return bw.value, Np.value


def tune_set_gemm(m: int, n: int, k: int, tile: int):
    _check(load().kfb_tune_set_gemm(int(m), int(n), int(k), int(tile)), "kfb_tune_set_gemm")


def tune_get_gemm(m: int, n: int, k: int) -> int:
    t = _i32()
    _check(load().kfb_tune_get_gemm(int(m), int(n), int(k), ctypes.byref(t)), "kfb_tune_get_gemm")
    return t.value
