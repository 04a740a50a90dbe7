"""CPU-side checks of the C-ABI library: it loads, exports every declared
symbol, and its host-side argument checks behave (no device work)."""
import ctypes
import os
import re

import pytest

from paper_2210_08494_amd import kfb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "kfb.h")).read()
    return sorted(set(re.findall(r"\b(kfb_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(kfb.LIB_PATH):
        pytest.fail("libkfb.so is not built (run __graft_entry__.build())")
    return kfb.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 15
    for nm in names:
        assert hasattr(lib, nm), nm
    assert set(names) == set(kfb.EXPORTS)


def test_state_bytes_and_limits(lib):
    b64 = lib.kfb_state_bytes(256, 32, 32, kfb.KFB_FP64)
    b32 = lib.kfb_state_bytes(256, 32, 32, kfb.KFB_FP32)
    assert b64 > b32 > 0
    # two U buffers of ld x (r + n_max) plus eigenvalues and status
    assert b64 >= 2 * 256 * 64 * 8
    assert lib.kfb_state_bytes(256, 200, 64, kfb.KFB_FP64) == 0   # r + n_max > d
    assert lib.kfb_state_bytes(256, 0, 0, kfb.KFB_FP64) == 0      # n_max = 0
    assert lib.kfb_state_bytes(256, 32, 32, 7) == 0               # bad precision
    assert lib.kfb_state_bytes(256, 224, 32, kfb.KFB_FP64) > 0    # r + n_max == d accepted


def test_create_rejects_bad_arguments_without_touching_memory(lib):
    h = ctypes.c_void_p()
    # null buffer
    rc = lib.kfb_state_create(ctypes.byref(h), 256, 32, 32, 0.95, kfb.KFB_FP64, None, 1 << 20, None)
    assert rc == 1
    # rho out of range (checked before any device call)
    rc = lib.kfb_state_create(ctypes.byref(h), 256, 32, 32, 1.5, kfb.KFB_FP64, ctypes.c_void_p(256), 1 << 20,
                              None)
    assert rc == 1
    # buffer too small
    rc = lib.kfb_state_create(ctypes.byref(h), 256, 32, 32, 0.5, kfb.KFB_FP64, ctypes.c_void_p(256), 16, None)
    assert rc == 2
    # misaligned buffer
    need = lib.kfb_state_bytes(256, 32, 32, kfb.KFB_FP64)
    rc = lib.kfb_state_create(ctypes.byref(h), 256, 32, 32, 0.5, kfb.KFB_FP64, ctypes.c_void_p(260), need, None)
    assert rc == 1


def test_strerror_and_build_info(lib):
    assert lib.kfb_strerror(0) == b"ok"
    assert lib.kfb_strerror(2).startswith(b"buffer")
    info = lib.kfb_build_info()
    assert b"gfx950" in info
    # the digest names the exact sources the library was built from
    from paper_2210_08494_amd import build as kbuild
    assert info.endswith(b"src=" + kbuild.source_digest().encode())
    assert lib.kfb_destroy(None) == 1


def test_grouped_call_layout_checks():
    # the binding refuses mismatched batches before any pointer reaches the library
    import pytest
    import torch
    from paper_2210_08494_amd import kfb
    a = torch.zeros(4, 8)
    kfb._same_layout([a, torch.zeros(4, 8)], "t", 2)
    for bad, cnt in (([a, torch.zeros(5, 8)], 2), ([a, torch.zeros(4, 8).t().contiguous().t()], 2),
                     ([a, torch.zeros(4, 8, dtype=torch.float64)], 2), ([a], 2), ([a[:, ::2]], 1)):
        with pytest.raises(kfb.KfbError):
            kfb._same_layout(bad, "t", cnt)


def test_size_limits_rejected_up_front(lib):
    # the CholeskyQR kernels take at most 2048 columns, the eigensolver at most
    # 4096 modes: such states cannot be created, so no call can reach the device
    assert lib.kfb_state_bytes(65536, 0, 2048, kfb.KFB_BF16_MIXED) > 0
    assert lib.kfb_state_bytes(65536, 0, 2049, kfb.KFB_BF16_MIXED) == 0
    assert lib.kfb_state_bytes(65536, 2048, 2048, kfb.KFB_FP64) > 0
    assert lib.kfb_state_bytes(65536, 2049, 2048, kfb.KFB_FP64) == 0
    h = ctypes.c_void_p()
    rc = lib.kfb_state_create(ctypes.byref(h), 65536, 0, 4096, 0.95, kfb.KFB_FP64, ctypes.c_void_p(256),
                              1 << 40, None)
    assert rc == 1
    # workspace queries on a null handle
    assert lib.kfb_reorth_workspace_bytes(None) == 0
    assert lib.kfb_reorthonormalize(None, None, 0, None) == 1
    assert lib.kfb_update_workspace_bytes(None, 16) == 0


def _fake_factor(torch, d, prec):
    # the binding's checks read d, prec, the batch dtype and the state buffer's device
    from types import SimpleNamespace
    return SimpleNamespace(d=d, prec=prec, mdtype=kfb._mdtype_of(prec), buf=torch.zeros(4, dtype=torch.uint8))


def test_binding_checks_every_tensor_against_its_state():
    import torch
    fa, fg = _fake_factor(torch, 8, kfb.KFB_FP32), _fake_factor(torch, 6, kfb.KFB_FP32)
    kfb._batch_check(torch.zeros(3, 8), fa, "t")
    for bad in (torch.zeros(3, 8, dtype=torch.float64),      # dtype of another form
                torch.zeros(3, 7),                            # wrong width
                torch.zeros(8, 3).t(),                        # columns not contiguous
                torch.zeros(0, 8),                            # no columns
                torch.zeros(3, 8, dtype=torch.bfloat16)):
        with pytest.raises(kfb.KfbError):
            kfb._batch_check(bad, fa, "t")
    kfb._grad_check(torch.zeros(6, 8), fg, fa, "t")
    for bad in (torch.zeros(8, 6), torch.zeros(6, 8, dtype=torch.float64), torch.zeros(5, 8),
                torch.zeros(8, 6).t()):
        with pytest.raises(kfb.KfbError):
            kfb._grad_check(bad, fg, fa, "t")
    # an FP64 pair wants double gradients
    f64a, f64g = _fake_factor(torch, 8, kfb.KFB_FP64), _fake_factor(torch, 6, kfb.KFB_FP64)
    kfb._grad_check(torch.zeros(6, 8, dtype=torch.float64), f64g, f64a, "t")
    with pytest.raises(kfb.KfbError):
        kfb._grad_check(torch.zeros(6, 8), f64g, f64a, "t")
    # the two sides: distinct states of one form
    with pytest.raises(kfb.KfbError):
        kfb._pair_check(fa, fa, "t")
    with pytest.raises(kfb.KfbError):
        kfb._pair_check(f64g, fa, "t")
    kfb._dense_check(torch.zeros(8, 8), fa, "t")
    with pytest.raises(kfb.KfbError):
        kfb._dense_check(torch.zeros(8, 8, dtype=torch.float64), fa, "t")


def test_gemm_tile_table(lib):
    # host-side tuning table of the BF16 products' output tile
    t = ctypes.c_int32()
    assert lib.kfb_tune_get_gemm(512, 4096, 4096, ctypes.byref(t)) == 0 and t.value == 128
    assert lib.kfb_tune_set_gemm(512, 4096, 4096, 256) == 0
    assert lib.kfb_tune_get_gemm(512, 4096, 4096, ctypes.byref(t)) == 0 and t.value == 256
    assert lib.kfb_tune_set_gemm(512, 4096, 4096, 0) == 0
    assert lib.kfb_tune_get_gemm(512, 4096, 4096, ctypes.byref(t)) == 0 and t.value == 128
    for bad in ((0, 1, 1, 128), (1, 1, 1, 64), (1, -1, 1, 256)):
        assert lib.kfb_tune_set_gemm(*bad) == 1


def test_jacobi_table_and_built_in_choice(lib):
    # host-side eigensolver table: built-in choices per form and size, the streamed
    # and refined configurations' admissibility, and removal
    S, REF = 0x100, 0x200
    bw, Np = ctypes.c_int32(), ctypes.c_int32()

    def get(prec, N):
        assert lib.kfb_tune_get_jacobi(prec, N, ctypes.byref(bw), ctypes.byref(Np)) == 0
        return bw.value, Np.value
    assert get(0, 512) == (S | 32, 512)          # FP64: streamed 32-column panels at N >= 256
    assert get(1, 512) == (S | 32, 512)          # FP32: the same kernel on FP32 MFMA
    assert get(2, 512) == (S | REF | 32, 512)    # mixed: FP32 iteration + FP64 refinement
    assert get(2, 150)[0] & S == 0               # below 256: a panel held in LDS
    assert lib.kfb_tune_set_jacobi(2, 512, S | 32) == 0 and get(2, 512) == (S | 32, 512)
    assert lib.kfb_tune_set_jacobi(2, 512, 0) == 0 and get(2, 512) == (S | REF | 32, 512)
    for prec, cfg in ((0, S | REF | 32), (1, S | REF | 32), (2, S | REF | 16), (2, REF | 32), (1, S | 16)):
        assert lib.kfb_tune_set_jacobi(prec, 512, cfg) == 1, (prec, hex(cfg))
