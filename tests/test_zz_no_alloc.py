"""The allocation-free update (kfb_brand_update_scratch) against the update
with a caller workspace (kfb_brand_update), called through the C-ABI: bit for
bit, on two calls in a row, the second with a smaller batch (the library-owned
array keeps the first call's contents), and the size limit."""
import ctypes

import numpy as np
import pytest

from paper_2210_08494_amd import synth

pytestmark = pytest.mark.gpu


def _bf16_batch(torch, cfg, k, n, d):
    x = synth.to_bf16_values(synth.batch_for(cfg, k, "A", n, d))
    return torch.from_numpy(x).to(device="cuda:0", dtype=torch.bfloat16)


def test_scratch_update_equals_workspace_update(kfb):
    import torch
    lib = kfb.load()
    assert lib.kfb_scratch_bytes() == 64 << 20
    d, r, nmax, rho = 2048, 128, 128, 0.95
    for prec, mk in ((kfb.KFB_BF16_MIXED, lambda k, n: _bf16_batch(torch, 90, k, n, d)),
                     (kfb.KFB_FP64, lambda k, n: torch.from_numpy(synth.batch_for(91, k, "G", n, d)).to("cuda:0"))):
        a = kfb.Factor(d, r, nmax, rho, prec)     # caller workspace
        b = kfb.Factor(d, r, nmax, rho, prec)     # library-owned array
        ws = kfb.Workspace()
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        for k, n in enumerate((nmax, nmax, 96, 40)):   # two full calls, then smaller batches
            M = mk(k, n)
            need = lib.kfb_update_workspace_bytes(a.handle, n)
            w = ws.get(need)
            rc = lib.kfb_brand_update(a.handle, ctypes.c_void_p(M.data_ptr()), int(M.stride(0)), n,
                                      ctypes.c_void_p(w.data_ptr()), int(w.numel()), stream)
            assert rc == 0
            rc = lib.kfb_brand_update_scratch(b.handle, ctypes.c_void_p(M.data_ptr()), int(M.stride(0)), n, stream)
            assert rc == 0
            torch.cuda.synchronize()
            Ua, Da = a.front()
            Ub, Db = b.front()
            assert torch.equal(Ua, Ub) and torch.equal(Da, Db), f"prec {prec} call {k} (n={n}) differs"
        assert a.status() == 0 and b.status() == 0


def test_scratch_update_rejects_oversized_problem(kfb):
    import torch
    lib = kfb.load()
    d, r, n = 16384, 1024, 1024          # the update needs far more than the 64 MiB array
    f = kfb.Factor(d, r, n, 0.95, kfb.KFB_BF16_MIXED)
    assert lib.kfb_update_workspace_bytes(f.handle, n) > lib.kfb_scratch_bytes()
    M = torch.zeros((n, d), dtype=torch.bfloat16, device="cuda:0")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.kfb_brand_update_scratch(f.handle, ctypes.c_void_p(M.data_ptr()), d, n, stream)
    assert rc == 2                       # KFB_EWORKSPACE, nothing enqueued
    assert f.info()["step"] == 0 and f.info()["k_valid"] == 0
