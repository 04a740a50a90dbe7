"""Autotuner for the core eigensolver's configuration.

For a shape bucket (precision form, width d, rank r, batch n, group size),
times grouped Brand updates under every admissible configuration of the block
Jacobi eigensolver (block width, with the block pair's panel in LDS where the
LDS limit admits it, or streamed from global memory) and installs the fastest
in the library's tuning table (kfb_tune_set_jacobi), keyed by
(precision, N = r + n).
Results with a given table are deterministic; different widths change only
the rotation order (all within the form's tolerance).
"""
from __future__ import annotations

import time

from . import kfb


DEFAULT_CANDIDATES = (4, 8, 16, 32, kfb.KFB_JAC_STREAMED | 16, kfb.KFB_JAC_STREAMED | 32)


def config_name(cfg: int) -> str:
    return f"s{cfg & 0xff}" if cfg & kfb.KFB_JAC_STREAMED else str(cfg)


def tune_jacobi(prec: int, d: int, r: int, n: int, count: int = 8, reps: int = 3, device="cuda",
                candidates=DEFAULT_CANDIDATES, seed: int = 0, verbose: bool = False):
    import torch
    dev = torch.device(device)
    N = r + n
    mdt = {kfb.KFB_FP64: torch.float64, kfb.KFB_FP32: torch.float32, kfb.KFB_BF16_MIXED: torch.bfloat16}[prec]
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    k = torch.arange(1, d + 1, device=dev, dtype=torch.float32)
    # a fresh batch for every update: a batch already absorbed lies in span(U), its
    # residual vanishes and the core degenerates, which would flatter the eigensolver
    sets = [[(torch.relu(torch.randn(n, d, generator=g, device=dev) * k ** -1.0)).to(mdt) for _ in range(count)]
            for _ in range(reps + 2)]
    ws = kfb.Workspace(dev)
    timings = {}
    for bw in candidates:
        try:
            kfb.tune_set_jacobi(prec, N, bw)
        except kfb.KfbError:
            continue
        states = [kfb.Factor(d, r, n, 0.95, prec, device=dev) for _ in range(count)]
        kfb.update_batched(states, sets[0], ws)      # -> n modes
        kfb.update_batched(states, sets[1], ws)      # -> r + n modes (the tuned N)
        torch.cuda.synchronize()
        ts = []
        for j in range(reps):
            t0 = time.perf_counter()
            kfb.update_batched(states, sets[2 + j], ws)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        timings[bw] = sorted(ts)[len(ts) // 2]
        if verbose:
            print(f"tune prec={prec} N={N} count={count} cfg={config_name(bw)}: {1e3 * timings[bw]:.2f} ms", flush=True)
        del states
    if not timings:
        kfb.tune_set_jacobi(prec, N, 0)
        return None, {}
    best = min(timings, key=timings.get)
    kfb.tune_set_jacobi(prec, N, best)
    return best, timings
