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


DEFAULT_CANDIDATES = (4, 8, 16, 32, kfb.KFB_JAC_STREAMED | 16, kfb.KFB_JAC_STREAMED | 32,
                      kfb.KFB_JAC_STREAMED | kfb.KFB_JAC_REFINE | 32)


def config_name(cfg: int) -> str:
    if cfg & kfb.KFB_JAC_STREAMED:
        return f"s{cfg & 0xff}" + ("r" if cfg & kfb.KFB_JAC_REFINE else "")
    return str(cfg)


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


# ---------------------------------------------------------------------------
# Output tiles of the BF16 MFMA products (the mixed form's inverse application)
# ---------------------------------------------------------------------------
TILE_CANDIDATES = (128, 256)


def precond_product_shapes(d_out: int, d_in: int, NG: int, NA: int):
    """(m, n, k) of the two-sided application's products (Algorithm 1's inverse
    lines in the spectral form): T1 = U_G^T G, T2 = G U_A, T3 = T1 U_A,
    X2 = T2 + U_G T3, S = G / (lam lam) + [U_G | X2] [X1 ; U_A^T]."""
    return [(NG, d_in, d_out), (d_out, NA, d_in), (NG, NA, d_in), (d_out, NA, NG), (d_out, d_in, NG + NA)]


def factored_product_shapes(d_out: int, d_in: int, n: int):
    """(m, n, k) of the factored application's single-term product S = Y_G Y_A^T."""
    return [(d_out, d_in, n)]


def tune_gemm_tiles(run, shapes, reps: int = 3, candidates=TILE_CANDIDATES, verbose: bool = False):
    """Time `run()` (a call issuing the products of `shapes`) with every candidate
    tile installed for all of them, keep the fastest; returns (best, {tile: s})."""
    import torch
    timings = {}
    for tile in candidates:
        for (m, n, k) in shapes:
            kfb.tune_set_gemm(m, n, k, tile)
        run()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            run()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        timings[tile] = sorted(ts)[len(ts) // 2]
        if verbose:
            print(f"tune gemm tile {tile}: {1e3 * timings[tile]:.3f} ms", flush=True)
    best = min(timings, key=timings.get)
    for (m, n, k) in shapes:
        kfb.tune_set_gemm(m, n, k, best)
    return best, timings
