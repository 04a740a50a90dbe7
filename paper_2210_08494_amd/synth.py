"""Seeded synthetic workloads for the Brand-update K-factor path.

This module only draws random numbers and shapes them; it contains none of the
method's arithmetic (no projections, no factorisations, no exponential
averaging).  Both the HIP path (tests, benchmark) and the FP64 CPU oracle take
their inputs from here, so the two sides always see the same values.

Recipe (mirrors the shape of the paper's FC-layer workload, Section 6: a wide
fully-connected layer fed batches of n samples):

* activations  a = ReLU(Z . diag(k^-alpha)),  Z ~ N(0,1)^{n x d_feat},
  k = 1..d_feat (1-based feature index), alpha = 1.0 by default; an optional
  constant column of ones is appended (the homogeneous bias coordinate), so
  d = d_feat + 1.  The K-factor input is M_A = a^T (d x n).
* output grads g = Z' . diag(k^-beta), Z' ~ N(0,1)^{n x d}, beta = 0.7, no ReLU.
  The K-factor input is M_G = g^T.
* layer gradient G ~ N(0,1)^{d_out x d_in}, a fresh draw every step.
* the Gaussian test matrix of a randomized SVD, iid N(0,1), d x l (stream 4),
  and the columns a light correction picks (stream 5): the method's random
  draws are inputs, so both sides get the same ones.

Every array is generated in float64 by numpy's PCG64, seeded from
SeedSequence(entropy=20221015, spawn_key=(config_id, step, stream)), and
returned in the layout the C-ABI consumes: a batch M (d x n, column-major,
leading dimension d) is the row-major numpy array of shape (n, d).
"""
from __future__ import annotations

import numpy as np

ENTROPY = 20221015
STREAM_A, STREAM_G, STREAM_GRAD, STREAM_SERVE = 0, 1, 2, 3


def rng_for(config_id: int, step: int, stream: int) -> np.random.Generator:
    ss = np.random.SeedSequence(entropy=ENTROPY, spawn_key=(int(config_id), int(step), int(stream)))
    return np.random.Generator(np.random.PCG64(ss))


def activations(rng: np.random.Generator, n: int, d_feat: int, alpha: float = 1.0,
                relu: bool = True, bias: bool = False) -> np.ndarray:
    """Return an (n, d) float64 array: row i is sample i (= column i of M_A)."""
    k = np.arange(1, d_feat + 1, dtype=np.float64)
    z = rng.standard_normal((n, d_feat)) * (k ** -alpha)[None, :]
    if relu:
        z = np.maximum(z, 0.0)
    if bias:
        z = np.concatenate([z, np.ones((n, 1))], axis=1)
    return np.ascontiguousarray(z)


def output_grads(rng: np.random.Generator, n: int, d: int, beta: float = 0.7) -> np.ndarray:
    """Return an (n, d) float64 array: row i is sample i (= column i of M_G)."""
    k = np.arange(1, d + 1, dtype=np.float64)
    return np.ascontiguousarray(rng.standard_normal((n, d)) * (k ** -beta)[None, :])


def gradient(rng: np.random.Generator, d_out: int, d_in: int) -> np.ndarray:
    """Return a row-major (d_out, d_in) float64 layer gradient, iid N(0,1)."""
    return rng.standard_normal((d_out, d_in))


def batch_for(config_id: int, step: int, side: str, n: int, d: int, *, bias: bool = False,
              alpha: float = 1.0, beta: float = 0.7) -> np.ndarray:
    """The (n, d) batch of one factor at one step.  side is 'A' or 'G'.

    For side 'A' with bias=True, d counts the appended ones column.
    """
    if side == "A":
        rng = rng_for(config_id, step, STREAM_A)
        return activations(rng, n, d - 1 if bias else d, alpha=alpha, relu=True, bias=bias)
    if side == "G":
        rng = rng_for(config_id, step, STREAM_G)
        return output_grads(rng, n, d, beta=beta)
    raise ValueError(side)


def grad_for(config_id: int, step: int, d_out: int, d_in: int) -> np.ndarray:
    return gradient(rng_for(config_id, step, STREAM_GRAD), d_out, d_in)


STREAM_SKETCH = 4


def sketch_for(config_id: int, step: int, d: int, l: int) -> np.ndarray:
    """The Gaussian test matrix of a randomized SVD: (l, d) iid N(0,1) rows.

    As a d x l column-major matrix (the layout the C-ABI takes) it is the
    row-major numpy array of shape (l, d)."""
    return rng_for(config_id, step, STREAM_SKETCH).standard_normal((l, d))


STREAM_CORRECT = 5


def correction_columns(config_id: int, step: int, r: int, n_crc: int) -> np.ndarray:
    """n_crc distinct column indices out of the leading r (B-KFAC-C's random choice)."""
    return rng_for(config_id, step, STREAM_CORRECT).choice(r, size=n_crc, replace=False).astype(np.int32)


def to_bf16_values(x: np.ndarray) -> np.ndarray:
    """Round float64 values to the nearest bfloat16 (ties to even), returned as float64.

    Used to hand both sides the exact values a BF16 input buffer holds.
    """
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# Named workloads (shapes of the five measured configurations)
# ---------------------------------------------------------------------------
CONFIGS = {
    # plain FP64 single FC layer
    1: dict(name="fp64_d256_r32_n32", prec="fp64", d_in=256, d_out=256, n=32, r=32, rho=0.95,
            lam=0.1, steps=50, bias=False),
    # plain FP32 at realistic width (bias row included in d_in)
    2: dict(name="fp32_d4097x4096_r256_n256", prec="fp32", d_in=4097, d_out=4096, n=256, r=256,
            rho=0.95, lam=0.01, steps=200, bias=True),
    # BF16-mixed wide layer
    3: dict(name="mixed_d8192_r512_n512", prec="mixed", d_in=8192, d_out=8192, n=512, r=512,
            rho=0.95, lam=0.01, steps=100, bias=False),
    # headline shape for throughput: d=4096 r=256 n=256 (both factors)
    6: dict(name="headline_d4096_r256_n256", prec="mixed", d_in=4096, d_out=4096, n=256, r=256,
            rho=0.95, lam=0.01, steps=200, bias=False),
}
