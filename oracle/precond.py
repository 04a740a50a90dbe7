"""The regularised K-factor inverse applied to a layer gradient (FP64 oracle).

Parity unpinned: none.  The spectral forms are pinned against dense Cholesky
solves (scipy) and eigenvector checks in tests/test_oracle_pins.py.

Section 2.1: with Kronecker factors A (input side) and Gamma (output side),
the preconditioned step of a layer with matrix gradient J (d_out x d_in) is
S = (Gamma + lam_G I)^{-1} J (A + lam_A I)^{-1}.

Algorithm 1 (its inverse-application lines) uses low-rank eigen-
representations X ~ U diag(D) U^T:
    (U D U^T + lam I)^{-1} Y = U [(D + lam)^{-1} - 1/lam] U^T Y + Y / lam,
applied first on the right (A side), then on the left (Gamma side).

Algorithm 8 (Section 5) applies each side to the factored gradient
J = G_k A_k^T instead:  S = [inv(Gamma) G_k] [A_k^T inv(A)].

Section 3.5 (spectrum continuation): the eigenvalues missing from the
low-rank representation are set to the smallest kept one, i.e.
lam <- lam + m, D <- D - m with m the smallest kept eigenvalue.  Reading: a
mode of eigenvalue exactly 0 is not a kept mode (it is an empty slot, a zero
column left by a dropped null direction or by zero padding), so m is the
smallest positive eigenvalue; such slots stay at 0 and add nothing.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import cho_factor, cho_solve


def precondition_dense(XG: np.ndarray, XA: np.ndarray, J: np.ndarray, lamG: float, lamA: float):
    """Definition: dense Cholesky solves with the d x d regularised factors."""
    dG, dA = XG.shape[0], XA.shape[0]
    cG = cho_factor(XG + lamG * np.eye(dG), lower=True)
    cA = cho_factor(XA + lamA * np.eye(dA), lower=True)
    left = cho_solve(cG, J)                 # (Gamma + lam I)^{-1} J
    return cho_solve(cA, left.T).T          # ... (A + lam I)^{-1}   (A symmetric)


def lowrank_inverse_apply(U: np.ndarray, D: np.ndarray, lam: float, Y: np.ndarray):
    """(U diag(D) U^T + lam I)^{-1} Y for orthonormal U (Algorithm 1 / Algorithm 8)."""
    c = 1.0 / (D + lam) - 1.0 / lam
    return U @ (c[:, None] * (U.T @ Y)) + Y / lam


def precondition_lowrank(UG, DG, UA, DA, J, lamG: float, lamA: float):
    """Algorithm 1, inverse-application lines: right side (A) first, then left (Gamma)."""
    mid = lowrank_inverse_apply(UA, DA, lamA, J.T).T       # J (A~ + lam_A I)^{-1}
    return lowrank_inverse_apply(UG, DG, lamG, mid)        # (Gamma~ + lam_G I)^{-1} mid


def precondition_factored(UG, DG, UA, DA, Gk, Ak, lamG: float, lamA: float):
    """Algorithm 8: per-side application to G_k (d_out x n) and A_k (d_in x n), then S = G A^T."""
    Gb = lowrank_inverse_apply(UG, DG, lamG, Gk)
    Ab = lowrank_inverse_apply(UA, DA, lamA, Ak)
    return Gb @ Ab.T


def spectrum_continuation(D: np.ndarray, lam: float):
    """Section 3.5: missing eigenvalues are set to the smallest kept (positive) one."""
    D = np.asarray(D, dtype=np.float64)
    pos = D[D > 0]
    m = float(np.min(pos)) if pos.size else 0.0
    return np.maximum(D - m, 0.0), lam + m
