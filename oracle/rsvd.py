"""B-R-KFAC pieces of the FP64 oracle: the dense EA K-factor and its randomized SVD.

TEST INFRASTRUCTURE ONLY (see the package docstring).
Parity unpinned: none.  Pinned in tests/test_oracle_pins.py: exact recovery of
low-rank factors (library eigendecomposition), the span of the sketch against
an explicit matrix power, the rank-l reconstruction identity, a probabilistic
error bound of the randomized range finder, and the overwrite case of
Proposition 3.2 together with the optimality of Proposition 3.1.

What the paper fixes (Section 3.3, Algorithm 5, B-R-KFAC): every T_RSVD
steps the B-KFAC representation of a factor is overwritten by an RSVD of the
dense EA factor of the previous step, in place of the usual truncation, and
the B-update then proceeds as in Algorithm 4.  The dense EA factor is the
definition of Section 2.1 (the EA K-factor), with the batch weight reading of
the rest of the oracle (1/n at the first step, (1 - rho)/n afterwards).

The RSVD is the randomized SVD the paper borrows from randomized K-FAC
(Algorithm 1): a Gaussian sketch Omega (d x l, l = r + oversampling), the
range finder with q power (subspace) iterations re-orthonormalised after
every product with the factor, B = Q^T X, and an SVD of the small B.  The
paper writes the result as U~ D~ U~^T: the left singular vectors Q U_B and
the singular values s of B (for the symmetric PSD factor they approximate its
leading eigenpairs), truncated to the target rank r.
"""
from __future__ import annotations

import numpy as np


def ea_update(E, M: np.ndarray, rho: float):
    """One step of the dense EA factor: E <- rho E + w M M^T (E None: the first step, w = 1/n)."""
    M = np.asarray(M, dtype=np.float64)
    n = M.shape[1]
    if E is None:
        return (M @ M.T) / n
    return rho * E + ((1.0 - rho) / n) * (M @ M.T)


def range_basis(X: np.ndarray, Omega: np.ndarray, power_its: int) -> np.ndarray:
    """Orthonormal basis Q of the randomized range finder with q power iterations.

    Each power iteration multiplies by X^T and by X (the two coincide for a
    symmetric factor, but the scheme is written for a general matrix) and
    re-orthonormalises after each product (Householder QR)."""
    Q, _ = np.linalg.qr(X @ Omega)
    for _ in range(power_its):
        Q, _ = np.linalg.qr(X.T @ Q)
        Q, _ = np.linalg.qr(X @ Q)
    return Q


def rsvd(X: np.ndarray, Omega: np.ndarray, r: int, power_its: int):
    """Randomized SVD truncated to rank r: (U~ = Q U_B[:, :r], s[:r], V_B^T[:r]) with B = Q^T X."""
    Q = range_basis(X, Omega, power_its)
    B = Q.T @ X
    Ub, s, Vt = np.linalg.svd(B, full_matrices=False)
    return Q @ Ub[:, :r], s[:r], Vt[:r]


def rsvd_overwrite(E: np.ndarray, Omega: np.ndarray, r: int, power_its: int):
    """The representation B-R-KFAC writes into a factor's state: (U~, D~) of rank r."""
    U, s, _ = rsvd(E, Omega, r, power_its)
    return U, s
