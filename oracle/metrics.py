"""Basis-invariant comparisons between eigen-representations (FP64).

Eigenvector signs, rotations inside degenerate eigenspaces and the choice of
the QR basis are not unique (Section 2.3, the QR footnote), so comparisons use
quantities that do not depend on them.
"""
from __future__ import annotations

import numpy as np


def e_rec_dense(U: np.ndarray, D: np.ndarray, X: np.ndarray) -> float:
    """|| U diag(D) U^T - X ||_F / ||X||_F, forming the d x d matrix."""
    Y = (U * D[None, :]) @ U.T
    return float(np.linalg.norm(Y - X) / np.linalg.norm(X))


def _joint(U1, U2):
    Y = np.concatenate([U1, U2], axis=1)
    # Householder QR gives an orthonormal basis even when [U1 U2] is rank
    # deficient (U1 and U2 nearly span the same space, the usual case).
    Q, _ = np.linalg.qr(Y, mode="reduced")
    return Q


def e_rec_lowrank(U1, D1, U2, D2) -> float:
    """|| U1 D1 U1^T - U2 D2 U2^T ||_F / || U2 D2 U2^T ||_F without forming d x d.

    Both products live in the span of [U1 U2]; expressed in an orthonormal basis
    Q of that span the difference is a small m x m matrix with the same
    Frobenius norm, so no cancellation between large traces occurs."""
    U1 = np.asarray(U1, dtype=np.float64)
    U2 = np.asarray(U2, dtype=np.float64)
    Q = _joint(U1, U2)
    T1 = Q.T @ U1
    T2 = Q.T @ U2
    A = (T1 * D1[None, :]) @ T1.T
    B = (T2 * D2[None, :]) @ T2.T
    return float(np.linalg.norm(A - B) / np.linalg.norm(B))


def e_D(D1, D2) -> float:
    """max_i |D1_i - D2_i| / max(D2), both sorted descending, zero-padded."""
    a = np.sort(np.asarray(D1, dtype=np.float64))[::-1]
    b = np.sort(np.asarray(D2, dtype=np.float64))[::-1]
    m = max(a.size, b.size)
    a = np.pad(a, (0, m - a.size))
    b = np.pad(b, (0, m - b.size))
    return float(np.max(np.abs(a - b)) / b[0])


def e_orth(U, D=None, rel_floor: float = 0.0) -> float:
    """max |U^T U - I| over columns (optionally only those with D > rel_floor * max D)."""
    U = np.asarray(U, dtype=np.float64)
    if D is not None and rel_floor > 0:
        keep = np.asarray(D) > rel_floor * np.max(D)
        U = U[:, keep]
    G = U.T @ U
    return float(np.max(np.abs(G - np.eye(G.shape[0])))) if G.size else 0.0


def e_S(S1, S2) -> float:
    """|| S1 - S2 ||_F / || S2 ||_F."""
    S1 = np.asarray(S1, dtype=np.float64)
    S2 = np.asarray(S2, dtype=np.float64)
    return float(np.linalg.norm(S1 - S2) / np.linalg.norm(S2))


def e_S_proj(S1, S2, UG, UA) -> float:
    """|| UG^T (S1 - S2) UA ||_F / || UG^T S2 UA ||_F.

    The two-sided inverse (Section 2.1; the spectral form of Algorithm 1's
    inverse lines) maps the part of G outside span(UG) x span(UA) by the plain
    scalar 1/(lam_G lam_A); with a small lambda that part dominates ||S||_F and
    hides errors in the low-rank terms.  Restricted to the modes' span, the
    error is measured where the representations act.  UG, UA: orthonormal
    bases of the modes used (the oracle's)."""
    D = np.asarray(S1, dtype=np.float64) - np.asarray(S2, dtype=np.float64)
    UG = np.asarray(UG, dtype=np.float64)
    UA = np.asarray(UA, dtype=np.float64)
    num = np.linalg.norm(UG.T @ D @ UA)
    den = np.linalg.norm(UG.T @ np.asarray(S2, dtype=np.float64) @ UA)
    return float(num / den)


# ----------------------------------------------------------------------------
# The error metrics of the paper's numerical error study (Section 4.2): an
# approximate algorithm against K-FAC holding the exact regularised inverse of
# the current EA factors.
# ----------------------------------------------------------------------------
def regularised_inverse_lowrank(U, D, lam: float) -> np.ndarray:
    """(U diag(D) U^T + lam I)^{-1} as a dense matrix (U orthonormal), spectral form."""
    U = np.asarray(U, dtype=np.float64)
    c = 1.0 / (np.asarray(D, dtype=np.float64) + lam) - 1.0 / lam
    return (U * c[None, :]) @ U.T + np.eye(U.shape[0]) / lam


def e_inverse(U, D, lam: float, E: np.ndarray, lam_ref: float) -> float:
    """Metrics (1) and (2): || inv~ - inv_ref ||_F / || inv_ref ||_F with
    inv_ref = (E + lam_ref I)^{-1} of the exact EA factor (dense solve)."""
    ref = np.linalg.solve(E + lam_ref * np.eye(E.shape[0]), np.eye(E.shape[0]))
    return float(np.linalg.norm(regularised_inverse_lowrank(U, D, lam) - ref) / np.linalg.norm(ref))


def e_angle(S1, S2) -> float:
    """Metric (4): 1 - cos of the angle between two steps (Frobenius inner product)."""
    S1 = np.asarray(S1, dtype=np.float64)
    S2 = np.asarray(S2, dtype=np.float64)
    return float(1.0 - np.sum(S1 * S2) / (np.linalg.norm(S1) * np.linalg.norm(S2)))
