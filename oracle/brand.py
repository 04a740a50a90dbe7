"""Oracle-B: the structured FP64 Brand update, as the paper states it.

Parity unpinned: none.  Pinned against Oracle-D (a dense eigendecomposition
of the definition) and against the exactness / trace / special-case checks in
tests/test_oracle_pins.py.

Algorithm 3 (Symmetric Brand) computes the eigendecomposition of
X^ = U D U^T + A A^T from that of X = U D U^T:

  P  = U^T A                       (projection)
  Zp = A - U P                     (component of A outside span(U))
  Q R = thin QR of Zp              (Householder here; any orthonormal Q works)
  M_S = L diag(D, I) L^T,  L = [[I, P], [0, R]]   (eqn. for M_S, Section 2.3)
  W Lam W^T = EVD(M_S)             (M_S is symmetric PSD, so EVD = SVD)
  U' = [U Q] W,  D' = Lam

Algorithm 4 (B-KFAC) drives it per factor: truncate (U, D) to r columns, then
call it with (U, rho D, sqrt(w) M), where w is the batch weight (1/n on the
very first update, (1 - rho)/n afterwards; see oracle/bprocess.py).
"""
from __future__ import annotations

import numpy as np


def symmetric_brand(U: np.ndarray, D: np.ndarray, A: np.ndarray):
    """Algorithm 3.  U: (d, r) orthonormal, D: (r,), A: (d, n).  Returns (U', D')."""
    U = np.asarray(U, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    d, r = U.shape
    n = A.shape[1]
    P = U.T @ A
    Zp = A - U @ P
    Q, R = np.linalg.qr(Zp, mode="reduced")
    N = r + n
    L = np.zeros((N, N))
    L[:r, :r] = np.eye(r)
    L[:r, r:] = P
    L[r:, r:] = R
    mid = np.concatenate([D, np.ones(n)])
    MS = (L * mid[None, :]) @ L.T
    MS = 0.5 * (MS + MS.T)
    lam, W = np.linalg.eigh(MS)
    order = np.argsort(-lam, kind="stable")
    lam = np.clip(lam[order], 0.0, None)
    W = W[:, order]
    Unew = np.concatenate([U, Q], axis=1) @ W
    return Unew, lam


class BrandFactor:
    """One K-factor held as its low-rank eigen-representation (U, D)."""

    def __init__(self, d: int, r: int, rho: float):
        self.d, self.r, self.rho = int(d), int(r), float(rho)
        self.U = np.zeros((self.d, 0))
        self.D = np.zeros(0)
        self.k = 0

    def overwrite(self, U: np.ndarray, D: np.ndarray) -> None:
        """B-R-KFAC (Algorithm 5): replace the representation by (U, D) (an RSVD of
        the previous EA factor); the next update truncates it as usual."""
        self.U = np.asarray(U, dtype=np.float64).copy()
        self.D = np.asarray(D, dtype=np.float64).copy()

    def update(self, M: np.ndarray) -> None:
        """Algorithm 4 for one factor; M: (d, n) float64 columns are samples."""
        M = np.asarray(M, dtype=np.float64)
        n = M.shape[1]
        if self.k == 0:
            w = 1.0 / n
            Ut, Dt = self.U[:, :0], self.D[:0]
        else:
            w = (1.0 - self.rho) / n
            keep = min(self.r, self.D.shape[0])
            Ut, Dt = self.U[:, :keep], self.rho * self.D[:keep]
        self.U, self.D = symmetric_brand(Ut, Dt, np.sqrt(w) * M)
        self.k += 1


def reorthonormalize(U: np.ndarray, D: np.ndarray):
    """Drift recovery: the matrix U diag(D) U^T re-expressed on an orthonormal basis.

    The method assumes an orthonormal U (Section 2.3); rounded products let it
    drift.  With U = Q R (Householder QR), U D U^T = Q (R D R^T) Q^T, and the
    EVD R D R^T = W Lam W^T gives the representation (Q W, Lam): the same
    matrix (Rayleigh-Ritz on span(U), exact in exact arithmetic), modes
    sorted descending, eigenvalues clipped at 0."""
    U = np.asarray(U, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    Q, R = np.linalg.qr(U, mode="reduced")
    K = (R * D[None, :]) @ R.T
    K = 0.5 * (K + K.T)
    lam, W = np.linalg.eigh(K)
    order = np.argsort(-lam, kind="stable")
    return Q @ W[:, order], np.clip(lam[order], 0.0, None)
