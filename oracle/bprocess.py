"""Oracle-D: the dense FP64 definition of what B-KFAC computes for one K-factor.

Parity unpinned: none.  Pinned by tests/test_oracle_pins.py against closed
forms (the summed EA factor), library SVDs, interlacing, the error recursion
of Proposition 3.2, the bounds of Propositions 3.1 and 4.2, and brute force.

Definitions followed (Section 2.1, the EA K-factor; Section 3.2, the K-factor
process and the B-process; Algorithm 4, B-KFAC):

* The true EA factor:  E_0 = w_0 M_0 M_0^T,  E_k = rho E_{k-1} + w M_k M_k^T.
* The B-process iterate: X_0 = E_0;  X_k = rho B_{k-1} + w M_k M_k^T, where
  B_{k-1} is the optimal rank-r truncation of X_{k-1} (its r leading
  eigenpairs).
* B-KFAC represents X_k by its eigenpairs; the representation handed to the
  inverse keeps min(kept_{k-1}, r) + n modes (truncation happens just before
  each update, Section 3.1).

Reading of the weights (the paper leaves the FC-factor normalisation to the
original K-FAC paper): a batch of n samples enters with weight w_0 = 1/n at
k = 0 (kappa(0) = 1) and w = (1 - rho)/n afterwards, i.e. the paper's A_k is
M_k / sqrt(n).
"""
from __future__ import annotations

import numpy as np


def sorted_eigh(X: np.ndarray):
    """Eigenpairs of a symmetric matrix, eigenvalues descending.

    Ties keep the lower index of numpy's ascending order first (stable sort)."""
    lam, V = np.linalg.eigh(X)
    order = np.argsort(-lam, kind="stable")
    return lam[order], V[:, order]


def truncate_rank(X: np.ndarray, r: int) -> np.ndarray:
    """Optimal rank-r truncation of a symmetric PSD matrix (its r leading modes).

    Negative rounding noise in the kept eigenvalues is clipped to zero."""
    lam, V = sorted_eigh(X)
    lr = np.clip(lam[:r], 0.0, None)
    Vr = V[:, :r]
    return (Vr * lr[None, :]) @ Vr.T


class DenseFactor:
    """One K-factor (A or Gamma) of one layer: dense B-process + dense EA factor."""

    def __init__(self, d: int, r: int, rho: float):
        self.d, self.r, self.rho = int(d), int(r), float(rho)
        self.X = None       # B-process iterate  (M~_{B,k})
        self.E = None       # true EA factor     (calligraphic M_k)
        self.B_prev = None  # B_{k-1}, kept for the error-recursion checks
        self.k = 0
        self.kept = 0       # modes the B-KFAC representation carries

    def weight(self, n: int) -> float:
        return 1.0 / n if self.k == 0 else (1.0 - self.rho) / n

    def update(self, M: np.ndarray) -> None:
        """M: (d, n) float64, columns are samples."""
        M = np.asarray(M, dtype=np.float64)
        d, n = M.shape
        assert d == self.d
        w = self.weight(n)
        C = w * (M @ M.T)
        if self.k == 0:
            self.X = C
            self.E = C.copy()
            self.B_prev = None
            self.kept = min(n, d)
        else:
            r_eff = min(self.r, self.kept)
            B = truncate_rank(self.X, r_eff)
            self.B_prev = B
            self.X = self.rho * B + C
            self.E = self.rho * self.E + C
            self.kept = min(r_eff + n, d)
        self.k += 1

    def overwrite(self, U: np.ndarray, D: np.ndarray) -> None:
        """B-R-KFAC (Algorithm 5): the current iterate is replaced by U diag(D) U^T
        (the RSVD of the previous EA factor) in place of the usual truncation."""
        self.X = (U * D[None, :]) @ U.T
        self.kept = U.shape[1]

    def modes(self):
        """(V, lam): the kept eigenpairs of X_k, eigenvalues descending, clipped >= 0."""
        lam, V = sorted_eigh(self.X)
        K = self.kept
        return V[:, :K], np.clip(lam[:K], 0.0, None)

    def truncated(self, r: int | None = None) -> np.ndarray:
        """B_k: the optimal rank-r truncation of the current iterate."""
        return truncate_rank(self.X, self.r if r is None else r)
