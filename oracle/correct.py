"""B-KFAC-C pieces of the FP64 oracle: the light correction of Algorithm 6.

TEST INFRASTRUCTURE ONLY (see the package docstring).
Parity unpinned: none.  Pinned in tests/test_oracle_pins.py: the projected
error vanishes on the corrected subspace, the error never grows (the
orthogonal-split argument of Section 3.4's footnote), orthonormality and the
untouched modes are kept, and with every mode selected the correction is the
Rayleigh-Ritz projection of the EA factor (library eigendecomposition).

Algorithm 6 (Section 3.4): from the B-KFAC representation (U, D), pick n_crc
of the leading r columns at random without replacement (the indices are an
input here: the method's random draws come from the input generator), project
the EA factor onto them, M_S = U_c^T M U_c, take its symmetric EVD
M_S = W L W^T, and replace those columns and eigenvalues by U_c W and L.
Algorithm 7 applies it after the B-update every T_corct steps.

Reading: the paper writes the corrected columns back in place; the modes are
then re-sorted by eigenvalue, descending (stable), so that the next
truncation keeps the r largest as everywhere else in B-KFAC.
"""
from __future__ import annotations

import numpy as np

from .bprocess import sorted_eigh


def light_correction(U: np.ndarray, D: np.ndarray, E: np.ndarray, col_idx):
    """Algorithm 6 on (U, D) with the EA factor E and the chosen columns; returns (U', D') sorted."""
    U = np.array(U, dtype=np.float64, copy=True)
    D = np.array(D, dtype=np.float64, copy=True)
    idx = np.asarray(col_idx, dtype=np.int64)
    assert len(set(idx.tolist())) == idx.size, "columns are drawn without replacement"
    Uc = U[:, idx]
    MS = Uc.T @ E @ Uc
    lam, W = sorted_eigh(0.5 * (MS + MS.T))
    U[:, idx] = Uc @ W
    D[idx] = lam
    order = np.argsort(-D, kind="stable")
    return U[:, order], D[order]
