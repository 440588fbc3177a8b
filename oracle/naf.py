"""Natural auxiliary functions (oracle; test infrastructure only).

Eq. 11 defines the metric K_PQ = sum_nm R^P_nm R^Q_nm.  Sec. 2 (after
Eq. 13) omits the virtual-virtual part of the sum and multiplies by two for
closed-shell spatial orbitals.  With a symmetric tensor the remaining ordered
pairs are the occupied-occupied block plus the occupied-virtual block taken
twice (ia and ai), so K = 2 (R_oo^T R_oo + 2 R_ov^T R_ov), frozen core
excluded (Sec. 3: frozen orbitals take part in no post-SCF step).

Eq. 12 diagonalises K; the transformation U keeps the eigenvectors whose
eigenvalue exceeds eps_NAF (strict), optionally capped at the ``max_keep``
largest.  Eq. 13 transforms the tensor, R~ = R U; with every eigenvector
kept this is an orthogonal transformation.
"""
from __future__ import annotations

import numpy as np

SPIN = 2.0


def naf_metric(R_oo: np.ndarray, R_ov: np.ndarray) -> np.ndarray:
    """K = s (sum_ij R_ij R_ij^T + 2 sum_ia R_ia R_ia^T), s = 2."""
    A = R_ov.shape[-1]
    oo = R_oo.reshape(-1, A)
    return SPIN * (oo.T @ oo + 2.0 * (R_ov.T @ R_ov))


def naf_basis(K: np.ndarray, eps_naf: float, max_keep: int = 0):
    """Eigenvalues (descending) of K and the kept eigenvectors U [A][N]."""
    lam, vec = np.linalg.eigh(K)
    order = np.argsort(lam)[::-1]
    lam, vec = lam[order], vec[:, order]
    keep = int(np.count_nonzero(lam > eps_naf))
    if max_keep > 0:
        keep = min(keep, max_keep)
    return lam, vec[:, :keep]


def naf_transform(R: np.ndarray, U: np.ndarray) -> np.ndarray:
    """Eq. 13: R~^{P~} = sum_P R^P U_{P P~} (last axis is the aux index)."""
    return R @ U
