"""Polarizability, screening and W_nm (oracle; test infrastructure only).

Eq. 3 gives the RI irreducible polarizability in spin orbitals,
Pi_PQ(iw) = -2 sum_ia R^P_ia D_ia / (w^2 + D_ia^2) R^Q_ia, D_ia = e_a - e_i.
For closed-shell spatial orbitals the spin sum adds a factor s = 2, so the
prefactor is -2 s = -4 (the same closed-shell factor Sec. 2 applies to the
NAF metric).

Eq. 8 writes 1/(w^2 + D^2) as a Laplace integral; Eq. 9 replaces it by the
quadrature sum_m w_m exp(-w^2 x_m) exp(-D^2 x_m) (plus-sign reading of the
printed minus, see ``grids``).  Eq. 10 then factorises
Pi(iw) ~ -2 s sum_m M^m exp(-w^2 x_m), M^m_PQ = sum_ia R^P_ia w_m D_ia
exp(-D_ia^2 x_m) R^Q_ia.

Eq. 2 gives the correlation part of W in the MO basis:
W_nm(iw) = sum_PQ R^P_nm {[1 - Pi(iw)]^-1 - 1}_PQ R^Q_nm.
"""
from __future__ import annotations

import numpy as np

SPIN = 2.0


def delta_ov(eps: np.ndarray, n_fc: int, n_occ: int) -> np.ndarray:
    """D_ia = e_a - e_i over active i (frozen core excluded), i-major."""
    e_i = eps[n_fc:n_occ]
    e_a = eps[n_occ:]
    return (e_a[None, :] - e_i[:, None]).ravel()


def pi_sos(Rt_ov: np.ndarray, d: np.ndarray, omega: np.ndarray) -> np.ndarray:
    """Eq. 3 (closed shell), one [N][N] matrix per imaginary frequency."""
    out = np.empty((len(omega), Rt_ov.shape[1], Rt_ov.shape[1]))
    for j, w in enumerate(omega):
        f = d / (w * w + d * d)
        out[j] = -2.0 * SPIN * (Rt_ov.T @ (f[:, None] * Rt_ov))
    return out


def m_lt(Rt_ov: np.ndarray, d: np.ndarray, x: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Eq. 10: M^m = sum_ia R_ia w_m D_ia exp(-D_ia^2 x_m) R_ia^T."""
    out = np.empty((len(x), Rt_ov.shape[1], Rt_ov.shape[1]))
    for m in range(len(x)):
        f = w[m] * d * np.exp(-d * d * x[m])
        out[m] = Rt_ov.T @ (f[:, None] * Rt_ov)
    return out


def m_lt_columns(Rt_ov: np.ndarray, d: np.ndarray, x: np.ndarray, w: np.ndarray,
                 cols: np.ndarray) -> np.ndarray:
    """Eq. 10 restricted to the columns Q in ``cols``: M^m[:, cols] =
    sum_ia R_ia w_m D_ia exp(-D_ia^2 x_m) R_ia[cols]^T, shape [L][N][len(cols)]
    (for sizes where the whole M^m is too costly to form on the host)."""
    cols = np.asarray(cols)
    out = np.empty((len(x), Rt_ov.shape[1], len(cols)))
    for m in range(len(x)):
        f = w[m] * d * np.exp(-d * d * x[m])
        out[m] = Rt_ov.T @ (f[:, None] * Rt_ov[:, cols])
    return out


def pi_lt(M: np.ndarray, x: np.ndarray, omega: np.ndarray) -> np.ndarray:
    """Eq. 10: Pi(iw_j) ~ -2 s sum_m M^m exp(-w_j^2 x_m)."""
    out = np.empty((len(omega),) + M.shape[1:])
    for j, w in enumerate(omega):
        out[j] = -2.0 * SPIN * np.tensordot(np.exp(-w * w * x), M, axes=(0, 0))
    return out


def screen(Pi: np.ndarray) -> np.ndarray:
    """Eq. 2: W^ = [1 - Pi]^-1 - 1 per frequency (dense inverse)."""
    n = Pi.shape[-1]
    eye = np.eye(n)
    out = np.empty_like(Pi)
    for j in range(Pi.shape[0]):
        out[j] = np.linalg.inv(eye - Pi[j]) - eye
    return out


def w_diag(Rt_qp: np.ndarray, What: np.ndarray) -> np.ndarray:
    """Eq. 2: W_nm(iw_j) = R_nm^T W^_j R_nm for every (n, m) row of Rt_qp.

    Rt_qp is [Q][M][N]; returns [F][Q][M]."""
    Q, M, N = Rt_qp.shape
    rows = Rt_qp.reshape(Q * M, N)
    out = np.empty((What.shape[0], Q * M))
    for j in range(What.shape[0]):
        out[j] = np.einsum("rp,pq,rq->r", rows, What[j], rows, optimize=True)
    return out.reshape(What.shape[0], Q, M)
