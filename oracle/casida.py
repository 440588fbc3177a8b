"""Brute-force real-axis G0W0 from RPA excitations (oracle; test infra only).

This is the "fully analytic" RI G0W0 the paper compares against (Sec. 1,
O(N^6); the "Analytic RI" rows of Table 1), used here on tiny systems to pin
the imaginary-axis chain end to end.

Closed-shell RPA in Casida form: C = D^2 + 2 s D^1/2 (R_ov R_ov^T) D^1/2
(s = 2, D the diagonal of occupied-virtual differences), C Z_k = W_k^2 Z_k.
Excitation densities rho^k_P = sqrt(s) sum_ia R^P_ia sqrt(D_ia / W_k) Z^k_ia,
couplings w^k_nm = sum_P R^P_nm rho^k_P and the correlation self-energy
    Sigma^c_n(z) = sum_m sum_k (w^k_nm)^2 / (z - e_m + sgn(e_F - e_m) W_k),
analytic off the real axis.  On the imaginary axis z = e_F + i w this equals
Eq. 7 with W_nm(iw') = -sum_k (w^k_nm)^2 2 W_k / (w'^2 + W_k^2), which is
Eq. 2 with the polarizability of Eq. 3; with zero coupling the poles reduce
to the bare differences D_ia.
"""
from __future__ import annotations

import numpy as np

SPIN = 2.0


def rpa_excitations(Rt_ov: np.ndarray, d: np.ndarray):
    """Excitation energies W_k and densities rho [K][N]."""
    sd = np.sqrt(d)
    C = np.diag(d * d) + 2.0 * SPIN * (sd[:, None] * (Rt_ov @ Rt_ov.T) * sd[None, :])
    w2, Z = np.linalg.eigh(C)
    Om = np.sqrt(w2)
    rho = np.sqrt(SPIN) * ((Rt_ov * (sd[:, None])).T @ (Z / np.sqrt(Om)[None, :])).T
    return Om, rho


def sigma_casida(Rt_qp: np.ndarray, eps_m: np.ndarray, eps_f: float,
                 Om: np.ndarray, rho: np.ndarray, z: np.ndarray) -> np.ndarray:
    """Sigma^c_n(z) for every QP row n of Rt_qp [Q][M][N]; z [K] complex."""
    wk = np.einsum("qmp,kp->qmk", Rt_qp, rho)                 # [Q][M][K]
    sgn = np.where(eps_m < eps_f, 1.0, -1.0)                  # occupied: +
    den = (z[None, :, None] - eps_m[:, None, None]
           + sgn[:, None, None] * Om[None, None, :])          # [M][Z][K]
    return np.einsum("qmk,mzk->qz", wk * wk, 1.0 / den)


def qp_casida(e_n: float, c_n: float, Rt_qp_n: np.ndarray, eps_m, eps_f,
              Om, rho, eta: float, tol: float = 1e-10, max_iter: int = 200):
    """Fixed point E = e_n + Re Sigma_n(E + i eta) + c_n on the real axis."""
    E = e_n
    for _ in range(max_iter):
        s = sigma_casida(Rt_qp_n[None], eps_m, eps_f, Om, rho,
                         np.array([E + 1j * eta]))[0, 0]
        En = e_n + s.real + c_n
        if abs(En - E) < tol:
            return En, True
        E = En
    return E, False
