"""Correlation self-energy on the imaginary axis (oracle; test infra only).

Eq. 7: Sigma^c_n(iw) = -(1/pi) sum_m int_0^inf dw' (iw + e_F - e_m) /
((iw + e_F - e_m)^2 + w'^2) W_nm(iw'), integrated with the modified
Gauss-Legendre rule (Sec. 2).  Here "Sigma_n(iw)" is the self-energy at the
complex energy e_F + iw.  The paper does not define e_F; the midpoint of the
HOMO and LUMO energies is used.  The m-sum runs over active orbitals and
carries no spin factor.
"""
from __future__ import annotations

import numpy as np


def fermi_level(eps: np.ndarray, n_occ: int) -> float:
    return 0.5 * (eps[n_occ - 1] + eps[n_occ])


def sigma_iw(W: np.ndarray, eps_m: np.ndarray, eps_f: float,
             omega: np.ndarray, w_omega: np.ndarray,
             omega_eval: np.ndarray) -> np.ndarray:
    """W [F][Q][M] on the integration nodes -> Sigma [Q][K] (complex) at
    e_F + i omega_eval[k]."""
    F, Q, M = W.shape
    out = np.zeros((Q, len(omega_eval)), dtype=np.complex128)
    for k, wk in enumerate(omega_eval):
        a = 1j * wk + eps_f - eps_m                               # [M]
        g = a[None, :] / (a[None, :] ** 2 + omega[:, None] ** 2)  # [F][M]
        # sum_j w_j sum_m g_jm W_jnm
        out[:, k] = -(1.0 / np.pi) * np.einsum("j,jm,jqm->q", w_omega, g, W)
    return out
