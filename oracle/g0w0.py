"""The whole LT-AC G0W0 chain in plain FP64 (oracle; test infra only).

Order of steps as in the paper: frozen core (Sec. 3), NAF compression
(Eqs. 11-13), frequency grids (Sec. 2, Sec. 3), polarizability -- sum over
states (Eq. 3) or Laplace-transformed (Eqs. 8-10) -- screening and W_nm
(Eq. 2), the self-energy quadrature (Eq. 7), Pade continuation and the QP
fixed point (Sec. 2, Sec. 3).  The default is the sum-over-states form with
no Laplace transformation; ``lt=(x, w)`` switches to the Laplace form with
the given points and weights.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import grids, naf, pade, rpa, sigma


@dataclasses.dataclass
class Result:
    n_naf: int
    lam: np.ndarray          # K eigenvalues, descending
    U: np.ndarray            # [A][N]
    Rt_ov: np.ndarray        # [o*v][N]
    Rt_qp: np.ndarray        # [Q][M][N]
    omega: np.ndarray        # integration nodes
    w_omega: np.ndarray      # integration weights
    omega_pade: np.ndarray   # Pade nodes
    eps_f: float
    Pi: np.ndarray | None    # [F][N][N]
    M: np.ndarray | None     # [L][N][N] (Laplace form only)
    W: np.ndarray            # [F][Q][M]
    sigma: np.ndarray        # [Q][Pd] complex, at e_F + i omega_pade
    eps_qp: np.ndarray
    z: np.ndarray
    converged: np.ndarray


def g0w0(eps, n_fc, n_occ, qp, R_oo, R_ov, R_qp, *, eps_naf, max_keep=0,
         n_freq=32, n_pade=16, x0=0.5, eta=1e-3, lt=None, static=None,
         tol=1e-6, max_iter=100, keep=False, U=None) -> Result:
    # NAF (Eqs. 11-13); U may be supplied to pin the basis
    if U is None:
        K = naf.naf_metric(R_oo, R_ov)
        lam, U = naf.naf_basis(K, eps_naf, max_keep)
    else:
        lam = np.array([])
    Rt_ov = naf.naf_transform(R_ov, U)
    Rt_qp = naf.naf_transform(R_qp, U)
    return g0w0_naf(eps, n_fc, n_occ, qp, Rt_ov, Rt_qp, lam=lam, U=U, n_freq=n_freq,
                    n_pade=n_pade, x0=x0, eta=eta, lt=lt, static=static, tol=tol,
                    max_iter=max_iter, keep=keep)


def g0w0_naf(eps, n_fc, n_occ, qp, Rt_ov, Rt_qp, *, lam=None, U=None, n_freq=32,
             n_pade=16, x0=0.5, eta=1e-3, lt=None, static=None, tol=1e-6,
             max_iter=100, keep=False) -> Result:
    """The chain after the NAF transformation (Eq. 13), from the transformed
    tensors Rt_ov [o*v][N] and Rt_qp [Q][M][N]."""
    eps = np.asarray(eps, dtype=np.float64)
    qp = np.asarray(qp)
    # grids
    omega, w_omega = grids.modified_gauss_legendre(n_freq, x0)
    omega_pade, _ = grids.modified_gauss_legendre(n_pade, x0)
    d = rpa.delta_ov(eps, n_fc, n_occ)
    M = None
    if lt is None:
        Pi = rpa.pi_sos(Rt_ov, d, omega)
    else:
        x, w = lt
        M = rpa.m_lt(Rt_ov, d, np.asarray(x), np.asarray(w))
        Pi = rpa.pi_lt(M, np.asarray(x), omega)
    What = rpa.screen(Pi)
    if not keep:
        del Pi
        Pi = None
    W = rpa.w_diag(Rt_qp, What)
    del What
    eps_f = sigma.fermi_level(eps, n_occ)
    eps_m = eps[n_fc:]
    S = sigma.sigma_iw(W, eps_m, eps_f, omega, w_omega, omega_pade)
    z_nodes = 1j * omega_pade
    c = np.zeros(len(qp)) if static is None else np.asarray(static, dtype=np.float64)
    E = np.empty(len(qp))
    Z = np.empty(len(qp))
    conv = np.zeros(len(qp), dtype=bool)
    for q, n in enumerate(qp):
        a = pade.thiele_coefficients(z_nodes, S[q])
        E[q], Z[q], conv[q] = pade.qp_solve(eps[n], c[q], eps_f, z_nodes, a, eta,
                                            tol=tol, max_iter=max_iter)
    return Result(n_naf=Rt_ov.shape[1], lam=np.array([]) if lam is None else lam,
                  U=U, Rt_ov=Rt_ov, Rt_qp=Rt_qp,
                  omega=omega, w_omega=w_omega, omega_pade=omega_pade,
                  eps_f=eps_f, Pi=Pi, M=M if keep else None,
                  W=W, sigma=S, eps_qp=E, z=Z, converged=conv)


def g0w0_problem(prob, lt=None, **kw) -> Result:
    """Convenience wrapper for a ``gwsynth.Problem``."""
    c = prob.cfg
    args = dict(eps_naf=c.eps_naf, max_keep=c.max_keep, n_freq=c.n_freq,
                n_pade=c.n_pade, x0=c.x0, eta=c.eta)
    args.update(kw)
    return g0w0(prob.eps, c.n_fc, c.n_occ, prob.qp, prob.R_oo, prob.R_ov,
                prob.R_qp, lt=lt, **args)
