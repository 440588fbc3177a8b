"""Pade analytic continuation and the QP equation (oracle; test infra only).

Sec. 2 continues Sigma^c to the real axis with an N-point Pade approximant
built as in the appendix of Vidberg and Serene (1977): the Thiele continued
fraction
    C(z) = a_1 / (1 + a_2 (z - z_1) / (1 + a_3 (z - z_2) / (1 + ...)))
whose coefficients follow from the reciprocal-difference table
    g_1(z_i) = u_i,
    g_p(z_i) = (g_{p-1}(z_{p-1}) - g_{p-1}(z_i)) / ((z_i - z_{p-1}) g_{p-1}(z_i)),
    a_p = g_p(z_p).
The nodes are z_k = i w_k (w_k a modified Gauss-Legendre grid, Sec. 3), the
data Sigma(e_F + i w_k), and the approximant is evaluated at
z = E - e_F + i eta (Sec. 3: eta = 0.001 a.u.).

The QP equation is not written out in the paper (Sec. 2, Sec. 3 only say
that QP iterations are performed).  The reading used is
E = e_n + Re Sigma^c_n(E) + c_n, with c_n = Sigma^x - V^xc an input that is
0 for a Hartree-Fock reference, solved by fixed-point iteration from e_n.
"""
from __future__ import annotations

import numpy as np


def thiele_coefficients(z: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Coefficients a_p (0-based: a[p] = g_{p+1}(z_{p+1})).  A zero
    coefficient ends the continued fraction; later ones are set to zero."""
    n = len(z)
    g = np.array(u, dtype=np.complex128)       # g_1(z_i) for all i
    a = np.empty(n, dtype=np.complex128)
    a[0] = g[0]
    for p in range(1, n):
        if a[p - 1] == 0:                      # the fraction terminates here
            a[p:] = 0
            break
        prev = g.copy()                        # g_p(z_i)
        for i in range(p, n):
            g[i] = (prev[p - 1] - prev[i]) / ((z[i] - z[p - 1]) * prev[i])
        a[p] = g[p]
    return a


def thiele_eval(z_nodes: np.ndarray, a: np.ndarray, z: complex) -> complex:
    """Evaluate the continued fraction from the innermost level outwards."""
    n = len(a)
    t = 1.0 + 0.0j
    for p in range(n - 1, 0, -1):
        t = 1.0 + a[p] * (z - z_nodes[p - 1]) / t
    return a[0] / t


def qp_solve(e_n: float, c_n: float, eps_f: float, z_nodes, a, eta: float,
             tol: float = 1e-6, max_iter: int = 100):
    """Fixed point E = e_n + Re Sigma(E - e_F + i eta) + c_n.

    Returns (E, Z, converged) with Z = 1 / (1 - d Re Sigma / dE) from a
    central difference of the continued fraction."""
    E = e_n
    conv = False
    for _ in range(max_iter):
        En = e_n + thiele_eval(z_nodes, a, E - eps_f + 1j * eta).real + c_n
        if abs(En - E) < tol:
            E = En
            conv = True
            break
        E = En
    h = 1e-5
    dS = (thiele_eval(z_nodes, a, E + h - eps_f + 1j * eta).real
          - thiele_eval(z_nodes, a, E - h - eps_f + 1j * eta).real) / (2 * h)
    return E, 1.0 / (1.0 - dS), conv
