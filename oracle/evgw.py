"""Eigenvalue-self-consistent GW (oracle; test infra only).

Sec. 3 and Table 3: evGW repeats the G0W0 evaluation for a fixed number of
cycles (five in the paper), each time with the orbital energies replaced by
the quasiparticle energies of the previous cycle.  Everything that depends
on the energies is rebuilt every cycle: the occupied-virtual gaps of the
polarizability (so the Laplace matrices M^m too), the Laplace grid bounds,
the Fermi level and the poles of G in the self-energy.  The natural
auxiliary functions depend only on the three-index tensor and are kept.

The quasiparticle equation keeps the starting point as its base,
    E_n = e^0_n + c_n + Re Sigma^c_n[e^(c)](E_n),
with Sigma^c built from the cycle's energies e^(c) (the exchange part,
folded into c_n, does not depend on the energies).

Energies of orbitals outside the quasiparticle set (Sec. 3): they are
shifted by the correction of the lowest and of the highest quasiparticle
state.  Reading taken: active occupied orbitals that are not quasiparticle
states move with the lowest state, active virtual ones with the highest;
frozen-core orbitals do not enter any step and are left as they are.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import grids, naf
from .g0w0 import g0w0


def shifted_energies(eps0: np.ndarray, n_fc: int, n_occ: int, qp: np.ndarray,
                     e_qp: np.ndarray) -> np.ndarray:
    """Orbital energies of the next cycle: quasiparticle states take their
    QP energies, other active orbitals the shift of the lowest (occupied) or
    highest (virtual) quasiparticle state (Sec. 3)."""
    eps0 = np.asarray(eps0, dtype=np.float64)
    qp = np.asarray(qp)
    out = eps0.copy()
    lo, hi = int(np.argmin(qp)), int(np.argmax(qp))
    d_lo = e_qp[lo] - eps0[qp[lo]]
    d_hi = e_qp[hi] - eps0[qp[hi]]
    in_qp = np.zeros(len(eps0), dtype=bool)
    in_qp[qp] = True
    for m in range(n_fc, len(eps0)):
        if in_qp[m]:
            continue
        out[m] = eps0[m] + (d_lo if m < n_occ else d_hi)
    out[qp] = e_qp
    return out


@dataclasses.dataclass
class EvResult:
    eps_qp: np.ndarray        # [cycles][Q] quasiparticle energies per cycle
    eps: np.ndarray           # [cycles + 1][n_orb] orbital energies entering each cycle
    z: np.ndarray             # [Q] of the last cycle
    converged: np.ndarray     # [cycles][Q]
    n_naf: int


def evgw(eps, n_fc, n_occ, qp, R_oo, R_ov, R_qp, *, n_cycles=5, eps_naf, max_keep=0,
         n_freq=32, n_pade=16, x0=0.5, eta=1e-3, static=None, lt_points=None,
         tol=1e-6, max_iter=100) -> EvResult:
    """n_cycles G0W0 evaluations with updated energies.  lt_points = None:
    sum-over-states polarizability; an integer L: Laplace form with the
    L-point minimax grid on each cycle's bounds (Sec. 3)."""
    eps0 = np.asarray(eps, dtype=np.float64)
    qp = np.asarray(qp)
    c = np.zeros(len(qp)) if static is None else np.asarray(static, dtype=np.float64)
    K = naf.naf_metric(R_oo, R_ov)
    _, U = naf.naf_basis(K, eps_naf, max_keep)
    omega0 = grids.modified_gauss_legendre(n_freq, x0)[0][0]
    cur = eps0.copy()
    hist_e, hist_eps, conv = [], [cur.copy()], []
    z = None
    for _ in range(n_cycles):
        lt = None
        if lt_points is not None:
            lo, hi = grids.lt_bounds(cur, n_fc, n_occ, omega0)
            x, w, _ = grids.lt_grid(lt_points, lo, hi)
            lt = (x, w)
        # base of the QP equation: the starting energies (c_n kept)
        c_eff = eps0[qp] + c - cur[qp]
        res = g0w0(cur, n_fc, n_occ, qp, R_oo, R_ov, R_qp, eps_naf=eps_naf,
                   max_keep=max_keep, n_freq=n_freq, n_pade=n_pade, x0=x0, eta=eta,
                   lt=lt, static=c_eff, tol=tol, max_iter=max_iter, U=U)
        hist_e.append(res.eps_qp.copy())
        conv.append(res.converged.copy())
        z = res.z
        cur = shifted_energies(eps0, n_fc, n_occ, qp, res.eps_qp)
        hist_eps.append(cur.copy())
    return EvResult(eps_qp=np.array(hist_e), eps=np.array(hist_eps), z=z,
                    converged=np.array(conv), n_naf=U.shape[1])


def evgw_problem(prob, n_cycles=5, lt_points=None, **kw) -> EvResult:
    """Convenience wrapper for a ``gwsynth.Problem``."""
    cf = prob.cfg
    args = dict(eps_naf=cf.eps_naf, max_keep=cf.max_keep, n_freq=cf.n_freq,
                n_pade=cf.n_pade, x0=cf.x0, eta=cf.eta)
    args.update(kw)
    return evgw(prob.eps, cf.n_fc, cf.n_occ, prob.qp, prob.R_oo, prob.R_ov, prob.R_qp,
                n_cycles=n_cycles, lt_points=lt_points, **args)
