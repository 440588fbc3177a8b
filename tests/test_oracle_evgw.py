"""Pins for the oracle's eigenvalue-self-consistent GW (Sec. 3, Table 3):
one cycle is G0W0, the two-level model iterated with its closed-form
self-energy, the energy-shift rule for orbitals outside the quasiparticle
set, and the zero-coupling limit."""
import numpy as np

from conftest import HARTREE_MEV, two_level
from oracle.evgw import evgw, evgw_problem, shifted_energies
from oracle.g0w0 import g0w0_problem

S = 2.0


def test_one_cycle_is_g0w0(tiny_problem, tiny_sos):
    ev = evgw_problem(tiny_problem, n_cycles=1)
    assert np.array_equal(ev.eps_qp[0], tiny_sos.eps_qp)
    assert np.array_equal(ev.eps[0], tiny_problem.eps)


def _sigma_2l(t, z, n, e_i, e_a):
    """Closed-form self-energy of the two-level model with energies e_i, e_a
    (one aux function; W has the single RPA pole Omega)."""
    d = e_a - e_i
    Om = np.sqrt(d * d + 2 * S * t["r"] ** 2 * d)
    K = S * t["r"] ** 2 * d / Om
    Rn = {0: (t["p"], t["r"]), 1: (t["r"], t["q"])}[n]
    return Rn[0] ** 2 * K / (z - e_i + Om) + Rn[1] ** 2 * K / (z - e_a - Om)


def test_two_level_evgw_matches_closed_form():
    t = two_level()
    eps0 = np.array([t["e_i"], t["e_a"]])
    R_ov = np.array([[t["r"]]])
    R_oo = np.array([[[t["p"]]]])
    R_qp = np.array([[[t["p"]], [t["r"]]], [[t["r"]], [t["q"]]]])
    ev = evgw(eps0, 0, 1, np.array([0, 1]), R_oo, R_ov, R_qp, n_cycles=4, eps_naf=0.0,
              n_freq=512, n_pade=16, eta=1e-3, tol=1e-12, max_iter=500)
    e = eps0.copy()
    for cyc in range(4):
        E = np.empty(2)
        for n in (0, 1):
            x = e[n]
            for _ in range(3000):
                x = eps0[n] + _sigma_2l(t, x + 1e-3j, n, e[0], e[1]).real
            E[n] = x
        assert np.max(np.abs(ev.eps_qp[cyc] - E)) * HARTREE_MEV < 2e-3, (cyc, ev.eps_qp[cyc], E)
        e = E
    # self-consistency changes the answer beyond the G0W0 step
    assert np.max(np.abs(ev.eps_qp[-1] - ev.eps_qp[0])) * HARTREE_MEV > 1.0


def test_shift_rule_for_orbitals_outside_the_qp_set():
    eps0 = np.array([-20.0, -5.0, -1.0, -0.5, 0.1, 0.8, 2.0])   # n_fc = 1, n_occ = 4
    qp = np.array([2, 3, 4])                                     # HOMO-1, HOMO, LUMO
    E = np.array([-1.1, -0.45, 0.15])
    out = shifted_energies(eps0, 1, 4, qp, E)
    assert out[0] == -20.0                                       # frozen core untouched
    assert np.isclose(out[1], -5.0 + (-1.1 + 1.0))               # below: lowest QP shift
    assert np.allclose(out[2:5], E)
    assert np.allclose(out[5:], eps0[5:] + (0.15 - 0.1))          # above: highest QP shift
    # the shift is always taken from the starting energies (no accumulation)
    out2 = shifted_energies(eps0, 1, 4, qp, E + 0.01)
    assert np.isclose(out2[1] - out[1], 0.01)


def test_zero_coupling_keeps_the_starting_point(tiny_problem):
    p = tiny_problem
    c = p.cfg
    Z = lambda a: np.zeros_like(a)  # noqa: E731
    stat = np.array([0.01, -0.02])
    ev = evgw(p.eps, c.n_fc, c.n_occ, p.qp, Z(p.R_oo), Z(p.R_ov) + 1e-30, Z(p.R_qp),
              n_cycles=3, eps_naf=-1.0, n_freq=16, n_pade=8, static=stat)
    for cyc in range(3):
        assert np.allclose(ev.eps_qp[cyc], p.eps[p.qp] + stat, atol=1e-14)


def test_cycles_approach_a_fixed_point(tiny_problem):
    ev = evgw_problem(tiny_problem, n_cycles=6)
    steps = np.max(np.abs(np.diff(ev.eps_qp, axis=0)), axis=1)
    assert steps[-1] < 0.2 * steps[0]
    assert np.all(ev.converged)
