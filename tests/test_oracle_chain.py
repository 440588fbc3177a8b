"""Pins for the oracle's NAF, polarizability, screening, self-energy, Pade
and QP steps: two-level closed forms, invariants, brute force and the
real-axis Casida reference."""
import numpy as np
import pytest

from conftest import HARTREE_MEV, two_level
from oracle import casida, grids, naf, pade, rpa, sigma
from oracle.g0w0 import g0w0, g0w0_problem

S = 2.0


# ---------------------------------------------------------------- two-level

def _two_level_arrays(t):
    # active orbitals: i (occupied), a (virtual); one aux function
    eps = np.array([t["e_i"], t["e_a"]])
    R_ov = np.array([[t["r"]]])
    R_oo = np.array([[[t["p"]]]])
    R_qp = np.array([[[t["p"]], [t["r"]]],     # n = i: m = i, a
                     [[t["r"]], [t["q"]]]])    # n = a: m = i, a
    return eps, R_oo, R_ov, R_qp


def test_two_level_pi_and_screening_closed_form():
    t = two_level()
    d = np.array([t["e_a"] - t["e_i"]])
    om = np.array([0.0, 0.3, 2.0])
    Pi = rpa.pi_sos(np.array([[t["r"]]]), d, om)
    ref = -2 * S * t["r"] ** 2 * d[0] / (om ** 2 + d[0] ** 2)
    assert np.allclose(Pi[:, 0, 0], ref, rtol=1e-14)
    Wh = rpa.screen(Pi)
    Om2 = d[0] ** 2 + 2 * S * t["r"] ** 2 * d[0]
    assert np.allclose(Wh[:, 0, 0], -2 * S * t["r"] ** 2 * d[0] / (om ** 2 + Om2), rtol=1e-13)
    Rq = np.array([[[t["p"]], [t["r"]]]])
    W = rpa.w_diag(Rq, Wh)
    assert np.allclose(W[:, 0, 0], t["p"] ** 2 * Wh[:, 0, 0], rtol=1e-14)
    assert np.allclose(W[:, 0, 1], t["r"] ** 2 * Wh[:, 0, 0], rtol=1e-14)


def _two_level_sigma_exact(t, z, n):
    d = t["e_a"] - t["e_i"]
    Om = np.sqrt(d * d + 2 * S * t["r"] ** 2 * d)
    K = S * t["r"] ** 2 * d / Om
    Rn = {0: (t["p"], t["r"]), 1: (t["r"], t["q"])}[n]
    return Rn[0] ** 2 * K / (z - t["e_i"] + Om) + Rn[1] ** 2 * K / (z - t["e_a"] - Om)


def test_two_level_sigma_quadrature_converges_to_closed_form():
    t = two_level()
    eps, R_oo, R_ov, R_qp = _two_level_arrays(t)
    ef = 0.5 * (t["e_i"] + t["e_a"])
    wk = np.array([0.05, 0.5, 3.0])
    errs = []
    for F in (32, 128, 512):
        om, wt = grids.modified_gauss_legendre(F, 0.5)
        Pi = rpa.pi_sos(R_ov, np.array([t["e_a"] - t["e_i"]]), om)
        W = rpa.w_diag(R_qp, rpa.screen(Pi))
        Sg = sigma.sigma_iw(W, eps, ef, om, wt, wk)
        ref = np.array([[_two_level_sigma_exact(t, ef + 1j * w, n) for w in wk] for n in (0, 1)])
        errs.append(np.max(np.abs(Sg - ref)) / np.max(np.abs(ref)))
    assert errs[-1] < errs[0] and errs[-1] < 1e-6


def test_two_level_qp_matches_exact_root():
    t = two_level()
    eps, R_oo, R_ov, R_qp = _two_level_arrays(t)
    res = g0w0(eps, 0, 1, np.array([0, 1]), R_oo, R_ov, R_qp, eps_naf=0.0,
               n_freq=512, n_pade=16, eta=1e-3, tol=1e-12, max_iter=500)
    for q, n in enumerate((0, 1)):
        E = eps[n]
        for _ in range(2000):
            E = eps[n] + _two_level_sigma_exact(t, E + 1e-3j, n).real
        assert abs(res.eps_qp[q] - E) * HARTREE_MEV < 1e-3
        h = 1e-6
        dS = (_two_level_sigma_exact(t, E + h + 1e-3j, n).real
              - _two_level_sigma_exact(t, E - h + 1e-3j, n).real) / (2 * h)
        assert abs(res.z[q] - 1 / (1 - dS)) < 1e-4


# ---------------------------------------------------------------- NAF

def _full_pair_metric(prob):
    """Brute force over ordered active pairs (n, m) not both virtual."""
    c = prob.cfg
    from gwsynth.problem import _RowSource
    rng = np.random.default_rng(c.seed)
    from gwsynth.problem import _energies
    _energies(c, rng)
    src = _RowSource(c, rng)
    act = np.arange(c.n_fc, c.n_occ + c.n_virt)
    K = np.zeros((c.n_aux, c.n_aux))
    for n in act:
        for m in act:
            if n >= c.n_occ and m >= c.n_occ:
                continue
            row = src.rows(np.array([n]), np.array([m]))[0]
            K += np.outer(row, row)
    return 2.0 * K


def test_naf_metric_brute_force(tiny_problem):
    K = naf.naf_metric(tiny_problem.R_oo, tiny_problem.R_ov)
    Kb = _full_pair_metric(tiny_problem)
    assert np.allclose(K, Kb, rtol=1e-12, atol=1e-14 * np.abs(Kb).max())
    lam = np.linalg.eigvalsh(K)
    assert np.all(lam > 0)                    # SPD (Eq. 11)


def test_naf_threshold_selection():
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    lam = np.array([5.0, 2.0, 1.0, 0.5, 0.1, 0.01])
    K = (Q * lam) @ Q.T
    l, U = naf.naf_basis(K, 0.3)
    assert U.shape == (6, 4) and np.allclose(l, lam, rtol=1e-12)
    assert naf.naf_basis(K, 0.5 + 1e-9)[1].shape[1] == 3   # strict ">"
    assert naf.naf_basis(K, 0.5 - 1e-9)[1].shape[1] == 4
    assert naf.naf_basis(K, 0.0, max_keep=2)[1].shape[1] == 2
    # projector onto the kept space
    P = U @ U.T
    assert np.allclose(P, (Q[:, :4]) @ Q[:, :4].T, atol=1e-12)


def test_naf_zero_threshold_reproduces_uncompressed(tiny_problem, tiny_sos):
    p = tiny_problem
    c = p.cfg
    ident = g0w0(p.eps, c.n_fc, c.n_occ, p.qp, p.R_oo, p.R_ov, p.R_qp, eps_naf=0.0,
                 n_freq=c.n_freq, n_pade=c.n_pade, U=np.eye(c.n_aux))
    assert tiny_sos.n_naf == c.n_aux
    assert np.allclose(tiny_sos.U.T @ tiny_sos.U, np.eye(c.n_aux), atol=1e-12)
    assert np.allclose(ident.W, tiny_sos.W, rtol=1e-9, atol=1e-13)
    assert np.allclose(ident.sigma, tiny_sos.sigma, rtol=1e-9, atol=1e-13)
    assert np.max(np.abs(ident.eps_qp - tiny_sos.eps_qp)) < 1e-10


def test_naf_rotation_invariance(tiny_problem, tiny_sos, rng):
    p = tiny_problem
    c = p.cfg
    U = tiny_sos.U[:, :90]
    O, _ = np.linalg.qr(rng.standard_normal((90, 90)))
    r1 = g0w0(p.eps, c.n_fc, c.n_occ, p.qp, p.R_oo, p.R_ov, p.R_qp, eps_naf=0.0,
              n_freq=c.n_freq, n_pade=c.n_pade, U=U)
    r2 = g0w0(p.eps, c.n_fc, c.n_occ, p.qp, p.R_oo, p.R_ov, p.R_qp, eps_naf=0.0,
              n_freq=c.n_freq, n_pade=c.n_pade, U=U @ O)
    assert np.allclose(r1.W, r2.W, rtol=1e-9, atol=1e-13)
    assert np.max(np.abs(r1.eps_qp - r2.eps_qp)) < 1e-10


# ---------------------------------------------------------------- invariants

def test_polarizability_invariants(tiny_problem, tiny_sos, tiny_lt_grid):
    p = tiny_problem
    c = p.cfg
    d = rpa.delta_ov(p.eps, c.n_fc, c.n_occ)
    assert np.all(d > 0)
    x, w = tiny_lt_grid[0], tiny_lt_grid[1]
    M = rpa.m_lt(tiny_sos.Rt_ov, d, x, w)
    for m in range(len(x)):
        assert np.allclose(M[m], M[m].T, rtol=0, atol=1e-14 * np.abs(M[m]).max())
        assert np.linalg.eigvalsh(M[m]).min() > -1e-12 * np.abs(M[m]).max()
    Pi = rpa.pi_sos(tiny_sos.Rt_ov, d, tiny_sos.omega)
    Wh = rpa.screen(Pi)
    for j in range(len(tiny_sos.omega)):
        assert np.linalg.eigvalsh(Pi[j]).max() < 1e-12
        assert np.linalg.eigvalsh(np.eye(Pi.shape[1]) - Pi[j]).min() >= 1 - 1e-10
        assert np.linalg.eigvalsh(0.5 * (Wh[j] + Wh[j].T)).max() < 1e-12
    Q = len(p.qp)
    for q in range(Q):
        n_rel = p.qp[q] - c.n_fc
        assert np.all(tiny_sos.W[:, q, n_rel] <= 0)


def test_m_lt_brute_force_loop(tiny_problem, tiny_sos, tiny_lt_grid):
    p = tiny_problem
    c = p.cfg
    x, w = tiny_lt_grid[0][:2], tiny_lt_grid[1][:2]
    Rt = tiny_sos.Rt_ov[:, :12]
    M = rpa.m_lt(Rt, rpa.delta_ov(p.eps, c.n_fc, c.n_occ), x, w)
    o, v = c.n_act_occ, c.n_virt
    for m in range(2):
        ref = np.zeros((12, 12))
        for i in range(o):
            for a in range(v):
                dd = p.eps[c.n_occ + a] - p.eps[c.n_fc + i]
                f = w[m] * dd * np.exp(-dd * dd * x[m])
                row = Rt[i * v + a]
                ref += f * np.outer(row, row)
        assert np.allclose(M[m], ref, rtol=1e-12, atol=1e-16)


def test_m_lt_columns_brute_force_loop(tiny_problem, tiny_sos, tiny_lt_grid):
    """The column-restricted Laplace matrices against the explicit ia loop."""
    p = tiny_problem
    c = p.cfg
    x, w = tiny_lt_grid[0][:2], tiny_lt_grid[1][:2]
    Rt = tiny_sos.Rt_ov[:, :20]
    cols = np.array([0, 7, 19])
    Mc = rpa.m_lt_columns(Rt, rpa.delta_ov(p.eps, c.n_fc, c.n_occ), x, w, cols)
    assert Mc.shape == (2, 20, 3)
    o, v = c.n_act_occ, c.n_virt
    for m in range(2):
        ref = np.zeros((20, 3))
        for i in range(o):
            for a in range(v):
                dd = p.eps[c.n_occ + a] - p.eps[c.n_fc + i]
                f = w[m] * dd * np.exp(-dd * dd * x[m])
                row = Rt[i * v + a]
                ref += f * np.outer(row, row[cols])
        assert np.allclose(Mc[m], ref, rtol=1e-12, atol=1e-16)


def test_lt_polarizability_converges_to_sos(tiny_problem, tiny_sos):
    p = tiny_problem
    c = p.cfg
    d = rpa.delta_ov(p.eps, c.n_fc, c.n_occ)
    om = tiny_sos.omega
    Pi = rpa.pi_sos(tiny_sos.Rt_ov, d, om)
    lo, hi = grids.lt_bounds(p.eps, c.n_fc, c.n_occ, om[0])
    errs = []
    for L in (6, 10, 14):
        x, w, _ = grids.lt_grid(L, lo, hi)
        Pl = rpa.pi_lt(rpa.m_lt(tiny_sos.Rt_ov, d, x, w), x, om)
        # frequencies inside the window [lo, hi] of y = w^2 + D^2
        sel = om ** 2 + d.max() ** 2 <= hi
        errs.append(np.linalg.norm(Pl[sel] - Pi[sel]) / np.linalg.norm(Pi[sel]))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-3


def test_lt_qp_error_shrinks_with_grid(tiny_problem, tiny_sos):
    p = tiny_problem
    c = p.cfg
    lo, hi = grids.lt_bounds(p.eps, c.n_fc, c.n_occ, tiny_sos.omega[0])
    errs = []
    for L in (8, 12, 16):
        x, w, _ = grids.lt_grid(L, lo, hi)
        r = g0w0_problem(p, lt=(x, w))
        errs.append(np.max(np.abs(r.eps_qp - tiny_sos.eps_qp)) * HARTREE_MEV)
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.1                  # Sec. 3: < 0.1 meV at tight grids


# ---------------------------------------------------------------- sigma / pade

def test_sigma_conjugation_symmetry(tiny_problem, tiny_sos):
    p = tiny_problem
    c = p.cfg
    wk = np.array([0.1, 1.0])
    eps_m = p.eps[c.n_fc:]
    Sp = sigma.sigma_iw(tiny_sos.W, eps_m, tiny_sos.eps_f, tiny_sos.omega, tiny_sos.w_omega, wk)
    Sm = sigma.sigma_iw(tiny_sos.W, eps_m, tiny_sos.eps_f, tiny_sos.omega, tiny_sos.w_omega, -wk)
    assert np.allclose(Sm, np.conj(Sp), rtol=1e-13, atol=1e-16)


def test_zero_tensor_gives_zero_sigma(tiny_problem):
    p = tiny_problem
    c = p.cfg
    z = np.zeros_like
    static = np.array([0.01, -0.02])
    r = g0w0(p.eps, c.n_fc, c.n_occ, p.qp, z(p.R_oo), z(p.R_ov), z(p.R_qp),
             eps_naf=-1.0, n_freq=16, n_pade=8, static=static)
    assert np.all(r.sigma == 0)
    assert np.allclose(r.eps_qp, p.eps[p.qp] + static, atol=1e-15)


def test_pade_interpolates_and_reproduces_rational():
    rng = np.random.default_rng(7)
    wn, _ = grids.modified_gauss_legendre(16, 0.5)
    zn = 1j * wn
    poles = np.array([-0.7 + 0.0j, 0.4, 1.3])
    res = np.array([0.2, 0.05, 0.3])

    def f(z):
        return np.sum(res[None, :] / (np.atleast_1d(z)[:, None] - poles[None, :]), axis=1)

    a = pade.thiele_coefficients(zn, f(zn))
    for k in range(16):
        assert abs(pade.thiele_eval(zn, a, zn[k]) - f(zn[k])[0]) < 1e-12
    for z in (-0.3 + 0.001j, 0.1 + 0.001j, 2.0 + 0.05j, 0.8 + 1.0j):
        assert abs(pade.thiele_eval(zn, a, z) - f(z)[0]) < 1e-9 * (1 + abs(f(z)[0]))
    # random data: still interpolates
    u = rng.standard_normal(16) + 1j * rng.standard_normal(16)
    a2 = pade.thiele_coefficients(zn, u)
    assert max(abs(pade.thiele_eval(zn, a2, zn[k]) - u[k]) for k in range(16)) < 1e-9


# ---------------------------------------------------------------- Casida

def test_casida_reduces_to_bare_poles_without_coupling():
    d = np.array([0.5, 1.2, 3.0])
    Rt = np.zeros((3, 4))
    Om, rho = casida.rpa_excitations(Rt, d)
    assert np.allclose(np.sort(Om), d, rtol=1e-14)


def test_casida_matches_imaginary_axis_chain(tiny_problem, tiny_sos):
    p = tiny_problem
    c = p.cfg
    d = rpa.delta_ov(p.eps, c.n_fc, c.n_occ)
    Om, rho = casida.rpa_excitations(tiny_sos.Rt_ov, d)
    eps_m = p.eps[c.n_fc:]
    # W(iw) from the excitations equals Eq. 2 (exact, no quadrature)
    wk = tiny_sos.omega[[0, 10, 25]]
    Pi = rpa.pi_sos(tiny_sos.Rt_ov, d, wk)
    W = rpa.w_diag(tiny_sos.Rt_qp, rpa.screen(Pi))
    wnm = np.einsum("qmp,kp->qmk", tiny_sos.Rt_qp, rho)
    Wc = -np.einsum("qmk,jk->jqm", wnm ** 2, 2 * Om[None, :] / (wk[:, None] ** 2 + Om[None, :] ** 2))
    assert np.allclose(W, Wc, rtol=1e-9, atol=1e-14)
    # Sigma on the Pade nodes converges with the frequency grid
    S_c = casida.sigma_casida(tiny_sos.Rt_qp, eps_m, tiny_sos.eps_f, Om, rho,
                              tiny_sos.eps_f + 1j * tiny_sos.omega_pade)
    errs = [np.max(np.abs(g0w0_problem(p, n_freq=F).sigma - S_c)) for F in (32, 128, 512)]
    assert errs[0] > errs[1] > errs[2]
    # QP energies: AC + quadrature error far below 1 meV for HOMO / LUMO
    for q, n in enumerate(p.qp):
        E, ok = casida.qp_casida(p.eps[n], 0.0, tiny_sos.Rt_qp[q], eps_m,
                                 tiny_sos.eps_f, Om, rho, c.eta)
        assert ok
        assert abs(E - tiny_sos.eps_qp[q]) * HARTREE_MEV < 0.01
