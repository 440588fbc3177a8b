"""Pins for the oracle's quadrature grids (closed forms, equioscillation,
brute force)."""
import numpy as np
import pytest

from oracle import grids


@pytest.mark.parametrize("a", [0.05, 0.3, 1.0, 4.0])
def test_mgl_lorentzian_closed_form(a):
    # int_0^inf dw / (w^2 + a^2) = pi / (2 a).  Under w = x0 (1+t)/(1-t) the
    # integrand becomes a low-degree rational in t, integrated to rounding.
    for n in (32, 128):
        w, wt = grids.modified_gauss_legendre(n, 0.5)
        err = abs(np.sum(wt / (w * w + a * a)) - np.pi / (2 * a)) / (np.pi / (2 * a))
        assert err < 1e-10


def test_mgl_two_pole_closed_form():
    # int_0^inf a/(a^2+w^2) 1/(w^2+W^2) dw = pi / (2 W (a + W)), Re a > 0
    w, wt = grids.modified_gauss_legendre(256, 0.5)
    for a in (0.2 + 0.3j, 1.0 + 2.0j, 0.7 + 0.0j):
        for Om in (0.4, 2.5):
            num = np.sum(wt * a / (a * a + w * w) / (w * w + Om * Om))
            ref = np.pi / (2 * Om * (a + Om))
            assert abs(num - ref) < 1e-6 * abs(ref)


def test_mgl_exponential_and_ordering():
    w, wt = grids.modified_gauss_legendre(64, 0.5)
    assert np.all(np.diff(w) > 0) and np.all(w > 0) and np.all(wt > 0)
    assert abs(np.sum(wt * np.exp(-w)) - 1.0) < 1e-10
    # the mapping sends t = 0 to x0: the median node pair brackets x0
    assert w[31] < 0.5 < w[32]


def _alternation(alpha, omega, R, k):
    pts, vals = grids._extrema(R, alpha, omega, k, n_grid=40000)
    return pts, vals


@pytest.mark.parametrize("k,R", [(3, 50.0), (5, 2e3), (8, 8.16e4)])
def test_minimax_equioscillates(k, R):
    alpha, omega, e1 = grids.minimax_inverse(k, R)
    assert np.all(alpha > 0) and np.all(omega > 0)
    pts, vals = _alternation(alpha, omega, R, k)
    assert pts.size == 2 * k + 1
    assert np.all(np.sign(vals[1:]) == -np.sign(vals[:-1]))
    assert np.max(np.abs(vals)) - np.min(np.abs(vals)) < 1e-8 * abs(e1)
    xs = np.exp(np.linspace(0.0, np.log(R), 400000))
    assert np.max(np.abs(grids._err(xs, alpha, omega))) <= abs(e1) * (1 + 1e-8)
    assert 1.0 <= pts[0] and pts[-1] <= R


def test_minimax_error_decreases_with_k():
    errs = [abs(grids.minimax_inverse(k, 1e4)[2]) for k in (4, 6, 8, 10)]
    assert all(b < a for a, b in zip(errs, errs[1:]))


def test_minimax_k1_brute_force():
    # brute force over (alpha, omega) never beats the Remez level
    R = 10.0
    alpha, omega, e1 = grids.minimax_inverse(1, R)
    xs = np.exp(np.linspace(0.0, np.log(R), 2000))
    best = np.inf
    for a in np.linspace(0.5 * alpha[0], 1.5 * alpha[0], 201):
        for w in np.linspace(0.5 * omega[0], 1.5 * omega[0], 201):
            best = min(best, np.max(np.abs(1 / xs - w * np.exp(-a * xs))))
    assert best >= abs(e1) * (1 - 1e-9)
    assert best <= abs(e1) * 1.01


def test_lt_grid_scaling_and_bounds():
    x, w, err = grids.lt_grid(6, 0.25, 1e3)
    ys = np.exp(np.linspace(np.log(0.25), np.log(1e3), 20000))
    approx = np.exp(-np.outer(ys, x)) @ w
    # absolute error of 1/y bounded by err / y_min
    assert np.max(np.abs(approx - 1 / ys)) <= err / 0.25 * (1 + 1e-6)
    eps = np.array([-20.0, -15.0, -1.0, -0.4, 0.1, 2.0, 3.0])
    lo, hi = grids.lt_bounds(eps, n_fc=1, n_occ=4, omega_min=0.01)
    assert lo == pytest.approx(0.5 ** 2 + 0.01 ** 2)
    assert hi == 1e4                       # (3 - (-15))^2 = 324 -> raised to 1e4
    eps2 = np.array([-120.0, -0.4, 0.1, 30.0])
    assert grids.lt_bounds(eps2, 0, 2, 0.0)[1] == pytest.approx(150.0 ** 2)
