"""Frequency and Laplace quadrature grids (oracle; test infrastructure only).

* Modified Gauss-Legendre grid on [0, inf) used for the frequency integral of
  the correlation self-energy (Sec. 2 after Eq. 7; Sec. 3 uses 128 points
  for integration and a separate grid of 70 points for the Pade fit).  The
  scale x0 of the mapping is not given in the paper; x0 = 0.5 Ha is used.
* Minimax exponential-sum approximation of 1/y (Eq. 8 and Eq. 9; Sec. 3:
  the bounds of y are the squared HOMO-LUMO gap plus the squared smallest
  frequency, and the squared largest occupied-virtual difference, raised to
  at least 1e4).  Eq. 9 prints a minus sign in front of the sum; with
  positive weights and exponents the approximation of a positive function
  carries a plus sign, which is the reading taken here.

The minimax solution is computed here by an algorithm of its own: a
two-parameter trapezoid initial guess, L_p-norm refinement with increasing
p by SciPy's least squares, and a Remez exchange whose alternation system is
solved by SciPy's ``fsolve``.  The best approximation is unique, so any
correct algorithm lands on the same grid.
"""
from __future__ import annotations

import numpy as np
from scipy import optimize


def modified_gauss_legendre(n: int, x0: float = 0.5):
    """Nodes and weights for int_0^inf f(w) dw with w = x0 (1+t)/(1-t).

    t_k, v_k are the n-point Gauss-Legendre nodes and weights on [-1, 1];
    dw/dt = 2 x0 / (1-t)^2.  Returned in ascending order of w.
    """
    t, v = np.polynomial.legendre.leggauss(n)
    w = x0 * (1.0 + t) / (1.0 - t)
    wt = v * 2.0 * x0 / (1.0 - t) ** 2
    order = np.argsort(w)
    return w[order], wt[order]


# ----------------------------------------------------------------------------
# minimax approximation of 1/x on [1, R] by sum_nu omega_nu exp(-alpha_nu x)
# ----------------------------------------------------------------------------

def _expsum(x, alpha, omega):
    return np.exp(-np.outer(x, alpha)) @ omega


def _err(x, alpha, omega):
    return 1.0 / x - _expsum(x, alpha, omega)


def _trapezoid_guess(k: int, R: float, xs: np.ndarray):
    """1/x = int exp(t - x e^t) dt discretised at t = a + nu h."""
    def maxerr(p):
        a, h = p
        if h <= 0:
            return 1e300
        t = a + h * np.arange(k)
        return np.max(np.abs(_err(xs, np.exp(t), h * np.exp(t))))

    best = None
    for h in np.linspace(0.2, 3.0, 29):
        for a in np.linspace(-np.log(R) - 4.0, 0.0, 41):
            e = maxerr((a, h))
            if best is None or e < best[0]:
                best = (e, a, h)
    res = optimize.minimize(maxerr, x0=[best[1], best[2]], method="Nelder-Mead",
                            options={"xatol": 1e-10, "fatol": 1e-16, "maxiter": 4000})
    a, h = res.x
    t = a + h * np.arange(k)
    return np.exp(t), h * np.exp(t)


def _lp_refine(k, R, xs, alpha, omega):
    """Minimise the L_p norm of the error for p = 2, 4, ..., 128; return the
    last iterate whose error curve still has 2k+1 alternating extrema."""
    theta = np.concatenate([np.log(omega), np.log(alpha)])
    best = None
    for p in (2, 4, 8, 16, 32, 64, 128):
        scale = np.max(np.abs(_err(xs, np.exp(theta[k:]), np.exp(theta[:k]))))

        def resid(th, p=p, scale=scale):
            e = _err(xs, np.exp(th[k:]), np.exp(th[:k])) / scale
            return np.sign(e) * np.abs(e) ** (p / 2.0)

        sol = optimize.least_squares(resid, theta, method="lm", xtol=1e-15,
                                     ftol=1e-15, gtol=1e-15, max_nfev=20000)
        theta = sol.x
        a, w = np.exp(theta[k:]), np.exp(theta[:k])
        if _extrema(R, a, w, k)[0].size == 2 * k + 1:
            best = (a, w)
    if best is None:
        raise RuntimeError("L_p refinement found no equioscillating start")
    return best


def _extrema(R, alpha, omega, k, n_grid=20000):
    """Alternating extrema of the error on [1, R] (endpoints included)."""
    xs = np.exp(np.linspace(0.0, np.log(R), n_grid))
    e = _err(xs, alpha, omega)

    def de(x):
        return -1.0 / x ** 2 + (np.exp(-np.outer(np.atleast_1d(x), alpha)) @ (alpha * omega))

    cand = [1.0]
    d = np.diff(e)
    for i in range(1, n_grid - 1):
        if d[i - 1] * d[i] < 0:
            lo, hi = xs[i - 1], xs[i + 1]
            try:
                cand.append(optimize.brentq(lambda x: de(x)[0], lo, hi, xtol=1e-15 * hi))
            except ValueError:
                cand.append(xs[i])
    cand.append(R)
    cand = np.array(cand)
    ev = _err(cand, alpha, omega)
    # merge neighbours of equal sign, keeping the larger |e|
    pts, vals = [cand[0]], [ev[0]]
    for x, v in zip(cand[1:], ev[1:]):
        if np.sign(v) == np.sign(vals[-1]):
            if abs(v) > abs(vals[-1]):
                pts[-1], vals[-1] = x, v
        else:
            pts.append(x)
            vals.append(v)
    pts, vals = np.array(pts), np.array(vals)
    while pts.size > 2 * k + 1:       # drop the smaller end
        if abs(vals[0]) < abs(vals[-1]):
            pts, vals = pts[1:], vals[1:]
        else:
            pts, vals = pts[:-1], vals[:-1]
    return pts, vals


def _remez(k, R, alpha, omega, max_iter=60, tol=1e-12):
    E = 0.0
    for _ in range(max_iter):
        pts, vals = _extrema(R, alpha, omega, k)
        if pts.size != 2 * k + 1:
            raise RuntimeError(f"found {pts.size} alternation points, need {2 * k + 1}")
        emax = np.max(np.abs(vals))
        emin = np.min(np.abs(vals))
        if emax - emin <= tol * emax:
            return alpha, omega, vals[0], pts
        sgn = np.sign(vals[0]) * (-1.0) ** np.arange(2 * k + 1)

        def F(th):
            om, al, Ev = np.exp(th[:k]), np.exp(th[k:2 * k]), th[2 * k]
            return (_err(pts, al, om) - sgn * Ev) / emax

        th0 = np.concatenate([np.log(omega), np.log(alpha), [np.mean(np.abs(vals))]])
        th, info, ier, msg = optimize.fsolve(F, th0, full_output=True, xtol=1e-14)
        omega, alpha, E = np.exp(th[:k]), np.exp(th[k:2 * k]), th[2 * k]
    pts, vals = _extrema(R, alpha, omega, k)
    return alpha, omega, vals[0], pts


def minimax_inverse(k: int, R: float):
    """Best uniform approximation of 1/x on [1, R] by k exponentials.

    Returns (alpha, omega, err) with alpha ascending and err the signed error
    at x = 1; |err| is the equioscillation level.
    """
    xs = np.exp(np.linspace(0.0, np.log(R), 3000))
    alpha, omega = _trapezoid_guess(k, R, xs)
    alpha, omega = _lp_refine(k, R, xs, alpha, omega)
    alpha, omega, e1, _ = _remez(k, R, alpha, omega)
    order = np.argsort(alpha)
    return alpha[order], omega[order], e1


def lt_grid(k: int, y_min: float, y_max: float):
    """Laplace points x_m and weights w_m with 1/y ~ sum_m w_m exp(-x_m y)
    on [y_min, y_max] (Eq. 9, plus-sign reading); also the normalised
    maximum error max |1/t - sum| on t = y / y_min in [1, y_max / y_min]."""
    alpha, omega, e1 = minimax_inverse(k, y_max / y_min)
    return alpha / y_min, omega / y_min, abs(e1)


def lt_bounds(eps: np.ndarray, n_fc: int, n_occ: int, omega_min: float):
    """Sec. 3: lower bound (e_LUMO - e_HOMO)^2 + omega_min^2; upper bound the
    squared largest active occupied-virtual gap, at least 1e4."""
    e_homo, e_lumo = eps[n_occ - 1], eps[n_occ]
    lo = (e_lumo - e_homo) ** 2 + omega_min ** 2
    hi = max((eps[-1] - eps[n_fc]) ** 2, 1e4)
    return lo, hi
