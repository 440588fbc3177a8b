// Host-side FP64 grids and problem preparation (rows a1 and a3 of the path).
//
//  * gw_prepare: frozen-core ranges, Fermi level and the Laplace interval
//    (Sec. 3, computational details).
//  * gw_freq_grid_mgl: modified Gauss-Legendre rule on [0, inf) (Sec. 2 after
//    Eq. 7).  Legendre nodes by Newton's method on the three-term recurrence.
//  * gw_lt_grid_minimax: best uniform approximation of 1/y by a sum of
//    exponentials (Eqs. 8-9, Sec. 3).  Trapezoid start in log(alpha),
//    Levenberg-Marquardt on L_p norms of growing p, then a Remez exchange
//    whose alternation system is solved by damped Newton.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"

namespace {

constexpr int kMaxLt = 20;

struct ExpSum {
  int k = 0;
  double al[kMaxLt] = {};
  double om[kMaxLt] = {};
};

inline double err_at(const ExpSum& s, double x) {
  double v = 1.0 / x;
  for (int i = 0; i < s.k; ++i) v -= s.om[i] * std::exp(-s.al[i] * x);
  return v;
}

inline double derr_at(const ExpSum& s, double x) {
  double v = -1.0 / (x * x);
  for (int i = 0; i < s.k; ++i) v += s.om[i] * s.al[i] * std::exp(-s.al[i] * x);
  return v;
}

double max_err(const ExpSum& s, const std::vector<double>& xs) {
  double m = 0;
  for (double x : xs) m = std::max(m, std::fabs(err_at(s, x)));
  return m;
}

// Gaussian elimination with partial pivoting, A row-major n x n (destroyed).
bool solve_dense(int n, std::vector<double>& A, std::vector<double>& b) {
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[p * n + c])) p = r;
    if (!(std::fabs(A[p * n + c]) > 0)) return false;
    if (p != c) {
      for (int j = 0; j < n; ++j) std::swap(A[c * n + j], A[p * n + j]);
      std::swap(b[c], b[p]);
    }
    for (int r = c + 1; r < n; ++r) {
      double f = A[r * n + c] / A[c * n + c];
      if (f == 0) continue;
      for (int j = c; j < n; ++j) A[r * n + j] -= f * A[c * n + j];
      b[r] -= f * b[c];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    double v = b[r];
    for (int j = r + 1; j < n; ++j) v -= A[r * n + j] * b[j];
    b[r] = v / A[r * n + r];
  }
  return true;
}

ExpSum trapezoid(int k, double a, double h) {
  ExpSum s;
  s.k = k;
  for (int i = 0; i < k; ++i) {
    double t = a + h * i;
    s.al[i] = std::exp(t);
    s.om[i] = h * std::exp(t);
  }
  return s;
}

// 1/x = int exp(t - x e^t) dt sampled at t = a + i h: scan then pattern search.
ExpSum initial_guess(int k, double R, const std::vector<double>& xs) {
  double best = 1e300, ba = 0, bh = 1;
  for (double h = 0.2; h <= 3.0 + 1e-12; h += 0.1)
    for (double a = -std::log(R) - 4.0; a <= 1e-12; a += 0.1) {
      double e = max_err(trapezoid(k, a, h), xs);
      if (e < best) { best = e; ba = a; bh = h; }
    }
  for (double step = 0.05; step > 1e-7; step *= 0.5) {
    bool moved = true;
    while (moved) {
      moved = false;
      const double da[4] = {step, -step, 0, 0}, dh[4] = {0, 0, step, -step};
      for (int d = 0; d < 4; ++d) {
        double a = ba + da[d], h = bh + dh[d];
        if (h <= 0) continue;
        double e = max_err(trapezoid(k, a, h), xs);
        if (e < best) { best = e; ba = a; bh = h; moved = true; }
      }
    }
  }
  return trapezoid(k, ba, bh);
}

// Alternating extrema of the error on [1, R] (endpoints included).
void extrema(const ExpSum& s, double R, std::vector<double>& pts,
             std::vector<double>& vals, int n_grid = 4000) {
  const double lr = std::log(R);
  std::vector<double> xs(n_grid), e(n_grid);
  for (int i = 0; i < n_grid; ++i) {
    xs[i] = std::exp(lr * i / (n_grid - 1));
    e[i] = err_at(s, xs[i]);
  }
  std::vector<double> cand{1.0};
  for (int i = 1; i < n_grid - 1; ++i) {
    double d0 = e[i] - e[i - 1], d1 = e[i + 1] - e[i];
    if (d0 * d1 < 0) {
      double lo = xs[i - 1], hi = xs[i + 1];
      double flo = derr_at(s, lo), fhi = derr_at(s, hi);
      if (flo * fhi < 0) {
        for (int it = 0; it < 200 && hi - lo > 1e-15 * hi; ++it) {
          double mid = 0.5 * (lo + hi), fm = derr_at(s, mid);
          if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else { hi = mid; }
        }
        cand.push_back(0.5 * (lo + hi));
      } else {
        cand.push_back(xs[i]);
      }
    }
  }
  cand.push_back(R);
  pts.clear();
  vals.clear();
  for (double x : cand) {
    double v = err_at(s, x);
    if (!vals.empty() && ((v < 0) == (vals.back() < 0))) {
      if (std::fabs(v) > std::fabs(vals.back())) { pts.back() = x; vals.back() = v; }
    } else {
      pts.push_back(x);
      vals.push_back(v);
    }
  }
  while ((int)pts.size() > 2 * s.k + 1) {
    if (std::fabs(vals.front()) < std::fabs(vals.back())) {
      pts.erase(pts.begin());
      vals.erase(vals.begin());
    } else {
      pts.pop_back();
      vals.pop_back();
    }
  }
}

ExpSum from_theta(int k, const double* th) {
  ExpSum s;
  s.k = k;
  for (int i = 0; i < k; ++i) {
    s.om[i] = std::exp(th[i]);
    s.al[i] = std::exp(th[k + i]);
  }
  return s;
}

// Levenberg-Marquardt on sum_i |e_i / scale|^p, p = p0 .. 128 (doubling).
// Keeps the last iterate whose error still alternates 2k+1 times.
bool lp_refine(int k, double R, const std::vector<double>& xs, ExpSum& s, int p0 = 2) {
  const int n = 2 * k, m = (int)xs.size();
  std::vector<double> th(n), J((size_t)m * n), r(m), JtJ(n * n), g(n);
  for (int i = 0; i < k; ++i) { th[i] = std::log(s.om[i]); th[k + i] = std::log(s.al[i]); }
  bool have = false;
  ExpSum best = s;
  std::vector<double> pts, vals;
  for (int p = p0; p <= 128; p *= 2) {
    const double scale = max_err(from_theta(k, th.data()), xs);
    auto cost = [&](const std::vector<double>& t) {
      ExpSum q = from_theta(k, t.data());
      double c = 0;
      for (int i = 0; i < m; ++i) c += std::pow(std::fabs(err_at(q, xs[i]) / scale), p);
      return c;
    };
    double c0 = cost(th), lam = 1e-3;
    for (int it = 0; it < 400; ++it) {
      ExpSum q = from_theta(k, th.data());
      for (int i = 0; i < m; ++i) {
        double e = err_at(q, xs[i]) / scale, ae = std::fabs(e);
        r[i] = (e < 0 ? -1.0 : 1.0) * std::pow(ae, 0.5 * p);
        double f = 0.5 * p * std::pow(ae, 0.5 * p - 1.0) / scale;
        for (int j = 0; j < k; ++j) {
          double ex = std::exp(-q.al[j] * xs[i]);
          J[(size_t)i * n + j] = f * (-q.om[j] * ex);
          J[(size_t)i * n + k + j] = f * (q.om[j] * q.al[j] * xs[i] * ex);
        }
      }
      for (int a = 0; a < n; ++a) {
        g[a] = 0;
        for (int i = 0; i < m; ++i) g[a] += J[(size_t)i * n + a] * r[i];
        for (int b = 0; b <= a; ++b) {
          double v = 0;
          for (int i = 0; i < m; ++i) v += J[(size_t)i * n + a] * J[(size_t)i * n + b];
          JtJ[a * n + b] = JtJ[b * n + a] = v;
        }
      }
      bool improved = false;
      for (int tries = 0; tries < 30; ++tries) {
        std::vector<double> A(JtJ), d(n);
        // Marquardt scaling plus a small ridge: a term whose exponential has
        // underflowed on [1, R] leaves a zero column that would stop the solve.
        double dmax = 0;
        for (int a = 0; a < n; ++a) dmax = std::max(dmax, JtJ[a * n + a]);
        for (int a = 0; a < n; ++a) {
          A[a * n + a] = A[a * n + a] * (1.0 + lam) + lam * 1e-14 * dmax;
          d[a] = -g[a];
        }
        if (!solve_dense(n, A, d)) { lam *= 10; continue; }
        std::vector<double> tn(th);
        for (int a = 0; a < n; ++a) tn[a] += d[a];
        double c1 = cost(tn);
        if (std::isfinite(c1) && c1 < c0) {
          double rel = (c0 - c1) / c0;
          th = tn;
          c0 = c1;
          lam = std::max(lam * 0.3, 1e-12);
          improved = true;
          if (rel < 1e-13) it = 1 << 20;
          break;
        }
        lam *= 10;
      }
      if (!improved) break;
    }
    ExpSum q = from_theta(k, th.data());
    extrema(q, R, pts, vals);
    if ((int)pts.size() == 2 * k + 1) { best = q; have = true; }
  }
  s = best;
  return have;
}

// Absolute rounding noise of err_at near t = 1, where 1/t and the exponential
// sum are both of order one: the equioscillation test cannot be sharper.
constexpr double kErrNoise = 1e-14;

// Remez exchange: solve e(x_i) = sgn_i E at the alternation points by damped
// Newton in (log omega, log alpha, E), then move the points to the extrema.
// Converged once the extremal errors agree to 1e-9 relative or to the noise.
bool remez(int k, double R, ExpSum& s, double& E_out) {
  const int n = 2 * k + 1;
  std::vector<double> pts, vals;
  double prev_spread = 1e300;
  for (int outer = 0; outer < 100; ++outer) {
    extrema(s, R, pts, vals);
    // A start continued from a longer interval has lost the alternation at
    // t = R (the end value has the sign of the last interior extremum): R
    // joins the reference with the alternating sign, as in the classic
    // exchange, and the next iterate alternates there again.
    if ((int)pts.size() == n - 1 && pts.back() < R) {
      pts.push_back(R);
      vals.push_back(err_at(s, R));
    }
    if ((int)pts.size() != n) return false;
    double emax = 0, emin = 1e300;
    for (double v : vals) { emax = std::max(emax, std::fabs(v)); emin = std::min(emin, std::fabs(v)); }
    const double spread = emax - emin;
    if (spread <= std::max(1e-12 * emax, kErrNoise)) { E_out = vals[0]; return true; }
    // no longer improving at a level the final test accepts: rounding in
    // the extrema limits any further progress
    if (spread <= std::max(1e-9 * emax, kErrNoise) && spread > 0.5 * prev_spread) {
      E_out = vals[0];
      return true;
    }
    prev_spread = spread;
    std::vector<double> sg(n);
    for (int i = 0; i < n; ++i) sg[i] = ((vals[0] < 0) ? -1.0 : 1.0) * ((i & 1) ? -1.0 : 1.0);
    std::vector<double> th(n);
    for (int i = 0; i < k; ++i) { th[i] = std::log(s.om[i]); th[k + i] = std::log(s.al[i]); }
    double sum = 0;
    for (double v : vals) sum += std::fabs(v);
    th[2 * k] = sum / n;
    auto resid = [&](const std::vector<double>& t, std::vector<double>& F) {
      ExpSum q = from_theta(k, t.data());
      double nrm = 0;
      for (int i = 0; i < n; ++i) {
        F[i] = (err_at(q, pts[i]) - sg[i] * t[2 * k]) / emax;
        nrm += F[i] * F[i];
      }
      return nrm;
    };
    std::vector<double> F(n), Fn(n);
    double f0 = resid(th, F);
    for (int it = 0; it < 60 && f0 > 1e-30; ++it) {
      ExpSum q = from_theta(k, th.data());
      std::vector<double> J((size_t)n * n), d(n);
      for (int i = 0; i < n; ++i) {
        for (int j = 0; j < k; ++j) {
          double ex = std::exp(-q.al[j] * pts[i]);
          J[i * n + j] = -q.om[j] * ex / emax;
          J[i * n + k + j] = q.om[j] * q.al[j] * pts[i] * ex / emax;
        }
        J[i * n + 2 * k] = -sg[i] / emax;
        d[i] = -F[i];
      }
      if (!solve_dense(n, J, d)) return false;
      double step = 1.0;
      bool ok = false;
      for (int h = 0; h < 40; ++h, step *= 0.5) {
        std::vector<double> tn(th);
        for (int a = 0; a < n; ++a) tn[a] += step * d[a];
        double f1 = resid(tn, Fn);
        if (std::isfinite(f1) && f1 < f0) { th = tn; F = Fn; f0 = f1; ok = true; break; }
      }
      if (!ok) break;
    }
    s = from_theta(k, th.data());
  }
  extrema(s, R, pts, vals);
  if ((int)pts.size() != n) return false;
  double emax = 0, emin = 1e300;
  for (double v : vals) { emax = std::max(emax, std::fabs(v)); emin = std::min(emin, std::fabs(v)); }
  E_out = vals[0];
  return emax - emin <= std::max(1e-9 * emax, kErrNoise);
}

// Converged minimax solutions of 1/t on [1, R] for a grid of (k, log10 R),
// generated by make_minimax_table.py with this file's own solver.
struct MinimaxEntry {
  int k;
  double log10R;
  double log_alpha[kMaxLt];
  double log_omega[kMaxLt];
};
#include "minimax_table.inc"

// Table-seeded solve: start from the nearest table entry with the same k and
// continue in log R to the target with the Remez exchange, halving a step
// that fails (the same continuation that generated the table).
bool remez_continue(int k, double lr0, const ExpSum& s0, double lr1, ExpSum& out, double& E,
                    int depth) {
  ExpSum s = s0;
  if (remez(k, std::pow(10.0, lr1), s, E)) { out = s; return true; }
  if (depth >= 5) return false;
  const double mid = 0.5 * (lr0 + lr1);
  ExpSum half;
  double Eh = 0;
  if (!remez_continue(k, lr0, s0, mid, half, Eh, depth + 1)) return false;
  return remez_continue(k, mid, half, lr1, out, E, depth + 1);
}

// k-term start from a (k-1)-term solution: log(alpha) and the density
// log(omega / (alpha dlog(alpha)/di)) interpolated linearly in the index and
// resampled on k points over the same range.
ExpSum stretch(const ExpSum& p, int k) {
  const int m = p.k;
  std::vector<int> ord(m);
  for (int i = 0; i < m; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return p.al[a] < p.al[b]; });
  std::vector<double> la(m), lq(m);
  for (int i = 0; i < m; ++i) la[i] = std::log(p.al[ord[i]]);
  for (int i = 0; i < m; ++i) {
    const double d = i == 0 ? la[1] - la[0]
                   : i == m - 1 ? la[m - 1] - la[m - 2] : 0.5 * (la[i + 1] - la[i - 1]);
    lq[i] = std::log(p.om[ord[i]]) - la[i] - std::log(d);
  }
  ExpSum s;
  s.k = k;
  for (int j = 0; j < k; ++j) {
    const double ip = double(j) * (m - 1) / (k - 1);
    const int i0 = std::min(int(ip), m - 2);
    const double f = ip - i0;
    const double lA = la[i0] * (1 - f) + la[i0 + 1] * f;
    const double lQ = lq[i0] * (1 - f) + lq[i0 + 1] * f;
    const double d = (la[i0 + 1] - la[i0]) * double(m - 1) / (k - 1);
    s.al[j] = std::exp(lA);
    s.om[j] = std::exp(lQ + lA) * d;
  }
  return s;
}

std::vector<double> sample_points(double R) {
  std::vector<double> xs(3000);
  for (int i = 0; i < 3000; ++i) xs[i] = std::exp(std::log(R) * i / 2999.0);
  return xs;
}

bool table_solve(int k, double R, ExpSum& s, double& E) {
  const double lr = std::log10(R);
  const MinimaxEntry* best = nullptr;
  for (const MinimaxEntry& e : kMinimaxTable) {
    if (e.k != k) continue;
    if (!best || std::fabs(e.log10R - lr) < std::fabs(best->log10R - lr)) best = &e;
  }
  if (!best) return false;
  ExpSum s0;
  s0.k = k;
  for (int i = 0; i < k; ++i) {
    s0.al[i] = std::exp(best->log_alpha[i]);
    s0.om[i] = std::exp(best->log_omega[i]);
  }
  return remez_continue(k, best->log10R, s0, lr, s, E, 0);
}

// Unseeded solve: the table; else the (k-1)-term solution stretched to k
// terms, refined in L_p and finished by the Remez exchange; else from a
// trapezoid start.
bool unseeded_solve(int k, double R, ExpSum& s, double& E) {
  if (table_solve(k, R, s, E)) return true;
  const std::vector<double> xs = sample_points(R);
  ExpSum prev;
  double Ep = 0;
  if (k >= 3 && unseeded_solve(k - 1, R, prev, Ep)) {
    s = stretch(prev, k);
    if (lp_refine(k, R, xs, s) && remez(k, R, s, E)) return true;
  }
  s = initial_guess(k, R, xs);
  return lp_refine(k, R, xs, s) && remez(k, R, s, E);
}

}  // namespace

extern "C" {

gw_status gw_prepare(int n_occ, int n_fc, int n_virt, const double* eps,
                     double omega_min, double* eps_F, double* y_min,
                     double* y_max) {
  gw::clear_error(nullptr);
  if (!eps || !eps_F || !y_min || !y_max)
    return gw::fail(nullptr, GW_EINVAL, "gw_prepare: NULL argument");
  if (n_fc < 0 || n_occ <= n_fc || n_virt < 1)
    return gw::fail(nullptr, GW_EINVAL, "gw_prepare: need 0 <= n_fc < n_occ and n_virt >= 1");
  const double e_homo = eps[n_occ - 1], e_lumo = eps[n_occ];
  if (!(e_lumo > e_homo))
    return gw::fail(nullptr, GW_EINVAL, "gw_prepare: LUMO must lie above HOMO");
  *eps_F = 0.5 * (e_homo + e_lumo);
  const double gap = e_lumo - e_homo;
  *y_min = gap * gap + omega_min * omega_min;
  const double span = eps[n_occ + n_virt - 1] - eps[n_fc];
  *y_max = std::max(span * span, 1e4);
  return GW_OK;
}

gw_status gw_freq_grid_mgl(int n, double x0, double* omega, double* weight) {
  gw::clear_error(nullptr);
  if (n < 1 || n > 4096 || !(x0 > 0) || !omega || !weight)
    return gw::fail(nullptr, GW_EINVAL, "gw_freq_grid_mgl: need 1 <= n <= 4096, x0 > 0");
  std::vector<double> t(n), v(n);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(pi * (i + 0.75) / (n + 0.5)), dp = 0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;                 // P_0, P_1
      for (int l = 2; l <= n; ++l) {
        double p2 = ((2.0 * l - 1.0) * z * p1 - (l - 1.0) * p0) / l;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);  // P_n'
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int l = 2; l <= n; ++l) {
      double p2 = ((2.0 * l - 1.0) * z * p1 - (l - 1.0) * p0) / l;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    double wgt = 2.0 / ((1.0 - z * z) * dp * dp);
    t[i] = -z;  v[i] = wgt;               // ascending t
    t[n - 1 - i] = z;  v[n - 1 - i] = wgt;
  }
  if (n % 2 == 1) t[n / 2] = 0.0;
  for (int i = 0; i < n; ++i) {
    omega[i] = x0 * (1.0 + t[i]) / (1.0 - t[i]);
    weight[i] = v[i] * 2.0 * x0 / ((1.0 - t[i]) * (1.0 - t[i]));
  }
  return GW_OK;
}

// Minimax of 1/t on [1, R]: seeded Remez when a start is given (L_p
// refinement first if the start does not alternate yet); otherwise a start
// continued in log R from the table of converged solutions, then the
// (k-1)-term solution stretched to k terms, then the from-scratch route
// (trapezoid start, L_p refinement, Remez).
gw_status gw_minimax_inverse(int n_lt, double R, const double* alpha0,
                             const double* omega0, double* alpha, double* omega,
                             double* err) {
  gw::clear_error(nullptr);
  if (n_lt < 1 || n_lt > kMaxLt || !(R > 1.0) || !alpha || !omega)
    return gw::fail(nullptr, GW_EINVAL, "gw_minimax_inverse: need 1 <= n_lt <= %d, R > 1", kMaxLt);
  ExpSum s;
  double E = 0;
  bool ok = false;
  if (alpha0 && omega0) {
    s.k = n_lt;
    for (int i = 0; i < n_lt; ++i) { s.al[i] = alpha0[i]; s.om[i] = omega0[i]; }
    ok = remez(n_lt, R, s, E);
    if (!ok) {
      // the start does not alternate 2k+1 times on this interval: refine it
      // in L_p first (from p = 32: it is a near-minimax start already)
      s.k = n_lt;
      for (int i = 0; i < n_lt; ++i) { s.al[i] = alpha0[i]; s.om[i] = omega0[i]; }
      const std::vector<double> xs = sample_points(R);
      ok = lp_refine(n_lt, R, xs, s, 32) && remez(n_lt, R, s, E);
    }
  } else {
    ok = unseeded_solve(n_lt, R, s, E);
  }
  if (!ok) return gw::fail(nullptr, GW_ENOCONV, "gw_minimax_inverse: Remez exchange failed");
  std::vector<int> ord(n_lt);
  for (int i = 0; i < n_lt; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return s.al[a] < s.al[b]; });
  for (int i = 0; i < n_lt; ++i) {
    alpha[i] = s.al[ord[i]];
    omega[i] = s.om[ord[i]];
  }
  if (err) *err = std::fabs(E);
  return GW_OK;
}

gw_status gw_lt_grid_minimax(int n_lt, double y_min, double y_max, double* x,
                             double* w, double* err_norm) {
  gw::clear_error(nullptr);
  if (n_lt < 1 || n_lt > kMaxLt || !(y_min > 0) || !(y_max > y_min) || !x || !w)
    return gw::fail(nullptr, GW_EINVAL,
                    "gw_lt_grid_minimax: need 1 <= n_lt <= %d and 0 < y_min < y_max", kMaxLt);
  double al[kMaxLt], om[kMaxLt];
  gw_status st = gw_minimax_inverse(n_lt, y_max / y_min, nullptr, nullptr, al, om, err_norm);
  if (st != GW_OK) return st;
  for (int i = 0; i < n_lt; ++i) {
    x[i] = al[i] / y_min;
    w[i] = om[i] / y_min;
  }
  return GW_OK;
}

gw_status gw_lt_grid_auto(double eps_lt, int max_lt, double y_min, double y_max, int* n_lt,
                          double* x, double* w, double* err_norm) {
  gw::clear_error(nullptr);
  if (!(eps_lt > 0) || max_lt < 1 || max_lt > kMaxLt || !n_lt || !x || !w)
    return gw::fail(nullptr, GW_EINVAL, "gw_lt_grid_auto: need eps_lt > 0, 1 <= max_lt <= %d",
                    kMaxLt);
  double err = 0;
  for (int k = 1; k <= max_lt; ++k) {
    const gw_status st = gw_lt_grid_minimax(k, y_min, y_max, x, w, &err);
    if (st != GW_OK) return st;
    if (err <= eps_lt) {
      *n_lt = k;
      if (err_norm) *err_norm = err;
      return GW_OK;
    }
  }
  if (err_norm) *err_norm = err;
  return gw::fail(nullptr, GW_ENOCONV,
                  "gw_lt_grid_auto: %d points leave a minimax error of %.3g > %.3g", max_lt, err,
                  eps_lt);
}

}  // extern "C"
