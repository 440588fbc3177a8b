// One LT-AC G0W0 evaluation through the public entry points, in the paper's
// order: frozen core and bounds (Sec. 3), NAF (Eqs. 11-13), grids (Sec. 2,
// Sec. 3), LT polarizability (Eq. 10), screening (Eq. 2), self-energy
// (Eqs. 2, 7), Pade and QP (Sec. 2).  Intermediates live in the context's
// workspace; only the QP results (and optionally Sigma) return to the host.
#include <algorithm>
#include <future>
#include <vector>

#include "common.hpp"

namespace {

struct Events {
  hipEvent_t e[7] = {};
  bool ok = false;
  explicit Events(bool on) {
    if (!on) return;
    ok = true;
    for (auto& x : e)
      if (hipEventCreate(&x) != hipSuccess) ok = false;
  }
  ~Events() {
    for (auto& x : e)
      if (x) hipEventDestroy(x);
  }
  void rec(int i, hipStream_t s) {
    if (ok) hipEventRecord(e[i], s);
  }
  double ms(int a, int b) const {
    float t = 0.f;
    if (!ok || hipEventElapsedTime(&t, e[a], e[b]) != hipSuccess) return 0.0;
    return t;
  }
};

// The work after the NAF stage for one set of orbital energies: Laplace
// polarizability (Eq. 10), screening (Eq. 2), self-energy (Eqs. 2, 7), Pade
// and QP (Sec. 2).  eps: energies entering this evaluation (Delta in Pi, the
// poles of G, the Fermi level); the QP equation solved is
// E = eps[qp] + static + Re Sigma(E).  Times (ms) accumulate into t[0..3]
// (chi, screen, sigma, qp) when ev is on.
gw_status post_naf(gw_ctx ctx, gw_precision prec, const gw_params* P, const double* eps,
                   const int* qp, const double* static_n, const std::vector<double>& xl,
                   const std::vector<double>& wl, const std::vector<double>& om,
                   const std::vector<double>& wom, const std::vector<double>& omp, double eF,
                   int N, int64_t ldN, const void* Rt_ov, const void* Rt_qp, double* eps_qp,
                   double* z_factor, int* status, double* sigma_iw, Events& ev, double* t) {
  const int o = P->n_occ - P->n_fc, v = P->n_virt, Mo = o + v;
  const size_t esz = prec == GW_FP64 ? sizeof(double) : sizeof(float);
  ev.rec(1, ctx->stream);
  // a4: chi (Laplace matrices M^m, or without the Laplace transform the
  // sums P_j at every frequency)
  const int nm = P->no_lt ? P->n_freq : P->n_lt;
  double* Mm = static_cast<double*>(gw::ws_get(ctx, WS_G_M, (size_t)nm * N * N * sizeof(double)));
  if (!Mm) return GW_ENOMEM;
  if (P->no_lt)
    GW_TRY(gw_polarizability_sos(ctx, prec, N, P->n_freq, om.data(), o, v, eps + P->n_fc,
                                 eps + P->n_occ, Rt_ov, ldN, 0, 1, Mm));
  else
    GW_TRY(gw_polarizability_lt(ctx, prec, N, P->n_lt, xl.data(), wl.data(), o, v, eps + P->n_fc,
                                eps + P->n_occ, Rt_ov, ldN, 0, 1, Mm));
  ev.rec(2, ctx->stream);
  if (ev.ok) {
    GW_HIP(ctx, hipStreamSynchronize(ctx->stream));
    t[0] += ev.ms(1, 2);
  }

  // a5-a8 in frequency batches
  const int fb = P->freq_batch > 0 ? std::min(P->freq_batch, P->n_freq) : P->n_freq;
  void* What = gw::ws_get(ctx, WS_G_WHAT, (size_t)fb * N * N * esz);
  double* sig = static_cast<double*>(
      gw::ws_get(ctx, WS_G_SIGMA, (size_t)2 * P->n_qp * P->n_pade * sizeof(double)));
  if (!What || !sig) return GW_ENOMEM;
  for (int j0 = 0; j0 < P->n_freq; j0 += fb) {
    const int nb = std::min(fb, P->n_freq - j0);
    ev.rec(3, ctx->stream);
    if (P->no_lt)
      GW_TRY(gw_screen_sos(ctx, prec, N, nb, Mm + (size_t)j0 * N * N, What));
    else
      GW_TRY(gw_screen(ctx, prec, N, P->n_lt, xl.data(), Mm, nb, om.data() + j0, What));
    ev.rec(4, ctx->stream);
    GW_TRY(gw_sigma_diag(ctx, prec, N, P->n_qp, Mo, eps + P->n_fc, eF, Rt_qp, ldN, nb,
                         om.data() + j0,
                         wom.data() + j0, What, P->n_pade, omp.data(), j0 > 0, sig, nullptr));
    ev.rec(5, ctx->stream);
    if (ev.ok) {
      GW_HIP(ctx, hipStreamSynchronize(ctx->stream));
      t[1] += ev.ms(3, 4);
      t[2] += ev.ms(4, 5);
    }
  }

  // a9
  std::vector<double> en(P->n_qp);
  for (int q = 0; q < P->n_qp; ++q) en[q] = eps[qp[q]];
  GW_TRY(gw_qp_solve(ctx, P->n_qp, en.data(), static_n, eF, P->n_pade, omp.data(), sig, P->eta,
                     P->tol, P->max_iter, eps_qp, z_factor, status));
  ev.rec(6, ctx->stream);
  if (sigma_iw)
    GW_HIP(ctx, hipMemcpyAsync(sigma_iw, sig, (size_t)2 * P->n_qp * P->n_pade * sizeof(double),
                               hipMemcpyDeviceToHost, ctx->stream));
  GW_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (ev.ok) t[3] += ev.ms(5, 6);
  return GW_OK;
}

gw_status check_args(gw_ctx ctx, const char* who, const gw_params* P, const double* eps,
                     const int* qp, const void* R_oo, const void* R_ov, const void* R_qp,
                     const void* out, const int* status) {
  if (ctx->capturing)
    return gw::fail(ctx, GW_EUNSUPPORTED, "%s synchronises and cannot be captured", who);
  GW_REQUIRE(ctx, P && eps && qp && R_oo && R_ov && R_qp && out && status,
             "%s: NULL argument", who);
  const int o = P->n_occ - P->n_fc;
  GW_REQUIRE(ctx, o >= 1 && P->n_virt >= 1 && P->n_aux >= 1 && P->n_qp >= 1 &&
                      (P->n_lt >= 1 || P->eps_lt > 0) && P->n_freq >= 1 && P->n_pade >= 1,
             "%s: bad sizes", who);
  GW_REQUIRE(ctx, P->eps_lt >= 0, "%s: eps_lt = %g < 0", who, P->eps_lt);
  for (int q = 0; q < P->n_qp; ++q)
    GW_REQUIRE(ctx, qp[q] >= P->n_fc && qp[q] < P->n_occ + P->n_virt,
               "%s: QP state %d (orbital %d) is not active", who, q, qp[q]);
  return GW_OK;
}

// a3, Laplace grid on [ymin, ymax]: n_lt points, or with eps_lt > 0 the
// smallest grid meeting it (n_lt, at most 20, as the bound); P->n_lt of the
// copy Pg becomes the size taken.
gw_status laplace_grid(const gw_params* P, double ymin, double ymax, gw_params* Pg,
                       std::vector<double>& xl, std::vector<double>& wl, double* err) {
  *Pg = *P;
  if (P->eps_lt > 0) {
    const int max_lt = P->n_lt >= 1 && P->n_lt <= 20 ? P->n_lt : 20;
    xl.assign(max_lt, 0.0);
    wl.assign(max_lt, 0.0);
    int n = 0;
    GW_TRY(gw_lt_grid_auto(P->eps_lt, max_lt, ymin, ymax, &n, xl.data(), wl.data(), err));
    xl.resize(n);
    wl.resize(n);
    Pg->n_lt = n;
    return GW_OK;
  }
  xl.assign(P->n_lt, 0.0);
  wl.assign(P->n_lt, 0.0);
  return gw_lt_grid_minimax(P->n_lt, ymin, ymax, xl.data(), wl.data(), err);
}

// a2: NAF compression and transformation of the ov and QP rows.
gw_status naf_stage(gw_ctx ctx, gw_precision prec, const gw_params* P, const void* R_oo,
                    const void* R_ov, const void* R_qp, int* N_out, int64_t* ldN_out,
                    void** Rt_ov, void** Rt_qp) {
  const int o = P->n_occ - P->n_fc, v = P->n_virt, Mo = o + v, A = P->n_aux;
  const size_t esz = prec == GW_FP64 ? sizeof(double) : sizeof(float);
  double* K = static_cast<double*>(gw::ws_get(ctx, WS_G_K, (size_t)A * A * sizeof(double)));
  double* U = static_cast<double*>(gw::ws_get(ctx, WS_G_U, (size_t)A * A * sizeof(double)));
  if (!K || !U) return GW_ENOMEM;
  int N = 0;
  GW_TRY(gw_naf_compress(ctx, prec, A, (int64_t)o * o, R_oo, (int64_t)o * v, R_ov, K, 0, 1,
                         P->eps_naf, P->max_keep, &N, U, nullptr));
  if (N < 1) return gw::fail(ctx, GW_EINVAL, "no auxiliary function above eps_naf");
  const int64_t ldN = ((int64_t)N + 127) / 128 * 128;   // whole 128-column tiles
  *Rt_ov = gw::ws_get(ctx, WS_G_RT_OV, (size_t)o * v * ldN * esz);
  *Rt_qp = gw::ws_get(ctx, WS_G_RT_QP, (size_t)P->n_qp * Mo * ldN * esz);
  if (!*Rt_ov || !*Rt_qp) return GW_ENOMEM;
  GW_TRY(gw_naf_apply(ctx, prec, A, N, U, (int64_t)o * v, R_ov, *Rt_ov, ldN));
  GW_TRY(gw_naf_apply(ctx, prec, A, N, U, (int64_t)P->n_qp * Mo, R_qp, *Rt_qp, ldN));
  *N_out = N;
  *ldN_out = ldN;
  return GW_OK;
}

}  // namespace

extern "C" gw_status gw_g0w0(gw_ctx ctx, gw_precision prec, const gw_params* P,
                             const double* eps, const int* qp, const double* static_n,
                             const void* R_oo, const void* R_ov, const void* R_qp,
                             double* eps_qp, double* z_factor, int* status,
                             double* sigma_iw, gw_stats* stats) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_g0w0: ctx is NULL");
  gw::clear_error(ctx);
  GW_TRY(check_args(ctx, "gw_g0w0", P, eps, qp, R_oo, R_ov, R_qp, eps_qp, status));
  GW_HIP(ctx, hipSetDevice(ctx->device));
  Events ev(stats != nullptr);
  ev.rec(0, ctx->stream);

  // a3 (frequencies) and a1
  std::vector<double> om(P->n_freq), wom(P->n_freq), omp(P->n_pade), womp(P->n_pade);
  gw_status st = gw_freq_grid_mgl(P->n_freq, P->x0, om.data(), wom.data());
  if (st == GW_OK) st = gw_freq_grid_mgl(P->n_pade, P->x0, omp.data(), womp.data());
  if (st != GW_OK) return gw::fail(ctx, st, "gw_g0w0: %s", gw_last_error(nullptr));
  double eF = 0, ymin = 0, ymax = 0;
  st = gw_prepare(P->n_occ, P->n_fc, P->n_virt, eps, om[0], &eF, &ymin, &ymax);
  if (st != GW_OK) return gw::fail(ctx, st, "gw_g0w0: %s", gw_last_error(nullptr));

  // a3 (Laplace grid): host work, overlapped with the NAF stage on the device
  std::vector<double> xl, wl;
  double lt_err = 0;
  std::string lt_msg;
  gw_params Pg = *P;
  auto lt_job = std::async(std::launch::async, [&]() {
    if (P->no_lt) return GW_OK;
    gw_status s = laplace_grid(P, ymin, ymax, &Pg, xl, wl, &lt_err);
    if (s != GW_OK) lt_msg = gw_last_error(nullptr);
    return s;
  });

  // a2: NAF
  int N = 0;
  int64_t ldN = 0;
  void* Rt_ov = nullptr;
  void* Rt_qp = nullptr;
  st = naf_stage(ctx, prec, P, R_oo, R_ov, R_qp, &N, &ldN, &Rt_ov, &Rt_qp);
  lt_job.wait();
  if (st != GW_OK) return st;
  st = lt_job.get();
  if (st != GW_OK) return gw::fail(ctx, st, "gw_g0w0: %s", lt_msg.c_str());

  double t[4] = {0, 0, 0, 0};
  GW_TRY(post_naf(ctx, prec, &Pg, eps, qp, static_n, xl, wl, om, wom, omp, eF, N, ldN, Rt_ov,
                  Rt_qp, eps_qp, z_factor, status, sigma_iw, ev, t));
  if (stats) {
    stats->n_naf = N;
    stats->n_lt = P->no_lt ? 0 : Pg.n_lt;
    stats->lt_err_norm = lt_err;
    stats->t_naf_ms = ev.ms(0, 1);
    stats->t_chi_ms = t[0];
    stats->t_screen_ms = t[1];
    stats->t_sigma_ms = t[2];
    stats->t_qp_ms = t[3];
    stats->t_total_ms = ev.ms(0, 6);
  }
  return GW_OK;
}

extern "C" gw_status gw_evgw(gw_ctx ctx, gw_precision prec, const gw_params* P, int n_cycles,
                             const double* eps, const int* qp, const double* static_n,
                             const void* R_oo, const void* R_ov, const void* R_qp,
                             double* eps_qp, double* z_factor, int* status, double* eps_last,
                             gw_stats* stats) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_evgw: ctx is NULL");
  gw::clear_error(ctx);
  GW_TRY(check_args(ctx, "gw_evgw", P, eps, qp, R_oo, R_ov, R_qp, eps_qp, status));
  GW_REQUIRE(ctx, n_cycles >= 1, "gw_evgw: n_cycles = %d", n_cycles);
  GW_HIP(ctx, hipSetDevice(ctx->device));
  Events ev(stats != nullptr);
  ev.rec(0, ctx->stream);
  const int n_orb = P->n_occ + P->n_virt, Q = P->n_qp;
  std::vector<double> om(P->n_freq), wom(P->n_freq), omp(P->n_pade), womp(P->n_pade);
  gw_status st = gw_freq_grid_mgl(P->n_freq, P->x0, om.data(), wom.data());
  if (st == GW_OK) st = gw_freq_grid_mgl(P->n_pade, P->x0, omp.data(), womp.data());
  if (st != GW_OK) return gw::fail(ctx, st, "gw_evgw: %s", gw_last_error(nullptr));

  // a2 once: the natural auxiliary functions do not depend on the energies
  int N = 0;
  int64_t ldN = 0;
  void* Rt_ov = nullptr;
  void* Rt_qp = nullptr;
  GW_TRY(naf_stage(ctx, prec, P, R_oo, R_ov, R_qp, &N, &ldN, &Rt_ov, &Rt_qp));
  double t_naf = 0;
  ev.rec(1, ctx->stream);
  if (ev.ok) {
    GW_HIP(ctx, hipStreamSynchronize(ctx->stream));
    t_naf = ev.ms(0, 1);
  }

  // lowest and highest QP states: their corrections shift the other orbitals
  int lo = 0, hi = 0;
  std::vector<char> in_qp(n_orb, 0);
  for (int q = 0; q < Q; ++q) {
    in_qp[qp[q]] = 1;
    if (qp[q] < qp[lo]) lo = q;
    if (qp[q] > qp[hi]) hi = q;
  }
  std::vector<double> cur(eps, eps + n_orb), stat(Q), xl, wl;
  double t[4] = {0, 0, 0, 0}, lt_err = 0;
  int n_lt_last = 0;
  for (int c = 0; c < n_cycles; ++c) {
    double eF = 0, ymin = 0, ymax = 0;
    gw_params Pg = *P;
    st = gw_prepare(P->n_occ, P->n_fc, P->n_virt, cur.data(), om[0], &eF, &ymin, &ymax);
    if (st == GW_OK && !P->no_lt) st = laplace_grid(P, ymin, ymax, &Pg, xl, wl, &lt_err);
    if (st != GW_OK) return gw::fail(ctx, st, "gw_evgw: cycle %d: %s", c, gw_last_error(nullptr));
    n_lt_last = P->no_lt ? 0 : Pg.n_lt;
    // QP equation based on the starting energies: E = eps0 + c + Re Sigma[cur](E)
    for (int q = 0; q < Q; ++q)
      stat[q] = eps[qp[q]] + (static_n ? static_n[q] : 0.0) - cur[qp[q]];
    double* E = eps_qp + (size_t)c * Q;
    int* S = status + (size_t)c * Q;
    GW_TRY(post_naf(ctx, prec, &Pg, cur.data(), qp, stat.data(), xl, wl, om, wom, omp, eF, N, ldN,
                    Rt_ov, Rt_qp, E, c + 1 == n_cycles ? z_factor : nullptr, S, nullptr, ev, t));
    // energies of the next cycle (Sec. 3): QP states take their QP energies;
    // other active occupied orbitals the shift of the lowest QP state, other
    // virtual ones that of the highest
    const double d_lo = E[lo] - eps[qp[lo]], d_hi = E[hi] - eps[qp[hi]];
    for (int m = P->n_fc; m < n_orb; ++m)
      if (!in_qp[m]) cur[m] = eps[m] + (m < P->n_occ ? d_lo : d_hi);
    for (int q = 0; q < Q; ++q) cur[qp[q]] = E[q];
  }
  if (eps_last) std::copy(cur.begin(), cur.end(), eps_last);
  if (stats) {
    stats->n_naf = N;
    stats->n_lt = n_lt_last;
    stats->lt_err_norm = lt_err;
    stats->t_naf_ms = t_naf;
    stats->t_chi_ms = t[0];
    stats->t_screen_ms = t[1];
    stats->t_sigma_ms = t[2];
    stats->t_qp_ms = t[3];
    stats->t_total_ms = ev.ms(0, 6);
  }
  return GW_OK;
}
