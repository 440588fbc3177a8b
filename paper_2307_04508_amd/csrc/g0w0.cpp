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

}  // namespace

extern "C" gw_status gw_g0w0(gw_ctx ctx, gw_precision prec, const gw_params* P,
                             const double* eps, const int* qp, const double* static_n,
                             const void* R_oo, const void* R_ov, const void* R_qp,
                             double* eps_qp, double* z_factor, int* status,
                             double* sigma_iw, gw_stats* stats) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_g0w0: ctx is NULL");
  gw::clear_error(ctx);
  if (ctx->capturing)
    return gw::fail(ctx, GW_EUNSUPPORTED, "gw_g0w0 synchronises and cannot be captured");
  GW_REQUIRE(ctx, P && eps && qp && R_oo && R_ov && R_qp && eps_qp && status,
             "gw_g0w0: NULL argument");
  const int o = P->n_occ - P->n_fc, v = P->n_virt, Mo = o + v, A = P->n_aux;
  GW_REQUIRE(ctx, o >= 1 && v >= 1 && A >= 1 && P->n_qp >= 1 && P->n_lt >= 1 &&
                      P->n_freq >= 1 && P->n_pade >= 1,
             "gw_g0w0: bad sizes");
  for (int q = 0; q < P->n_qp; ++q)
    GW_REQUIRE(ctx, qp[q] >= P->n_fc && qp[q] < P->n_occ + P->n_virt,
               "gw_g0w0: QP state %d (orbital %d) is not active", q, qp[q]);
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
  std::vector<double> xl(P->n_lt), wl(P->n_lt);
  double lt_err = 0;
  std::string lt_msg;
  auto lt_job = std::async(std::launch::async, [&]() {
    gw_status s = gw_lt_grid_minimax(P->n_lt, ymin, ymax, xl.data(), wl.data(), &lt_err);
    if (s != GW_OK) lt_msg = gw_last_error(nullptr);
    return s;
  });

  // a2: NAF
  const size_t esz = prec == GW_FP64 ? sizeof(double) : sizeof(float);
  double* K = static_cast<double*>(gw::ws_get(ctx, WS_G_K, (size_t)A * A * sizeof(double)));
  double* U = static_cast<double*>(gw::ws_get(ctx, WS_G_U, (size_t)A * A * sizeof(double)));
  if (!K || !U) return GW_ENOMEM;
  int N = 0;
  int64_t ldN = 0;   // NAF-space rows padded to whole 128-column tiles
  void* Rt_ov = nullptr;
  void* Rt_qp = nullptr;
  st = gw_naf_compress(ctx, prec, A, (int64_t)o * o, R_oo, (int64_t)o * v, R_ov, K, 0, 1,
                       P->eps_naf, P->max_keep, &N, U, nullptr);
  if (st == GW_OK && N < 1)
    st = gw::fail(ctx, GW_EINVAL, "gw_g0w0: no auxiliary function above eps_naf");
  if (st == GW_OK) {
    ldN = ((int64_t)N + 127) / 128 * 128;
    Rt_ov = gw::ws_get(ctx, WS_G_RT_OV, (size_t)o * v * ldN * esz);
    Rt_qp = gw::ws_get(ctx, WS_G_RT_QP, (size_t)P->n_qp * Mo * ldN * esz);
    if (!Rt_ov || !Rt_qp) st = GW_ENOMEM;
  }
  if (st == GW_OK) st = gw_naf_apply(ctx, prec, A, N, U, (int64_t)o * v, R_ov, Rt_ov, ldN);
  if (st == GW_OK)
    st = gw_naf_apply(ctx, prec, A, N, U, (int64_t)P->n_qp * Mo, R_qp, Rt_qp, ldN);
  if (st != GW_OK) {
    lt_job.wait();
    return st;
  }
  ev.rec(1, ctx->stream);

  st = lt_job.get();
  if (st != GW_OK) return gw::fail(ctx, st, "gw_g0w0: %s", lt_msg.c_str());

  // a4: chi
  double* Mm = static_cast<double*>(gw::ws_get(ctx, WS_G_M, (size_t)P->n_lt * N * N * sizeof(double)));
  if (!Mm) return GW_ENOMEM;
  GW_TRY(gw_polarizability_lt(ctx, prec, N, P->n_lt, xl.data(), wl.data(), o, v, eps + P->n_fc,
                              eps + P->n_occ, Rt_ov, ldN, 0, 1, Mm));
  ev.rec(2, ctx->stream);

  // a5-a8 in frequency batches
  const int fb = P->freq_batch > 0 ? std::min(P->freq_batch, P->n_freq) : P->n_freq;
  void* What = gw::ws_get(ctx, WS_G_WHAT, (size_t)fb * N * N * esz);
  double* sig = static_cast<double*>(
      gw::ws_get(ctx, WS_G_SIGMA, (size_t)2 * P->n_qp * P->n_pade * sizeof(double)));
  if (!What || !sig) return GW_ENOMEM;
  double t_screen = 0, t_sigma = 0;
  for (int j0 = 0; j0 < P->n_freq; j0 += fb) {
    const int nb = std::min(fb, P->n_freq - j0);
    ev.rec(3, ctx->stream);
    GW_TRY(gw_screen(ctx, prec, N, P->n_lt, xl.data(), Mm, nb, om.data() + j0, What));
    ev.rec(4, ctx->stream);
    GW_TRY(gw_sigma_diag(ctx, prec, N, P->n_qp, Mo, eps + P->n_fc, eF, Rt_qp, ldN, nb,
                         om.data() + j0,
                         wom.data() + j0, What, P->n_pade, omp.data(), j0 > 0, sig, nullptr));
    ev.rec(5, ctx->stream);
    if (stats) {
      GW_HIP(ctx, hipStreamSynchronize(ctx->stream));
      t_screen += ev.ms(3, 4);
      t_sigma += ev.ms(4, 5);
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
  if (stats) {
    stats->n_naf = N;
    stats->lt_err_norm = lt_err;
    stats->t_naf_ms = ev.ms(0, 1);
    stats->t_chi_ms = ev.ms(1, 2);
    stats->t_screen_ms = t_screen;
    stats->t_sigma_ms = t_sigma;
    stats->t_qp_ms = ev.ms(5, 6);
    stats->t_total_ms = ev.ms(0, 6);
  }
  return GW_OK;
}
