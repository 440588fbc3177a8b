// Many molecules of uneven size through the whole hot path in shared
// launches.  The NAF stage (Eqs. 11-13) runs eagerly because the kept counts
// decide every later size; the rest (Eq. 10, Eq. 2, Eq. 7, Pade and QP) is a
// fixed sequence of batched launches that can be captured once into a HIP
// graph and replayed while the sizes, the NAF counts and the host inputs
// stay the same.
#include <algorithm>
#include <cstring>
#include <future>
#include <string>
#include <vector>

#include "common.hpp"

struct BatchGraph {
  hipGraphExec_t exec = nullptr;
  void* arena = nullptr;
  std::vector<uint64_t> key;
};

namespace gw {

void drop_batch_graph(gw_ctx ctx) {
  if (!ctx->batch_graph) return;
  hipStreamSynchronize(ctx->stream);
  if (ctx->batch_graph->exec) hipGraphExecDestroy(ctx->batch_graph->exec);
  if (ctx->batch_graph->arena) hipFree(ctx->batch_graph->arena);
  delete ctx->batch_graph;
  ctx->batch_graph = nullptr;
}

}  // namespace gw

namespace {

// FNV-1a over raw bytes: the graph cache key covers every host input the
// captured launches were given.
uint64_t fnv(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

template <typename T>
void key_add(std::vector<uint64_t>& k, const T& v) {
  uint64_t x = 0;
  std::memcpy(&x, &v, std::min(sizeof(T), sizeof(x)));
  k.push_back(x);
}

struct Mol {
  int o, v, A, Q, Mo, N;
  int64_t ldN;
  double eF, ymin, ymax;
  std::vector<double> x, w, eig, en;
  size_t u_off, rov_off, rqp_off, m_off, w_off, s_off, q_off;
};

struct Events {
  hipEvent_t e[3] = {};
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

extern "C" gw_status gw_g0w0_batched(gw_ctx ctx, gw_precision prec, const gw_batch_params* P,
                                     int n_mol, gw_mol* mols, int flags, gw_batch_stats* stats) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_g0w0_batched: ctx is NULL");
  gw::clear_error(ctx);
  if (ctx->capturing)
    return gw::fail(ctx, GW_EUNSUPPORTED, "gw_g0w0_batched synchronises and cannot be captured");
  GW_REQUIRE(ctx, prec == GW_FP64 || prec == GW_FP32 || prec == GW_BF16X3,
             "gw_g0w0_batched: unknown precision %d", (int)prec);
  GW_REQUIRE(ctx, P && mols && n_mol >= 1, "gw_g0w0_batched: NULL argument or no molecules");
  GW_REQUIRE(ctx, P->n_lt >= 1 && P->n_lt <= 20 && P->n_freq >= 1 && P->n_pade >= 1 &&
                      P->n_pade <= 256 && P->n_freq * P->n_lt <= 4096 && P->max_iter >= 1 &&
                      P->tol > 0 && P->x0 > 0,
             "gw_g0w0_batched: bad grid or QP parameters");
  for (int d = 0; d < n_mol; ++d) {
    const gw_mol& m = mols[d];
    GW_REQUIRE(ctx, m.n_occ - m.n_fc >= 1 && m.n_fc >= 0 && m.n_virt >= 1 && m.n_aux >= 1 &&
                        m.n_qp >= 1 && m.max_keep >= 0,
               "gw_g0w0_batched: molecule %d: bad sizes", d);
    GW_REQUIRE(ctx, m.eps && m.qp && m.R_oo && m.R_ov && m.R_qp && m.eps_qp && m.status,
               "gw_g0w0_batched: molecule %d: NULL argument", d);
    for (int q = 0; q < m.n_qp; ++q)
      GW_REQUIRE(ctx, m.qp[q] >= m.n_fc && m.qp[q] < m.n_occ + m.n_virt,
                 "gw_g0w0_batched: molecule %d: QP state %d (orbital %d) is not active", d, q,
                 m.qp[q]);
  }
  GW_HIP(ctx, hipSetDevice(ctx->device));
  Events ev(stats != nullptr);
  ev.rec(0, ctx->stream);
  const int n = n_mol, L = P->n_lt, F = P->n_freq, Pd = P->n_pade;

  // a3 frequencies (shared), a1 bounds per molecule
  std::vector<double> om(F), wom(F), omp(Pd), womp(Pd);
  gw_status st = gw_freq_grid_mgl(F, P->x0, om.data(), wom.data());
  if (st == GW_OK) st = gw_freq_grid_mgl(Pd, P->x0, omp.data(), womp.data());
  if (st != GW_OK) return gw::fail(ctx, st, "gw_g0w0_batched: %s", gw_last_error(nullptr));
  std::vector<Mol> mo(n);
  for (int d = 0; d < n; ++d) {
    const gw_mol& m = mols[d];
    Mol& g = mo[d];
    g.o = m.n_occ - m.n_fc;
    g.v = m.n_virt;
    g.A = m.n_aux;
    g.Q = m.n_qp;
    g.Mo = g.o + g.v;
    st = gw_prepare(m.n_occ, m.n_fc, m.n_virt, m.eps, om[0], &g.eF, &g.ymin, &g.ymax);
    if (st != GW_OK)
      return gw::fail(ctx, st, "gw_g0w0_batched: molecule %d: %s", d, gw_last_error(nullptr));
    g.x.resize(L);
    g.w.resize(L);
    g.eig.resize(g.A);
    g.en.resize(g.Q);
    for (int q = 0; q < g.Q; ++q) g.en[q] = m.eps[m.qp[q]];
  }
  // a3 Laplace grids on a host thread, overlapped with the NAF stage
  std::string lt_msg;
  auto lt_job = std::async(std::launch::async, [&]() {
    for (int d = 0; d < n; ++d) {
      gw_status s = gw_lt_grid_minimax(L, mo[d].ymin, mo[d].ymax, mo[d].x.data(), mo[d].w.data(),
                                       nullptr);
      if (s != GW_OK) {
        lt_msg = "molecule " + std::to_string(d) + ": " + gw_last_error(nullptr);
        return s;
      }
    }
    return GW_OK;
  });
  auto fail_after = [&](gw_status s) {
    lt_job.wait();
    return s;
  };

  // a2: NAF of every molecule
  const gw_precision mp = prec == GW_FP64 ? GW_FP64 : GW_FP32;
  const size_t esz = prec == GW_FP64 ? sizeof(double) : sizeof(float);
  size_t u_tot = 0;
  for (Mol& g : mo) {
    g.u_off = u_tot;
    u_tot += (size_t)g.A * g.A;
  }
  double* U = static_cast<double*>(gw::ws_get(ctx, WS_B_U, u_tot * sizeof(double)));
  if (!U) return fail_after(GW_ENOMEM);
  {
    std::vector<gw::SyrkJob> oo, ov;
    for (int d = 0; d < n; ++d) {
      const Mol& g = mo[d];
      double* K = U + g.u_off;   // the metric, replaced by the basis after the solve
      oo.push_back(gw::SyrkJob{mols[d].R_oo, (int64_t)g.o * g.o, g.A, g.A, 1, nullptr, 2.0, K, 0});
      ov.push_back(gw::SyrkJob{mols[d].R_ov, (int64_t)g.o * g.v, g.A, g.A, 1, nullptr, 4.0, K, 1});
    }
    st = gw::syrk_batched_launch(ctx, mp, oo, "naf_syrk");
    if (st == GW_OK) st = gw::syrk_batched_launch(ctx, mp, ov, "naf_syrk");
    if (st != GW_OK) return fail_after(st);
    std::vector<gw::NafEigJob> ej;
    for (int d = 0; d < n; ++d)
      ej.push_back(gw::NafEigJob{U + mo[d].u_off, mo[d].A, U + mo[d].u_off, mo[d].eig.data(),
                                 mols[d].eps_naf, mols[d].max_keep, false});
    st = gw::naf_eig_batched(ctx, ej);
    if (st != GW_OK) return fail_after(st);
  }
  size_t rov_tot = 0, rqp_tot = 0, m_tot = 0, w_tot = 0, s_tot = 0, q_tot = 0;
  for (int d = 0; d < n; ++d) {
    Mol& g = mo[d];
    int keep = 0;
    for (int p = 0; p < g.A; ++p) {
      if (g.eig[p] > mols[d].eps_naf) ++keep; else break;
    }
    if (mols[d].max_keep > 0) keep = std::min(keep, mols[d].max_keep);
    if (keep < 1)
      return fail_after(gw::fail(ctx, GW_EINVAL,
                                 "gw_g0w0_batched: molecule %d: no auxiliary function above eps_naf", d));
    g.N = keep;
    mols[d].n_naf = keep;
    g.ldN = ((int64_t)keep + 127) / 128 * 128;
    g.rov_off = rov_tot;
    rov_tot += (size_t)g.o * g.v * g.ldN;
    g.rqp_off = rqp_tot;
    rqp_tot += (size_t)g.Q * g.Mo * g.ldN;
    g.m_off = m_tot;
    m_tot += (size_t)L * g.N * g.N;
    g.w_off = w_tot;
    w_tot += (size_t)F * g.N * g.N;
    g.s_off = s_tot;
    s_tot += (size_t)2 * g.Q * Pd;
    g.q_off = q_tot;
    q_tot += (size_t)g.Q;
  }
  unsigned char* Rov = static_cast<unsigned char*>(gw::ws_get(ctx, WS_B_RT_OV, rov_tot * esz));
  unsigned char* Rqp = static_cast<unsigned char*>(gw::ws_get(ctx, WS_B_RT_QP, rqp_tot * esz));
  if (!Rov || !Rqp) return fail_after(GW_ENOMEM);
  {
    std::vector<gw::NafGemmJob> gj;
    for (int d = 0; d < n; ++d) {
      const Mol& g = mo[d];
      gj.push_back(gw::NafGemmJob{mols[d].R_ov, U + g.u_off, Rov + g.rov_off * esz,
                                  (int64_t)g.o * g.v, g.A, g.N, g.ldN});
      gj.push_back(gw::NafGemmJob{mols[d].R_qp, U + g.u_off, Rqp + g.rqp_off * esz,
                                  (int64_t)g.Q * g.Mo, g.A, g.N, g.ldN});
    }
    st = gw::naf_gemm_batched(ctx, prec, gj);
    if (st != GW_OK) return fail_after(st);
  }
  ev.rec(1, ctx->stream);
  st = lt_job.get();
  if (st != GW_OK) return gw::fail(ctx, st, "gw_g0w0_batched: %s", lt_msg.c_str());

  // a4-a9 buffers
  double* Mm = static_cast<double*>(gw::ws_get(ctx, WS_B_M, m_tot * sizeof(double)));
  unsigned char* What = static_cast<unsigned char*>(gw::ws_get(ctx, WS_B_WHAT, w_tot * esz));
  double* sig = static_cast<double*>(gw::ws_get(ctx, WS_B_SIGMA, (s_tot + 3 * q_tot) * sizeof(double)));
  if (!Mm || !What || !sig) return GW_ENOMEM;
  double* qout = sig + s_tot;

  // the host inputs of a4-a9 per molecule
  std::vector<std::vector<double>> eps_i(n), eps_a(n), eps_m(n), stat(n);
  for (int d = 0; d < n; ++d) {
    const gw_mol& m = mols[d];
    eps_i[d].assign(m.eps + m.n_fc, m.eps + m.n_occ);
    eps_a[d].assign(m.eps + m.n_occ, m.eps + m.n_occ + m.n_virt);
    eps_m[d].assign(m.eps + m.n_fc, m.eps + m.n_occ + m.n_virt);
    if (m.static_n) stat[d].assign(m.static_n, m.static_n + m.n_qp);
  }
  auto rest = [&]() -> gw_status {
    std::vector<gw_chi_job> cj;
    std::vector<gw_screen_job> sj;
    std::vector<gw_sigma_job> gj;
    for (int d = 0; d < n; ++d) {
      const Mol& g = mo[d];
      cj.push_back(gw_chi_job{g.N, g.o, g.v, g.x.data(), g.w.data(), eps_i[d].data(),
                              eps_a[d].data(), Rov + g.rov_off * esz, g.ldN, Mm + g.m_off});
      sj.push_back(gw_screen_job{g.N, g.x.data(), Mm + g.m_off, F, om.data(), What + g.w_off * esz});
      gj.push_back(gw_sigma_job{g.N, g.Q, g.Mo, eps_m[d].data(), g.eF, Rqp + g.rqp_off * esz, g.ldN,
                                F, om.data(), wom.data(), What + g.w_off * esz, Pd, omp.data(),
                                sig + g.s_off, nullptr});
    }
    GW_TRY(gw_polarizability_lt_batched(ctx, prec, L, n, cj.data(), 0, 0));
    GW_TRY(gw_screen_batched(ctx, prec, L, n, sj.data()));
    GW_TRY(gw_sigma_diag_batched(ctx, prec, n, gj.data(), 0));
    std::vector<gw::QpJob> qj;
    const double* d_op = gw::stage_t(ctx, omp.data(), Pd);
    if (!d_op) return GW_EINVAL;
    for (int d = 0; d < n; ++d) {
      const Mol& g = mo[d];
      const double* d_en = gw::stage_t(ctx, g.en.data(), g.Q);
      const double* d_st = stat[d].empty() ? nullptr : gw::stage_t(ctx, stat[d].data(), g.Q);
      if (!d_en || (!stat[d].empty() && !d_st)) return GW_EINVAL;
      qj.push_back(gw::QpJob{g.Q, Pd, d_op, sig + g.s_off, d_en, d_st, g.eF});
    }
    return gw::qp_batched_launch(ctx, qj, P->eta, P->tol, P->max_iter, qout);
  };

  // graph cache key: sizes, every host input of a4-a9 (hashed) and the
  // device buffers the launches read and write
  auto make_key = [&]() {
    std::vector<uint64_t> key;
    key_add(key, (int)prec);
    key_add(key, n);
    uint64_t h = 1469598103934665603ull;
    h = fnv(h, P, sizeof(*P));
    for (int d = 0; d < n; ++d) {
      const Mol& g = mo[d];
      const int dims[6] = {g.o, g.v, g.A, g.Q, g.N, (int)g.ldN};
      h = fnv(h, dims, sizeof dims);
      h = fnv(h, mols[d].eps, sizeof(double) * (mols[d].n_occ + mols[d].n_virt));
      h = fnv(h, g.x.data(), sizeof(double) * L);
      h = fnv(h, g.w.data(), sizeof(double) * L);
      h = fnv(h, g.en.data(), sizeof(double) * g.Q);
      if (!stat[d].empty()) h = fnv(h, stat[d].data(), sizeof(double) * g.Q);
    }
    key.push_back(h);
    const void* bufs[] = {Rov, Rqp, Mm, What, sig, ctx->ws[WS_SYRK_PART], ctx->ws[WS_SYRK_SCALE],
                          ctx->ws[WS_SCREEN_A], ctx->ws[WS_SCREEN_PANEL], ctx->ws[WS_SIGMA_PART],
                          ctx->ws[WS_SIGMA_W], ctx->ws[WS_SIGMA_RT]};
    for (const void* p : bufs)
      key_add(key, reinterpret_cast<uintptr_t>(p));
    return key;
  };
  int replayed = 0;
  if (flags & GW_BATCH_GRAPH) {
    if (ctx->batch_graph && ctx->batch_graph->key == make_key()) {
      GW_HIP(ctx, hipGraphLaunch(ctx->batch_graph->exec, ctx->stream));
      replayed = 1;
    } else {
      gw::drop_batch_graph(ctx);
      GW_TRY(rest());                 // eager run: sizes the workspace, gives this call's results
      const std::vector<uint64_t> key = make_key();
      GW_TRY(gw::begin_capture(ctx));
      const gw_status s = rest();
      gw_graph_s g;
      const gw_status se = gw::end_capture(ctx, &g);
      if (s != GW_OK) {
        if (se == GW_OK) {
          hipGraphExecDestroy(g.exec);
          hipFree(g.arena);
        }
        return s;
      }
      if (se != GW_OK) return se;
      ctx->batch_graph = new BatchGraph{g.exec, g.arena, key};
    }
  } else {
    GW_TRY(rest());
  }
  ev.rec(2, ctx->stream);

  std::vector<double> hs(s_tot + 3 * q_tot);
  GW_HIP(ctx, hipMemcpyAsync(hs.data(), sig, hs.size() * sizeof(double), hipMemcpyDeviceToHost,
                             ctx->stream));
  GW_HIP(ctx, hipStreamSynchronize(ctx->stream));
  GW_TRY(gw::check_flags(ctx));
  for (int d = 0; d < n; ++d) {
    const Mol& g = mo[d];
    gw_mol& m = mols[d];
    for (int q = 0; q < g.Q; ++q) {
      const double* r = hs.data() + s_tot + 3 * (g.q_off + q);
      m.eps_qp[q] = r[0];
      if (m.z_factor) m.z_factor[q] = r[1];
      m.status[q] = (int)r[2];
    }
    if (m.sigma_iw)
      std::memcpy(m.sigma_iw, hs.data() + g.s_off, sizeof(double) * 2 * g.Q * Pd);
  }
  if (stats) {
    stats->t_naf_ms = ev.ms(0, 1);
    stats->t_rest_ms = ev.ms(1, 2);
    stats->t_total_ms = ev.ms(0, 2);
    stats->graph_replayed = replayed;
  }
  return GW_OK;
}
