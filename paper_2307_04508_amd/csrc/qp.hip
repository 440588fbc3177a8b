// Pade analytic continuation and the quasiparticle fixed point (Sec. 2 and
// Sec. 3), FP64 on the device.  One workgroup per QP state: the Thiele
// reciprocal-difference table is built level by level with one thread per
// node, then one thread iterates E <- e_n + Re C(E - e_F + i eta) + c_n.
// The derivative for the renormalisation factor comes from differentiating
// the continued fraction's backward recurrence.
#include <cmath>
#include <vector>

#include "common.hpp"

namespace {

constexpr int kMaxPade = 256;

struct cplx {
  double re, im;
};
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, d = b.re + b.im * r;
    return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  }
  const double r = b.re / b.im, d = b.re * r + b.im;
  return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}

struct QpArgs {
  int Pd;
  const double* omega_p;   // [Pd]
  const double* sigma;     // [n_qp][Pd][2]
  const double* eps_n;     // [n_qp]
  const double* static_n;  // [n_qp] or nullptr
  double eps_f, eta, tol;
  int max_iter;
  double* out;             // [n_qp][3]: E, Z, status
};

__device__ __forceinline__ void qp_unit(const QpArgs& a, int q) {
  const int Pd = a.Pd;
  const double* __restrict__ omega_p = a.omega_p;
  const double* __restrict__ sigma = a.sigma;
  const double eps_f = a.eps_f, eta = a.eta, tol = a.tol;
  const int max_iter = a.max_iter;
  __shared__ cplx g[kMaxPade], prev[kMaxPade], coef[kMaxPade];
  __shared__ int stop;
  const int t = threadIdx.x;
  if (t < Pd) g[t] = {sigma[2 * ((int64_t)q * Pd + t)], sigma[2 * ((int64_t)q * Pd + t) + 1]};
  if (t == 0) stop = 0;
  __syncthreads();
  if (t == 0) coef[0] = g[0];
  __syncthreads();
  // level p: g_p(z_i) = (g_{p-1}(z_{p-1}) - g_{p-1}(z_i)) / ((z_i - z_{p-1}) g_{p-1}(z_i))
  for (int p = 1; p < Pd; ++p) {
    if (t == 0 && coef[p - 1].re == 0.0 && coef[p - 1].im == 0.0) stop = p;
    __syncthreads();
    if (stop) break;
    if (t < Pd) prev[t] = g[t];
    __syncthreads();
    if (t >= p && t < Pd) {
      const cplx dz = {0.0, omega_p[t] - omega_p[p - 1]};   // z = i w
      g[t] = cdiv(csub(prev[p - 1], prev[t]), cmul(dz, prev[t]));
    }
    __syncthreads();
    if (t == 0) coef[p] = g[p];
    __syncthreads();
  }
  if (t != 0) return;
  const int n_coef = stop ? stop : Pd;
  const double c_n = a.static_n ? a.static_n[q] : 0.0;
  // C(z) = a_0 / (1 + a_1 (z - z_0) / (1 + a_2 (z - z_1) / ...)) and dC/dz
  auto eval = [&](double E, cplx& C, cplx& dC) {
    const cplx z = {E - eps_f, eta};
    cplx tt = {1.0, 0.0}, dt = {0.0, 0.0};
    for (int p = n_coef - 1; p >= 1; --p) {
      const cplx u = {z.re, z.im - omega_p[p - 1]};          // z - z_{p-1}
      const cplx au = cmul(coef[p], u);
      const cplx nt = cadd({1.0, 0.0}, cdiv(au, tt));
      // d/dz [a u / t] = a / t - a u t' / t^2
      const cplx dnt = csub(cdiv(coef[p], tt), cdiv(cmul(au, dt), cmul(tt, tt)));
      tt = nt;
      dt = dnt;
    }
    C = cdiv(coef[0], tt);
    dC = cdiv(cmul({-coef[0].re, -coef[0].im}, dt), cmul(tt, tt));
  };
  double E = a.eps_n[q];
  int status = 1;
  cplx C, dC;
  for (int it = 0; it < max_iter; ++it) {
    eval(E, C, dC);
    const double En = a.eps_n[q] + C.re + c_n;
    if (!isfinite(En)) { status = 2; break; }
    const double d = fabs(En - E);
    E = En;
    if (d < tol) { status = 0; break; }
  }
  eval(E, C, dC);
  a.out[3 * q + 0] = E;
  a.out[3 * q + 1] = 1.0 / (1.0 - dC.re);
  a.out[3 * q + 2] = (double)status;
}

__global__ __launch_bounds__(kMaxPade) void qp_kernel(QpArgs a) { qp_unit(a, blockIdx.x); }

__global__ __launch_bounds__(kMaxPade) void qp_batched_kernel(Batch bt) {
  const int d = find_problem(bt.off, bt.n, blockIdx.x);
  const QpArgs a = static_cast<const QpArgs*>(bt.descs)[d];
  qp_unit(a, (int)(blockIdx.x - bt.off[d]));
}

}  // namespace

extern "C" gw_status gw_qp_solve(gw_ctx ctx, int n_qp, const double* eps_n,
                                 const double* static_n, double eps_F, int n_pade,
                                 const double* omega_pade, const double* sigma_iw,
                                 double eta, double tol, int max_iter, double* eps_qp,
                                 double* z_factor, int* status) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_qp_solve: ctx is NULL");
  gw::clear_error(ctx);
  if (ctx->capturing)
    return gw::fail(ctx, GW_EUNSUPPORTED, "gw_qp_solve synchronises and cannot be captured");
  GW_REQUIRE(ctx, n_qp >= 1 && n_pade >= 1 && n_pade <= kMaxPade && max_iter >= 1 && tol > 0,
             "gw_qp_solve: bad sizes (n_qp=%d n_pade=%d max_iter=%d)", n_qp, n_pade, max_iter);
  GW_REQUIRE(ctx, eps_n && omega_pade && sigma_iw && eps_qp && status,
             "gw_qp_solve: NULL argument");
  for (int i = 0; i < n_pade; ++i)
    for (int k = i + 1; k < n_pade; ++k)
      if (omega_pade[i] == omega_pade[k])
        return gw::fail(ctx, GW_EPADE, "gw_qp_solve: Pade nodes %d and %d coincide", i, k);
  GW_HIP(ctx, hipSetDevice(ctx->device));
  const double* d_op = gw::stage_t(ctx, omega_pade, n_pade);
  const double* d_en = gw::stage_t(ctx, eps_n, n_qp);
  const double* d_st = static_n ? gw::stage_t(ctx, static_n, n_qp) : nullptr;
  if (!d_op || !d_en || (static_n && !d_st)) return GW_EINVAL;
  double* d_out = static_cast<double*>(gw::ws_get(ctx, WS_QP, (size_t)3 * n_qp * sizeof(double)));
  if (!d_out) return GW_ENOMEM;
  hipLaunchKernelGGL(qp_kernel, dim3(n_qp), dim3(kMaxPade), 0, ctx->stream,
                     QpArgs{n_pade, d_op, sigma_iw, d_en, d_st, eps_F, eta, tol, max_iter, d_out});
  GW_TRY(gw::launch_check(ctx, "qp_kernel"));
  std::vector<double> h(3 * (size_t)n_qp);
  GW_HIP(ctx, hipMemcpyAsync(h.data(), d_out, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                             ctx->stream));
  GW_HIP(ctx, hipStreamSynchronize(ctx->stream));
  GW_TRY(gw::check_flags(ctx));
  for (int q = 0; q < n_qp; ++q) {
    eps_qp[q] = h[3 * q];
    if (z_factor) z_factor[q] = h[3 * q + 1];
    status[q] = (int)h[3 * q + 2];
  }
  return GW_OK;
}

namespace gw {

// Batched QP kernel into device outputs out[3 * state] (states of all jobs
// concatenated in job order); no synchronisation.
gw_status qp_batched_launch(gw_ctx ctx, const std::vector<QpJob>& jobs, double eta, double tol,
                            int max_iter, double* out) {
  std::vector<QpArgs> d;
  std::vector<int64_t> off(1, 0);
  size_t so = 0;
  for (const QpJob& j : jobs) {
    d.push_back(QpArgs{j.n_pade, j.omega_pade, j.sigma_iw, j.eps_n, j.static_n, j.eps_F, eta,
                       tol, max_iter, out + 3 * so});
    off.push_back(off.back() + j.n_qp);
    so += j.n_qp;
  }
  if (off.back() == 0) return GW_OK;
  Batch bt;
  GW_TRY(stage_batch(ctx, d, off, 1, bt));
  hipLaunchKernelGGL(qp_batched_kernel, dim3((unsigned)off.back()), dim3(kMaxPade), 0,
                     ctx->stream, bt);
  return launch_check(ctx, "qp_batched_kernel");
}

}  // namespace gw

extern "C" gw_status gw_qp_solve_batched(gw_ctx ctx, int n_jobs, const gw_qp_job* jobs,
                                         double eta, double tol, int max_iter) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_qp_solve_batched: ctx is NULL");
  gw::clear_error(ctx);
  if (ctx->capturing)
    return gw::fail(ctx, GW_EUNSUPPORTED, "gw_qp_solve_batched synchronises and cannot be captured");
  GW_REQUIRE(ctx, n_jobs >= 0 && (n_jobs == 0 || jobs) && max_iter >= 1 && tol > 0,
             "gw_qp_solve_batched: bad arguments");
  size_t n_states = 0;
  for (int d = 0; d < n_jobs; ++d) {
    const gw_qp_job& j = jobs[d];
    GW_REQUIRE(ctx, j.n_qp >= 1 && j.n_pade >= 1 && j.n_pade <= kMaxPade,
               "gw_qp_solve_batched: job %d: bad sizes", d);
    GW_REQUIRE(ctx, j.eps_n && j.omega_pade && j.sigma_iw && j.eps_qp && j.status,
               "gw_qp_solve_batched: job %d: NULL argument", d);
    for (int i = 0; i < j.n_pade; ++i)
      for (int k = i + 1; k < j.n_pade; ++k)
        if (j.omega_pade[i] == j.omega_pade[k])
          return gw::fail(ctx, GW_EPADE, "gw_qp_solve_batched: job %d: Pade nodes %d and %d coincide",
                          d, i, k);
    n_states += j.n_qp;
  }
  if (n_jobs == 0) return GW_OK;
  GW_HIP(ctx, hipSetDevice(ctx->device));
  std::vector<gw::QpJob> qj;
  for (int d = 0; d < n_jobs; ++d) {
    const gw_qp_job& j = jobs[d];
    const double* d_op = gw::stage_t(ctx, j.omega_pade, j.n_pade);
    const double* d_en = gw::stage_t(ctx, j.eps_n, j.n_qp);
    const double* d_st = j.static_n ? gw::stage_t(ctx, j.static_n, j.n_qp) : nullptr;
    if (!d_op || !d_en || (j.static_n && !d_st)) return GW_EINVAL;
    qj.push_back(gw::QpJob{j.n_qp, j.n_pade, d_op, j.sigma_iw, d_en, d_st, j.eps_F});
  }
  double* d_out = static_cast<double*>(gw::ws_get(ctx, WS_QP, 3 * n_states * sizeof(double)));
  if (!d_out) return GW_ENOMEM;
  GW_TRY(gw::qp_batched_launch(ctx, qj, eta, tol, max_iter, d_out));
  std::vector<double> h(3 * n_states);
  GW_HIP(ctx, hipMemcpyAsync(h.data(), d_out, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                             ctx->stream));
  GW_HIP(ctx, hipStreamSynchronize(ctx->stream));
  GW_TRY(gw::check_flags(ctx));
  size_t s = 0;
  for (int d = 0; d < n_jobs; ++d) {
    const gw_qp_job& j = jobs[d];
    for (int q = 0; q < j.n_qp; ++q, ++s) {
      j.eps_qp[q] = h[3 * s];
      if (j.z_factor) j.z_factor[q] = h[3 * s + 1];
      j.status[q] = (int)h[3 * s + 2];
    }
  }
  return GW_OK;
}
