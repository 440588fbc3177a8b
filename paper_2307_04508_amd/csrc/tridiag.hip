// Householder reduction of a symmetric matrix to tridiagonal form, the first
// stage of the NAF eigendecomposition (Eq. 12).  Output in the LAPACK
// dsytrd form (lower): diagonal d, sub-diagonal e, reflector scalars tau,
// and the reflectors v_k (v_k(k+1) = 1 implied) stored below the
// sub-diagonal of column k, column-major.
//
// The reduction is one column per step, with the whole matrix held on chip:
// a persistent cooperative launch of G workgroups, workgroup g keeping rows
// g, g + G, g + 2G, ... (at most 13) in registers (and, past 3072 columns, one
// column slot per row in LDS), thread t of it columns t, t + 512, ....  Step
// k of the unblocked algorithm needs
//   the Householder vector v_k of column k of A^(k-1),
//   p = tau A^(k-1) v_k (rows > k),   w = p - (tau/2)(p.v_k) v_k,
//   A^(k) = A^(k-1) - v_k w^T - w v_k^T.
// The rank-2 update of step k-1 and the product with v_k touch the same
// registers, so they run as one pass; column k of A^(k-1) is formed by every
// workgroup from the pre-update column (published by its owners in the
// previous pass) and the previous step's v and w.  A step then exchanges
// two vectors through HBM (p, and the next pre-update column) and needs a
// single barrier across the G workgroups.  Every workgroup computes v_k,
// tau and the reductions redundantly, in the same order, so all hold the
// same bits.  The barrier spins a bounded number of times; a timeout sets
// the error flag and every workgroup leaves.
#include <algorithm>
#include <cmath>

#include "common.hpp"

namespace {

constexpr int TNT = 512;          // threads per workgroup
constexpr int TNW = TNT / 64;     // waves per workgroup
constexpr int TR = 13;            // matrix rows held per workgroup (max)
constexpr int TC_MAX = 7;         // column slots per thread (max): n <= 3584
constexpr int TC_REG = 6;         // column slots per thread held in registers

struct TriJob {
  double* K;          // [n][n] symmetric (full); out: reflectors (column-major, below sub-diag)
  double* d;          // [n]
  double* e;          // [n - 1]
  double* tau;        // [n - 1]
  double* pbuf;       // [2][n] exchange buffers (by step parity)
  double* colbuf;     // [2][n]
  unsigned* count;    // barrier: top counter, then group counters kCtrStride apart; zero on entry
  int n, G, wg0;      // order, workgroups, first workgroup of the job in the grid
};

// The barrier is two-level: workgroups arrive on the counter of their group
// of kBarGroup, and the last arrival of a group arrives on the top counter,
// which everyone polls.  One counter under all ~230 arrivals serialises
// them (3.4 us per barrier at 231 workgroups, 1.8 us with groups of 32).
constexpr int kBarGroup = 32;
constexpr int kCtrStride = 32;    // unsigneds: one 128-byte line per counter

// Sum over the 64 lanes of a wave, complete in lane 63 only (other lanes
// hold partial sums): the half-wave sums (half_wave_sum), then lane 31
// broadcast into rows 2 and 3.  VALU only, no LDS round trip per step.
constexpr int kLastLane = 63;
__device__ __forceinline__ double wave_total(double v) {
  v = half_wave_sum(v);
  v += dpp_move<0x143, 0xC>(v);    // row_bcast:31 into rows 2 and 3
  return v;
}

// Exchange-buffer accesses are device-coherent (other workgroups, other
// XCDs), issued as global (not flat) memory operations.
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) unsigned guint;
typedef __attribute__((address_space(1))) int gint;
__device__ __forceinline__ double ld_dev(const double* p) {
  return __hip_atomic_load((const gdouble*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(double* p, double v) {
  __hip_atomic_store((gdouble*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Barrier across the G workgroups of one job (the counters only grow, so
// pass number q waits for q arrivals of each group on the top counter).
// Every wave first waits for its own memory operations to complete; only
// then does thread 0 arrive.  All data that crosses workgroups inside the
// kernel (pbuf, colbuf) is written and read with device-scope atomic
// accesses, which are performed at the device's coherence point, so
// completed stores are visible to the loads that follow the barrier without
// a release / acquire pair: those would add an L2 write-back and an L2
// invalidate per step (~2 us of a ~17 us step at order 3000) for plain data
// that no other workgroup reads before the kernel ends.  The group's last
// arrival sees the group count in the value its own increment returns, and
// only then increments the top counter, so every arrival of the group has
// been performed before the top counter moves.  Returns false after
// spin_limit polls or when another workgroup raised the error flag.
__device__ bool group_barrier(unsigned* count_ptr, int g, int G, unsigned pass, int* err_ptr,
                              int spin_limit, int* s_ok) {
  guint* count = (guint*)count_ptr;
  gint* err = (gint*)err_ptr;
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    const int gi = g / kBarGroup, n_grp = (G + kBarGroup - 1) / kBarGroup;
    const unsigned gsize = (unsigned)min(kBarGroup, G - gi * kBarGroup);
    const unsigned prev = __hip_atomic_fetch_add(count + (1 + gi) * kCtrStride, 1u,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (prev + 1 == pass * gsize)
      __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned target = pass * (unsigned)n_grp;
    int ok = 1;
    for (int it = 0;; ++it) {
      if (__hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
      if (it >= spin_limit || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    *s_ok = ok;
  }
  __syncthreads();
  return *s_ok != 0;
}

template <int C>
__global__ __launch_bounds__(TNT, 1) void tridiag_kernel(const TriJob* __restrict__ jobs,
                                                         int n_jobs, int* err, int spin_limit) {
  constexpr int NV = TNT * C;                       // vector length per workgroup (>= n)
  constexpr int CR = C < TC_REG ? C : TC_REG;       // slots in registers
  constexpr int CL = C - CR;                        // slots in LDS
  __shared__ double vsh[2][NV];                     // v of the last two steps (by parity)
  __shared__ double wsh[NV];                        // w of the previous step
  __shared__ double red[TNW][TR + 2];               // per-wave partial sums
  __shared__ double alds[CL > 0 ? CL * TR * TNT : 1];
  __shared__ double bc[2];
  __shared__ int s_ok;

  int jb = 0;
  while (jb + 1 < n_jobs && jobs[jb + 1].wg0 <= (int)blockIdx.x) ++jb;
  const TriJob J = jobs[jb];
  const int g = (int)blockIdx.x - J.wg0;
  if (g < 0 || g >= J.G) return;
  const int n = J.n, G = J.G;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int R = (n - g + G - 1) / G;                // rows of this workgroup (<= TR)

  // load the rows; publish column 0 (pre-update) for step 0
  double a[TR][CR > 0 ? CR : 1];
#pragma unroll
  for (int r = 0; r < TR; ++r) {
    const int i = g + G * r;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int j = tid + TNT * c;
      const double v = (r < R && j < n) ? J.K[(size_t)i * n + j] : 0.0;
      if (c < CR) a[r][c < CR ? c : 0] = v;
      else alds[((c - CR) * TR + r) * TNT + tid] = v;
    }
    if (tid == 0 && r < R) st_dev(&J.colbuf[i], a[r][0]);
  }
  for (int x = tid; x < NV; x += TNT) {
    vsh[0][x] = 0.0;
    vsh[1][x] = 0.0;
    wsh[x] = 0.0;
  }
  double vp[C], w[C], vn[C];
#pragma unroll
  for (int c = 0; c < C; ++c) vp[c] = w[c] = vn[c] = 0.0;
  double tau_prev = 0.0;
  // every workgroup has read K before any reflector is written into it
  if (!group_barrier(J.count, g, G, 1u, err, spin_limit, &s_ok)) return;

  for (int k = 0; k + 1 < n; ++k) {
    const int pc = k & 1, pp = pc ^ 1;
    // ---- column k of A^(k-1) and the previous step's w, on own indices
    double pv[C], cv[C];
    double sp = 0.0;
    const double pk = k > 0 ? ld_dev(&J.pbuf[pp * n + k]) : 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int j = tid + TNT * c;
      const bool on = j >= k && j < n;
      pv[c] = (on && k > 0) ? ld_dev(&J.pbuf[pp * n + j]) : 0.0;
      cv[c] = on ? ld_dev(&J.colbuf[pc * n + j]) : 0.0;
      sp += pv[c] * vp[c];
    }
    sp = wave_total(sp);
    if (lane == kLastLane) red[wave][TR] = sp;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < TNW; ++q) s += red[q][TR];
    const double h = 0.5 * tau_prev * s;
    const double vpk = vsh[pp][k];
    const double wk = pk - h * vpk;
    double xp = 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int j = tid + TNT * c;
      w[c] = pv[c] - h * vp[c];
      wsh[j] = w[c];
      cv[c] -= vp[c] * wk + w[c] * vpk;
      if (j >= k + 2 && j < n) xp += cv[c] * cv[c];
      if (j == k) bc[0] = cv[c];
      if (j == k + 1) bc[1] = cv[c];
    }
    xp = wave_total(xp);
    if (lane == kLastLane) red[wave][TR + 1] = xp;
    __syncthreads();
    double xn2 = 0.0;
#pragma unroll
    for (int q = 0; q < TNW; ++q) xn2 += red[q][TR + 1];
    const double dk = bc[0], alpha = bc[1];
    // ---- Householder vector of column k (LAPACK dlarfg convention)
    double beta = alpha, t = 0.0, scal = 0.0;
    if (xn2 > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
      t = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int j = tid + TNT * c;
      vn[c] = j == k + 1 ? 1.0 : ((j >= k + 2 && j < n) ? cv[c] * scal : 0.0);
      vsh[pc][j] = vn[c];
    }
    if (g == 0 && tid == 0) {
      J.d[k] = dk;
      J.e[k] = beta;
      J.tau[k] = t;
    }
    __syncthreads();
    if (tid < R) {
      const int i = g + G * tid;
      if (i >= k + 2) J.K[(size_t)k * n + i] = vsh[pc][i];
    }
    // ---- rank-2 update of step k-1 fused with p = tau A^(k-1) v_k
    const int tnext = (k + 1) % TNT, cnext = (k + 1) / TNT;
    // Rows i <= k and column slots wholly left of column k + 1 are finished:
    // nothing later reads them, so they are skipped (both tests are uniform
    // across the workgroup); the work per step shrinks with (n - k)^2.
#pragma unroll
    for (int r = 0; r < TR; ++r) {
      if (r < R && g + G * r > k) {
        const int i = g + G * r;
        const double vpi = vsh[pp][i], wi = wsh[i];
        double acc = 0.0, cn = 0.0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          if (TNT * (c + 1) <= k + 1) continue;
          double x;
          if (c < CR) {
            x = a[r][c < CR ? c : 0] - (vpi * w[c] + wi * vp[c]);
            a[r][c < CR ? c : 0] = x;
          } else {
            double& ref = alds[((c - CR) * TR + r) * TNT + tid];
            x = ref - (vpi * w[c] + wi * vp[c]);
            ref = x;
          }
          acc += x * vn[c];
          if (c == cnext) cn = x;
        }
        acc = wave_total(acc);
        if (lane == kLastLane) red[wave][r] = acc;
        if (tid == tnext && i >= k + 1) st_dev(&J.colbuf[pp * n + i], cn);
      }
    }
    __syncthreads();
    if (tid < R) {
      const int i = g + G * tid;
      if (i > k) {
        double p = 0.0;
#pragma unroll
        for (int q = 0; q < TNW; ++q) p += red[q][tid];
        st_dev(&J.pbuf[pc * n + i], t * p);
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) vp[c] = vn[c];
    tau_prev = t;
    if (!group_barrier(J.count, g, G, (unsigned)(k + 2), err, spin_limit, &s_ok)) return;
  }
  // last diagonal entry: column n-1 of A^(n-2)
  if (g == 0 && tid == 0) {
    if (n == 1) {
      J.d[0] = a[0][0];
    } else {
      const int k = n - 1, pp = (k - 1) & 1;
      const double p = ld_dev(&J.pbuf[pp * n + k]);
      const double vv = vsh[pp][k];
      const double wl = p - 0.5 * tau_prev * (p * vv) * vv;
      J.d[k] = ld_dev(&J.colbuf[(k & 1) * n + k]) - 2.0 * vv * wl;
    }
  }
}

template <int C>
void* tridiag_fn() {
  return reinterpret_cast<void*>(&tridiag_kernel<C>);
}

void* tridiag_fn_for(int C) {
  switch (C) {
    case 1: return tridiag_fn<1>();
    case 2: return tridiag_fn<2>();
    case 3: return tridiag_fn<3>();
    case 4: return tridiag_fn<4>();
    case 5: return tridiag_fn<5>();
    case 6: return tridiag_fn<6>();
    default: return tridiag_fn<7>();
  }
}

}  // namespace

namespace gw {

int tridiag_max_order(gw_ctx ctx) {
  int n_cu = 0;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device) !=
      hipSuccess)
    return 0;
  return std::min(TR * n_cu, TNT * TC_MAX);
}

// Reduce every job's matrix to tridiagonal form.  Jobs are packed, largest
// first, into cooperative launches whose workgroups are all resident; each
// launch uses the column-slot count of its largest job.  Asynchronous on the
// context's stream; a barrier timeout raises ctx->d_flags[1].
gw_status tridiag_jobs(gw_ctx ctx, const std::vector<TriIn>& in) {
  const int n_jobs = (int)in.size();
  if (n_jobs == 0) return GW_OK;
  int n_cu = 0;
  GW_HIP(ctx, hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device));
  // scratch: per job 4 n doubles of exchange buffers + the barrier counters
  // (top + one per group of kBarGroup workgroups, a 128-byte line each)
  auto workgroups = [&](int n) { return std::min(n_cu, (n + TR - 1) / TR); };
  auto ctr_doubles = [&](int n) {
    return (size_t)(1 + (workgroups(n) + kBarGroup - 1) / kBarGroup) * kCtrStride / 2;
  };
  size_t sc = 0;
  for (const TriIn& j : in) sc += 4 * (size_t)std::max(j.n, 1) + ctr_doubles(j.n);
  double* ws = static_cast<double*>(ws_get(ctx, WS_TRI, sc * sizeof(double)));
  if (!ws) return GW_ENOMEM;
  GW_TRY(fill_zero(ctx, ws, (int64_t)sc));
  std::vector<TriJob> all(n_jobs);
  size_t o = 0;
  for (int d = 0; d < n_jobs; ++d) {
    const TriIn& j = in[d];
    if (j.n < 1 || j.n > std::min(TR * n_cu, TNT * TC_MAX))
      return fail(ctx, GW_EINVAL, "tridiagonalisation: order %d outside [1, %d]", j.n,
                  std::min(TR * n_cu, TNT * TC_MAX));
    TriJob t{};
    t.K = j.K;
    t.d = j.d;
    t.e = j.e;
    t.tau = j.tau;
    t.pbuf = ws + o;
    t.colbuf = ws + o + 2 * (size_t)j.n;
    t.count = reinterpret_cast<unsigned*>(ws + o + 4 * (size_t)j.n);
    t.n = j.n;
    t.G = workgroups(j.n);
    t.wg0 = 0;
    all[d] = t;
    o += 4 * (size_t)j.n + ctr_doubles(j.n);
  }
  std::vector<int> order(n_jobs);
  for (int d = 0; d < n_jobs; ++d) order[d] = d;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return all[x].n > all[y].n; });
  size_t pos = 0;
  while (pos < order.size()) {
    const int C = (all[order[pos]].n + TNT - 1) / TNT;
    void* fn = tridiag_fn_for(C);
    int per_cu = 0;
    GW_HIP(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, TNT, 0));
    const int cap = per_cu * n_cu;
    if (cap < all[order[pos]].G)
      return fail(ctx, GW_EDEVICE, "tridiagonalisation: %d resident workgroups, %d needed", cap,
                  all[order[pos]].G);
    std::vector<TriJob> grp;
    int wg = 0;
    while (pos < order.size() && wg + all[order[pos]].G <= cap) {
      TriJob t = all[order[pos]];
      t.wg0 = wg;
      wg += t.G;
      grp.push_back(t);
      ++pos;
    }
    const TriJob* dj = static_cast<const TriJob*>(stage(ctx, grp.data(), grp.size() * sizeof(TriJob)));
    if (!dj) return GW_EINVAL;
    int nj = (int)grp.size();
    int* err = ctx->d_flags + 1;
    int spin = 1 << 21;
    void* args[] = {&dj, &nj, &err, &spin};
    GW_HIP(ctx, hipLaunchCooperativeKernel(fn, dim3(wg), dim3(TNT), args, 0, ctx->stream));
  }
  return GW_OK;
}

}  // namespace gw
