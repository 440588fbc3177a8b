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
// that no other workgroup reads before the kernel ends.  This visibility
// argument rests on how gfx950 performs agent-scope atomics (past the
// per-XCD L2 caches); the HIP memory model by itself orders relaxed atomics
// only through a release / acquire pair.  The group's last
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

// ---------------------------------------------------------------- blocked
// Orders past the on-chip limit: the matrix stays in HBM (full symmetric
// storage) and is reduced in panels of HB columns (the LAPACK dsytrd /
// dlatrd scheme).  Within a panel the trailing matrix keeps its values at
// the panel start; column k is corrected by the panel's earlier reflectors,
//   a = A(k:, k) - V W(k, :)^T - W V(k, :)^T,
// its Householder vector v taken, and
//   w = tau (A22 v - V (W^T v) - W (V^T v)),  w -= (tau / 2)(w^T v) v
// stored as a column of W.  After the panel, A22 -= V W^T + W V^T on FP64
// MFMA.  One cooperative launch per panel, two device-wide barriers per
// column: (1) the corrected column and its partial norms, (2) A22 v and the
// partial products W^T v, V^T v and v^T A22 v, from which every workgroup
// finishes w on its rows (yhat^T v = v^T A22 v - 2 (W^T v).(V^T v)).
// Workgroup g owns rows g, g + G, ...: thread t of it row g + G t in the
// row-wise phases; in A22 v each wave takes every fourth owned row and its
// lanes stride over the row, with v staged in LDS in chunks.  Values that
// cross workgroups are written and read with device-scope atomic accesses
// (as in the on-chip kernel); the matrix itself is read with plain loads
// (nothing writes the trailing rows during a launch).
constexpr int HB = 32;            // panel width (columns)
constexpr int HT = 512;           // threads per workgroup
constexpr int HCH = 8192;         // v chunk staged in LDS (doubles)
constexpr int HB2 = 2 * HB;       // row stride of the panel buffers
constexpr int HRED = 2 * HB + 2;  // per-workgroup partials: norm, W^T v, V^T v, v^T A22 v

struct HbmArgs {
  double* K;          // [n][n]; out: reflector k in K[k n + i], i >= k + 2
  int n, k0, jb;      // panel columns k0 .. k0 + jb - 1
  int last;           // this panel holds reflector n - 2 (also sets d[n - 1])
  double* d;
  double* e;
  double* tau;
  double* VW;         // [n][2 HB]: V in columns 0 .. HB-1, W in HB .. 2 HB-1
  double* WV;         // [n][2 HB]: the same with the halves swapped
  double* abuf;       // [HB][n] corrected column j of the panel in row j
  double* ybuf;       // [n] A22 v, then the corrected y
  double* red;        // [G][HRED]
  unsigned* count;    // barrier counters, zero before the first panel
  unsigned pass0;     // barriers passed by the earlier panels
  int* err;
  int spin_limit;
};

// Sum over the workgroup, result in every thread (deterministic order).
__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_total(v);
  __syncthreads();
  if (lane == kLastLane) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < HT / 64; ++q) t += sh[q];
  return t;
}

// Sum over workgroups of red[g][col] for cols in [c0, c0 + nc) (nc <= 64),
// into out[0 .. nc) in LDS: thread (col, q) sums workgroups q, q + 4, ...
// (loads issued 16 at a time), then the four partials in order.
__device__ __forceinline__ void sum_partials(const double* red, int G, int c0, int nc,
                                             double* part, double* out) {
  const int c = threadIdx.x & 63, q = threadIdx.x >> 6;
  double s = 0.0;
  if (c < nc) {
    for (int g0 = q; g0 < G; g0 += 16 * (HT / 64)) {
      double t[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int g = g0 + u * (HT / 64);
        t[u] = g < G ? ld_dev(&red[(size_t)g * HRED + c0 + c]) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) s += t[u];
    }
  }
  part[q * 64 + c] = s;
  __syncthreads();
  if (threadIdx.x < nc) {
    double t = 0.0;
#pragma unroll
    for (int r = 0; r < HT / 64; ++r) t += part[r * 64 + threadIdx.x];
    out[threadIdx.x] = t;
  }
  __syncthreads();
}

// Sum over workgroups of red[g][col] for one column, in every thread.
__device__ __forceinline__ double sum_column(const double* red, int G, int col, double* sh) {
  double s = 0.0;
  for (int g = threadIdx.x; g < G; g += HT) s += ld_dev(&red[(size_t)g * HRED + col]);
  return block_sum(s, sh);
}

constexpr int HROWS = 128;        // rows per workgroup (n <= HROWS x workgroups)
constexpr int HMLP = 16;          // loads in flight per lane in A22 v

__global__ __launch_bounds__(HT) void tri_hbm_panel_kernel(HbmArgs a) {
  __shared__ double vch[HCH];
  __shared__ double own[HROWS * HB2];               // own rows of [V | W] for this panel
  __shared__ double ownY[HROWS];                    // own rows of y (raw, then corrected)
  __shared__ double part[HT];
  __shared__ double sh[HT / 64];
  __shared__ double rowV[HB], rowW[HB], sWV[2 * HB];
  __shared__ int s_ok;
  const int g = blockIdx.x, G = gridDim.x, tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int n = a.n;
  const int R = (n - g + G - 1) / G;                // rows owned (<= HROWS)
  const int my = g + G * tid;                       // row of this thread in row-wise phases
  const bool mine = tid < R;                        // (my < n)
  double* ow = own + (size_t)(mine ? tid : 0) * HB2;
  unsigned pass = a.pass0;
  double tau_p = 0.0;                               // previous column's tau
  // Each column's corrected values go to a region of abuf of their own,
  // written once per launch (device-scope stores, which bypass the
  // per-XCD L2), so after the barrier the other workgroups read them with
  // plain loads: no cache holds an older copy once the caches are
  // invalidated here, at the start of the launch.
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  for (int j = 0; j <= a.jb; ++j) {
    const int k = a.k0 + j;
    double* acol = a.abuf + (size_t)j * n;
    // ---- phase 1: finish w of column j - 1 (jp), correct column k.
    // From the previous barrier: sWV = [W^T v, V^T v, v^T A22 v], so that
    // yhat = y - V (W^T v) - W (V^T v) and yhat^T v = v^T A22 v - 2 (W^T v).(V^T v)
    const int jp = j - 1;
    double c_p = 0.0;
    if (j > 0) {
      sum_partials(a.red, G, 1, 2 * jp + 1, part, sWV);
      double cross = 0.0;
      for (int q = 0; q < jp; ++q) cross += sWV[q] * sWV[jp + q];
      c_p = 0.5 * tau_p * tau_p * (sWV[2 * jp] - 2.0 * cross);
    }
    if (tid < j) {
      rowV[tid] = ld_dev(&a.VW[(size_t)k * HB2 + tid]);
      if (tid < jp) rowW[tid] = ld_dev(&a.VW[(size_t)k * HB2 + HB + tid]);
    }
    __syncthreads();
    if (j > 0 && tid == 0) {
      // row k of the just-finished column, from its raw y (v_k = 1)
      double y = ld_dev(&a.ybuf[k]);
      for (int q = 0; q < jp; ++q) y -= rowV[q] * sWV[q] + rowW[q] * sWV[jp + q];
      rowW[jp] = tau_p * y - c_p;
    }
    if (j > 0 && mine && my >= k) {
      double y = ownY[tid];
      for (int q = 0; q < jp; ++q) y -= ow[q] * sWV[q] + ow[HB + q] * sWV[jp + q];
      const double wi = tau_p * y - c_p * ow[jp];
      ow[HB + jp] = wi;
      st_dev(&a.VW[(size_t)my * HB2 + HB + jp], wi);
      st_dev(&a.WV[(size_t)my * HB2 + jp], wi);
    }
    __syncthreads();
    if (j == a.jb) {
      // after the panel's last column: the final diagonal entry
      if (a.last && mine && my == n - 1) {
        double x = a.K[(size_t)(n - 1) * n + (n - 1)];
        for (int q = 0; q < j; ++q) x -= ow[q] * rowW[q] + ow[HB + q] * rowV[q];
        a.d[n - 1] = x;
      }
      break;
    }
    double ai = 0.0, nrm = 0.0;
    if (mine && my >= k) {
      double x = a.K[(size_t)my * n + k];
      for (int q = 0; q < j; ++q) x -= ow[q] * rowW[q] + ow[HB + q] * rowV[q];
      ai = x;
      st_dev(&acol[my], x);
      if (my >= k + 2) nrm = x * x;
    }
    nrm = block_sum(nrm, sh);
    if (tid == 0) st_dev(&a.red[(size_t)g * HRED], nrm);
    if (!group_barrier(a.count, g, G, ++pass, a.err, a.spin_limit, &s_ok)) return;
    // ---- phase 2: Householder vector, A22 v, partial W^T v, V^T v, v^T A22 v
    const double xn2 = sum_column(a.red, G, 0, sh);
    const double alpha = acol[k + 1];
    double beta = alpha, t = 0.0, scal = 0.0;
    if (xn2 > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
      t = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    if (g == 0 && tid == 0) {
      a.d[k] = acol[k];
      a.e[k] = beta;
      a.tau[k] = t;
    }
    const int lo = k + 1;
    if (mine && my >= lo) {
      const double vi = my == lo ? 1.0 : ai * scal;
      ow[j] = vi;
      st_dev(&a.VW[(size_t)my * HB2 + j], vi);
      st_dev(&a.WV[(size_t)my * HB2 + HB + j], vi);
      if (my >= k + 2) a.K[(size_t)k * n + my] = vi;
    }
    // A22 v over rows and columns >= k + 1, v staged in LDS chunk by chunk;
    // row r of the workgroup's own rows is summed by wave r % (HT / 64) and
    // kept in lane r / (HT / 64) of it.  Successive columns visit the rows
    // in opposite directions: the passes over A22 (up to a few hundred MB)
    // then begin with the rows the previous pass read last, which the
    // memory-side cache still holds.  Each row's sum does not depend on
    // the order in which the rows are visited.
    const bool rows_down = (k & 1) != 0;
    const int my_rows = R > wave ? (R - 1 - wave) / (HT / 64) + 1 : 0;
    double yacc = 0.0;
    for (int c0 = lo; c0 < n; c0 += HCH) {
      const int c1 = min(n, c0 + HCH);
      __syncthreads();
      for (int l0 = c0 + tid; l0 < c1; l0 += 8 * HT) {
        double t8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int l = l0 + u * HT;
          t8[u] = (l < c1 && l > lo) ? acol[l] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int l = l0 + u * HT;
          if (l < c1) vch[l - c0] = l == lo ? 1.0 : t8[u] * scal;
        }
      }
      __syncthreads();
      for (int q = 0; q < my_rows; ++q) {
        const int r = wave + (HT / 64) * (rows_down ? my_rows - 1 - q : q);
        const int i = g + G * r;
        if (i < lo) continue;
        const double* row = a.K + (size_t)i * n;
        // HMLP independent partial sums keep HMLP loads in flight per lane:
        // the pass is bound by memory latency times the loads in flight, so
        // a row costs ceil(len / (64 HMLP)) round trips.  Past the row's end
        // a lane reloads its last element (clamped index, no branch) and
        // multiplies it by zero, so the last pass is one round trip too.
        double p[HMLP];
#pragma unroll
        for (int u = 0; u < HMLP; ++u) p[u] = 0.0;
        for (int l = c0 + lane; l < c1; l += HMLP * 64) {
          double x[HMLP], vv[HMLP];
#pragma unroll
          for (int u = 0; u < HMLP; ++u) {
            const int li = l + u * 64;
            const int lc = li < c1 ? li : c1 - 1;
            x[u] = row[lc];
            vv[u] = li < c1 ? vch[lc - c0] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < HMLP; ++u) p[u] += x[u] * vv[u];
        }
#pragma unroll
        for (int w = HMLP / 2; w > 0; w /= 2)
#pragma unroll
          for (int u = 0; u < w; ++u) p[u] += p[u + w];
        double s = wave_total(p[0]);
        const double sr = __shfl(s, kLastLane);
        if (lane == r / (HT / 64)) yacc += sr;
      }
    }
    {
      const int r = (HT / 64) * lane + wave;         // the row this lane accumulated
      const int i = g + G * r;
      if (r < R) {
        ownY[r] = yacc;
        if (i >= lo) st_dev(&a.ybuf[i], yacc);
      }
    }
    __syncthreads();
    // partials over own rows: W^T v (0 .. j-1), V^T v (j .. 2j-1), v^T y (2j)
    {
      const int c = tid & 63, q = tid >> 6;
      double sacc = 0.0;
      if (c <= 2 * j) {
        for (int r = q; r < R; r += HT / 64) {
          const int i = g + G * r;
          if (i < lo) continue;
          const double vr = own[(size_t)r * HB2 + j];
          const double x = c < j ? own[(size_t)r * HB2 + HB + c]
                                 : (c < 2 * j ? own[(size_t)r * HB2 + c - j] : ownY[r]);
          sacc += x * vr;
        }
      }
      part[q * 64 + c] = sacc;
      __syncthreads();
      if (tid <= 2 * j) {
        double u = 0.0;
#pragma unroll
        for (int q2 = 0; q2 < HT / 64; ++q2) u += part[q2 * 64 + tid];
        st_dev(&a.red[(size_t)g * HRED + 1 + tid], u);
      }
    }
    tau_p = t;
    if (!group_barrier(a.count, g, G, ++pass, a.err, a.spin_limit, &s_ok)) return;
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
gw_status tridiag_jobs(gw_ctx ctx, const std::vector<TriIn>& in, WsSlot slot) {
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
  double* ws = static_cast<double*>(ws_get(ctx, slot, sc * sizeof(double)));
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
  // First fit decreasing: a launch takes the largest job left, then every
  // smaller job left that still fits its resident workgroups (a launch lasts
  // as long as its largest job, so the smaller ones ride along)
  std::vector<char> done(n_jobs, 0);
  size_t pos = 0;
  while (pos < order.size()) {
    while (pos < order.size() && done[order[pos]]) ++pos;
    if (pos == order.size()) break;
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
    for (size_t q = pos; q < order.size(); ++q) {
      const int d = order[q];
      if (done[d] || wg + all[d].G > cap) continue;
      TriJob t = all[d];
      t.wg0 = wg;
      wg += t.G;
      grp.push_back(t);
      done[d] = 1;
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

gw_status tridiag_blocked(gw_ctx ctx, const TriIn& job) {
  const int n = job.n;
  if (n < 1) return fail(ctx, GW_EINVAL, "tridiag_blocked: order %d", n);
  if (n == 1) {
    GW_HIP(ctx, hipMemcpyAsync(job.d, job.K, sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    return GW_OK;
  }
  int n_cu = 0, per_cu = 0;
  GW_HIP(ctx, hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device));
  GW_HIP(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(
                  &per_cu, reinterpret_cast<const void*>(&tri_hbm_panel_kernel), HT, 0));
  if (per_cu < 1) return fail(ctx, GW_EDEVICE, "tridiag_blocked: kernel does not fit a CU");
  const int G = std::min(n_cu, (n + 7) / 8);          // workgroups, one per CU
  if ((int64_t)G * HROWS < n) return fail(ctx, GW_EINVAL, "tridiag_blocked: order %d too large", n);
  const size_t ctr = (size_t)(1 + (G + kBarGroup - 1) / kBarGroup) * kCtrStride / 2;
  const size_t sc = 2 * (size_t)n * HB2 + (size_t)(HB + 1) * n + (size_t)G * HRED + ctr;
  double* ws = static_cast<double*>(ws_get(ctx, WS_TRI, sc * sizeof(double)));
  if (!ws) return GW_ENOMEM;
  double* VW = ws;
  double* WV = VW + (size_t)n * HB2;
  double* abuf = WV + (size_t)n * HB2;
  double* ybuf = abuf + (size_t)HB * n;
  double* red = ybuf + n;
  unsigned* count = reinterpret_cast<unsigned*>(red + (size_t)G * HRED);
  GW_TRY(fill_zero(ctx, reinterpret_cast<double*>(count), (int64_t)ctr));
  // Panels run up to the first panel boundary kend whose trailing block
  // (order n - kend) the on-chip reduction takes: per column it costs a few
  // microseconds of latency instead of a pass over the block in HBM plus two
  // device-wide exchanges (A = 7000: the last 3300 columns ~52 ms in panels).
  const int lim = tridiag_max_order(ctx);
  int kend = n - 1;
  if (lim >= 2 && n > lim) kend = (n - lim + HB - 1) / HB * HB;
  const int pt = prof_begin(ctx);
  unsigned pass0 = 0;
  for (int k0 = 0; k0 < kend; k0 += HB) {
    const int jb = std::min(HB, n - 1 - k0);
    HbmArgs a{job.K, n, k0, jb, k0 + jb == n - 1 ? 1 : 0, job.d, job.e, job.tau, VW, WV, abuf,
              ybuf, red, count, pass0, ctx->d_flags + 1, 1 << 21};
    void* args[] = {&a};
    GW_HIP(ctx, hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&tri_hbm_panel_kernel),
                                           dim3(G), dim3(HT), args, 0, ctx->stream));
    pass0 += 2u * (unsigned)jb;
    if (!a.last) {
      // A22 -= [V W] [W V]^T over the rows and columns past the panel
      const int ke = k0 + jb, m = n - ke;
      GW_TRY(dgemm_run(ctx, {DGemm{false, false, VW + (size_t)ke * HB2, WV + (size_t)ke * HB2,
                                   job.K + (size_t)ke * n + ke, m, m, HB2, HB2, HB2, n, -1.0,
                                   1.0}},
                       1, nullptr));
    }
  }
  if (kend < n - 1) {
    // The updated trailing block A(kend:, kend:) is an ordinary symmetric
    // matrix of order m: reduce it on chip (its d, e, tau land at offset
    // kend, its reflectors in its rows in the same convention), then put the
    // block with the reflectors back for the back-transformation.
    const int m = n - kend;
    double* Kc = static_cast<double*>(ws_get(ctx, WS_TRI_COPY, (size_t)m * m * sizeof(double)));
    if (!Kc) return GW_ENOMEM;
    double* blk = job.K + (size_t)kend * n + kend;
    GW_HIP(ctx, hipMemcpy2DAsync(Kc, (size_t)m * sizeof(double), blk, (size_t)n * sizeof(double),
                                 (size_t)m * sizeof(double), (size_t)m, hipMemcpyDeviceToDevice,
                                 ctx->stream));
    GW_TRY(tridiag_jobs(ctx, {TriIn{Kc, m, job.d + kend, job.e + kend, job.tau + kend}},
                        WS_TRI_SUB));
    GW_HIP(ctx, hipMemcpy2DAsync(blk, (size_t)n * sizeof(double), Kc, (size_t)m * sizeof(double),
                                 (size_t)m * sizeof(double), (size_t)m, hipMemcpyDeviceToDevice,
                                 ctx->stream));
  }
  prof_end(ctx, pt, "naf_tridiag", 0.0, 0.0);
  return GW_OK;
}

}  // namespace gw
