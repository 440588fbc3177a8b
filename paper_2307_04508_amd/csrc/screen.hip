// Screening: Pi_j = -2 s sum_m exp(-w_j^2 x_m) M^m (Eq. 10), A_j = 1 - Pi_j,
// W^_j = A_j^-1 - 1 (Eq. 2), in FP64, batched over frequencies.
//
// The inverse uses the symmetric sweep (block Gauss-Jordan) form: for each
// pivot block K of 64 columns, with D = A_KK and the rest R,
//     A_RR <- A_RR - A_RK D^-1 A_KR,   A_RK <- A_RK D^-1,   A_KK <- -D^-1,
// which keeps every intermediate symmetric, so only the lower triangle is
// stored and updated; after the last block A holds -A^-1.  The pivots D are
// Schur complements of the symmetric positive definite 1 - Pi, so no pivoting
// is needed; a non-positive pivot raises the deferred GW_ENOTSPD flag.  The
// rank-64 update of each step runs on v_mfma_f64_16x16x4f64 and is the whole
// O(N^3) cost (N^3 flops per matrix with the triangle).
#include <algorithm>
#include <cmath>

#include "common.hpp"

namespace {

constexpr int B = 64;         // pivot block and update tile edge
constexpr int LDP = B + 2;    // LDS row stride (doubles) of panel tiles

inline int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  return (int)std::min<int64_t>(std::max<int64_t>(g, 1), 65536);
}

// A_j[p][q] = delta_pq + 2 s sum_m exp(-w_j^2 x_m) M^m[p][q], lower triangle.
__global__ void assemble_kernel(const double* __restrict__ M, int L, int N,
                                const double* __restrict__ x, const double* __restrict__ omega,
                                int F, double* __restrict__ A) {
  extern __shared__ double coef[];   // [F][L]
  for (int i = threadIdx.x; i < F * L; i += blockDim.x) {
    const int j = i / L, m = i % L;
    coef[i] = 4.0 * exp(-omega[j] * omega[j] * x[m]);   // 2 s, s = 2
  }
  __syncthreads();
  const int64_t NN = (int64_t)N * N;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < NN;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int p = (int)(idx / N), q = (int)(idx % N);
    if (q > p) continue;
    double mv[32];
    for (int m = 0; m < L; ++m) mv[m] = M[m * NN + idx];
    const double d = (p == q) ? 1.0 : 0.0;
    for (int j = 0; j < F; ++j) {
      double v = d;
      for (int m = 0; m < L; ++m) v += coef[j * L + m] * mv[m];
      A[j * NN + idx] = v;
    }
  }
}

// C[j][r][c] = A_j(r, kb + c) read from the lower triangle; zero for c >= bw.
__global__ void gather_panel_kernel(const double* __restrict__ A, int N, int F, int kb,
                                    int bw, double* __restrict__ C) {
  const int64_t NN = (int64_t)N * N;
  const int64_t total = (int64_t)F * N * B;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(idx % B);
    const int r = (int)((idx / B) % N);
    const int j = (int)(idx / ((int64_t)B * N));
    double v = 0.0;
    if (c < bw) {
      const int col = kb + c;
      v = (r >= col) ? A[j * NN + (int64_t)r * N + col] : A[j * NN + (int64_t)col * N + r];
    }
    C[idx] = v;
  }
}

// One workgroup per frequency sweeps the 64 x 64 pivot block, stored in
// registers: thread (tr, tc) owns rows 4 tr .. 4 tr + 3 and columns
// 4 tc .. 4 tc + 3.  Each step the owners of pivot column k and row k publish
// them through double-buffered LDS (one barrier per step).  A partial block
// (bw < 64) is padded with the identity, which the sweep leaves as -1 and
// does not couple to the valid part.  Stores D^-1 (zero-padded).
constexpr int PIV_THREADS = 256;
__global__ __launch_bounds__(PIV_THREADS) void pivot_kernel(const double* __restrict__ C, int N,
                                                            int kb, int bw,
                                                            double* __restrict__ Dinv,
                                                            int* __restrict__ flags, int j_offset) {
  __shared__ double colb[2][B], rowb[2][B];
  const int j = blockIdx.x;
  const double* Cj = C + (int64_t)j * N * B;
  const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
  double d[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int gr = 4 * tr + r, gc = 4 * tc + c;
      d[r][c] = (gr < bw && gc < bw) ? Cj[(int64_t)(kb + gr) * B + gc] : (gr == gc ? 1.0 : 0.0);
    }
  bool bad = false;
  for (int k4 = 0; k4 < B / 4; ++k4) {
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int k = 4 * k4 + kk, buf = k & 1;
      if (tc == k4) {
#pragma unroll
        for (int r = 0; r < 4; ++r) colb[buf][4 * tr + r] = d[r][kk];
      }
      if (tr == k4) {
#pragma unroll
        for (int c = 0; c < 4; ++c) rowb[buf][4 * tc + c] = d[kk][c];
      }
      __syncthreads();
      const double piv = colb[buf][k];
      bad = bad || !(piv > 0.0) || !isfinite(piv);
      const double inv = 1.0 / piv;
      double cr[4], rc[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        cr[e] = colb[buf][4 * tr + e];
        rc[e] = rowb[buf][4 * tc + e];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int gr = 4 * tr + r, gc = 4 * tc + c;
          double v;
          if (gr == k && gc == k) v = -inv;
          else if (gr == k) v = rc[c] * inv;
          else if (gc == k) v = cr[r] * inv;
          else v = d[r][c] - cr[r] * rc[c] * inv;
          d[r][c] = v;
        }
    }
  }
  // every thread sees the same pivots, so `bad` is uniform
  if (bad && threadIdx.x == 0) atomicCAS(flags, 0, j_offset + j + 1);
  double* out = Dinv + (int64_t)j * B * B;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int gr = 4 * tr + r, gc = 4 * tc + c;
      out[gr * B + gc] = (gr < bw && gc < bw && !bad) ? -d[r][c] : 0.0;   // d holds -D^-1
    }
}

// P[j][r][c] = sum_c' C[j][r][c'] Dinv[j][c'][c] for every row r.
__global__ __launch_bounds__(256) void panel_kernel(const double* __restrict__ C,
                                                    const double* __restrict__ Dinv, int N,
                                                    double* __restrict__ P) {
  __shared__ double Ds[B][B + 1];
  __shared__ double Cs[4][B];
  const int j = blockIdx.y;
  const double* Dj = Dinv + (int64_t)j * B * B;
  for (int i = threadIdx.x; i < B * B; i += blockDim.x) Ds[i / B][i % B] = Dj[i];
  const int rsub = threadIdx.x / B, c = threadIdx.x % B;
  for (int r0 = blockIdx.x * 4; r0 < N; r0 += gridDim.x * 4) {
    __syncthreads();
    const int r = r0 + rsub;
    Cs[rsub][c] = (r < N) ? C[((int64_t)j * N + r) * B + c] : 0.0;
    __syncthreads();
    if (r < N) {
      double v = 0.0;
#pragma unroll 8
      for (int k = 0; k < B; ++k) v += Cs[rsub][k] * Ds[k][c];
      P[((int64_t)j * N + r) * B + c] = v;
    }
  }
}

// A[I][J] -= P[I rows] C[J rows]^T for lower tiles I >= J, I, J != pivot tile.
__global__ __launch_bounds__(256) void update_kernel(double* __restrict__ A,
                                                     const double* __restrict__ P,
                                                     const double* __restrict__ C, int N,
                                                     int T, int kt) {
  __shared__ double Ps[B][LDP];
  __shared__ double Cs[B][LDP];
  const int n_tiles = T * (T + 1) / 2;
  const int64_t lid = xcd_remap(blockIdx.x, gridDim.x);
  const int j = (int)(lid / n_tiles);
  const int t = (int)(lid % n_tiles);
  int I = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  const int J = t - I * (I + 1) / 2;
  if (I == kt || J == kt) return;
  const double* Pj = P + (int64_t)j * N * B;
  const double* Cj = C + (int64_t)j * N * B;
  double* Aj = A + (int64_t)j * N * N;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wy = wave >> 1, wx = wave & 1;
  // Read this thread's part of the A tile first: its latency overlaps the
  // panel loads and the MFMA block.
  double av[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = I * B + wy * 32 + a * 16 + (lane >> 4) + 4 * r;
        const int col = J * B + wx * 32 + b * 16 + (lane & 15);
        av[a][b][r] = (row < N && col < N) ? Aj[(int64_t)row * N + col] : 0.0;
      }
  for (int i = tid; i < B * B / 2; i += 256) {
    const int r = i / (B / 2), c2 = (i % (B / 2)) * 2;
    const int gr = I * B + r, gc = J * B + r;
    double2 pv = make_double2(0.0, 0.0), cv = pv;
    if (gr < N) pv = *reinterpret_cast<const double2*>(Pj + (int64_t)gr * B + c2);
    if (gc < N) cv = *reinterpret_cast<const double2*>(Cj + (int64_t)gc * B + c2);
    *reinterpret_cast<double2*>(&Ps[r][c2]) = pv;
    *reinterpret_cast<double2*>(&Cs[r][c2]) = cv;
  }
  __syncthreads();
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int k = 0; k < B; k += 4) {
    const int kr = k + (lane >> 4);
    double af[2], bf[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      af[a] = Ps[wy * 32 + a * 16 + (lane & 15)][kr];
      bf[a] = Cs[wx * 32 + a * 16 + (lane & 15)][kr];
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = I * B + wy * 32 + a * 16 + (lane >> 4) + 4 * r;
        const int col = J * B + wx * 32 + b * 16 + (lane & 15);
        if (row < N && col < N) Aj[(int64_t)row * N + col] = av[a][b][r] - acc[a][b][r];
      }
}

// Pivot row / column after the update: A(r, K) <- P[r] for r outside K,
// A(K, K) <- -D^-1 (lower triangle storage).
__global__ void writeback_kernel(double* __restrict__ A, const double* __restrict__ P,
                                 const double* __restrict__ Dinv, int N, int F, int kb,
                                 int bw) {
  const int64_t NN = (int64_t)N * N;
  const int64_t total = (int64_t)F * N * B;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(idx % B);
    const int r = (int)((idx / B) % N);
    const int j = (int)(idx / ((int64_t)B * N));
    if (c >= bw) continue;
    const int col = kb + c;
    double* Aj = A + j * NN;
    if (r >= kb && r < kb + bw) {
      const int rr = r - kb;
      if (rr >= c) Aj[(int64_t)r * N + col] = -Dinv[((int64_t)j * B + rr) * B + c];
    } else {
      const double v = P[idx];
      if (r > col) Aj[(int64_t)r * N + col] = v;
      else Aj[(int64_t)col * N + r] = v;
    }
  }
}

// W^ = -S - 1 from the swept lower triangle S = -A^-1; both triangles.
template <typename T>
__global__ void finish_kernel(const double* __restrict__ S, int N, int F, T* __restrict__ W) {
  const int64_t NN = (int64_t)N * N;
  const int64_t total = (int64_t)F * NN;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = idx / NN, e = idx % NN;
    const int p = (int)(e / N), q = (int)(e % N);
    if (q > p) continue;
    const double v = -S[j * NN + e] - (p == q ? 1.0 : 0.0);
    W[j * NN + (int64_t)p * N + q] = (T)v;
    W[j * NN + (int64_t)q * N + p] = (T)v;
  }
}

}  // namespace

extern "C" gw_status gw_screen(gw_ctx ctx, gw_precision prec, int n_naf, int n_lt,
                               const double* x_lt, const double* M, int n_w,
                               const double* omega, void* W_hat) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_screen: ctx is NULL");
  gw::clear_error(ctx);
  GW_REQUIRE(ctx, prec == GW_FP64 || prec == GW_FP32 || prec == GW_BF16X3,
             "gw_screen: unknown precision %d", (int)prec);
  GW_REQUIRE(ctx, n_naf >= 1 && n_lt >= 1 && n_lt <= 32 && n_w >= 1 && n_w * n_lt <= 4096,
             "gw_screen: bad sizes (n_naf=%d n_lt=%d n_w=%d)", n_naf, n_lt, n_w);
  GW_REQUIRE(ctx, x_lt && M && omega && W_hat, "gw_screen: NULL argument");
  GW_HIP(ctx, hipSetDevice(ctx->device));
  const int N = n_naf, F = n_w;
  const int64_t NN = (int64_t)N * N;
  const double* dx = gw::stage_t(ctx, x_lt, n_lt);
  const double* dw = gw::stage_t(ctx, omega, n_w);
  if (!dx || !dw) return GW_EINVAL;
  double* A = nullptr;
  if (prec == GW_FP64) {
    A = static_cast<double*>(W_hat);
  } else {
    A = static_cast<double*>(gw::ws_get(ctx, WS_SCREEN_A, (size_t)F * NN * sizeof(double)));
    if (!A) return GW_ENOMEM;
  }
  const size_t panel = (size_t)F * N * B;
  double* pan = static_cast<double*>(
      gw::ws_get(ctx, WS_SCREEN_PANEL, (2 * panel + (size_t)F * B * B) * sizeof(double)));
  if (!pan) return GW_ENOMEM;
  double* C = pan;
  double* P = pan + panel;
  double* Dinv = pan + 2 * panel;

  const int pi = gw::prof_begin(ctx);
  hipLaunchKernelGGL(assemble_kernel, dim3(grid_for(NN, 256)), dim3(256),
                     (size_t)F * n_lt * sizeof(double), ctx->stream, M, n_lt, N, dx, dw, F, A);
  GW_TRY(gw::launch_check(ctx, "assemble_kernel"));
  const int T = (N + B - 1) / B;
  const int n_tiles = T * (T + 1) / 2;
  for (int kt = 0; kt < T; ++kt) {
    const int kb = kt * B, bw = std::min(B, N - kb);
    hipLaunchKernelGGL(gather_panel_kernel, dim3(grid_for((int64_t)F * N * B, 256)), dim3(256),
                       0, ctx->stream, A, N, F, kb, bw, C);
    hipLaunchKernelGGL(pivot_kernel, dim3(F), dim3(PIV_THREADS), 0, ctx->stream, C, N, kb, bw,
                       Dinv, ctx->d_flags, 0);
    hipLaunchKernelGGL(panel_kernel, dim3(std::min(1024, (N + 3) / 4), F), dim3(256), 0,
                       ctx->stream, C, Dinv, N, P);
    if (T > 1)
      hipLaunchKernelGGL(update_kernel, dim3((unsigned)((int64_t)F * n_tiles)), dim3(256), 0,
                         ctx->stream, A, P, C, N, T, kt);
    hipLaunchKernelGGL(writeback_kernel, dim3(grid_for((int64_t)F * N * B, 256)), dim3(256), 0,
                       ctx->stream, A, P, Dinv, N, F, kb, bw);
    GW_TRY(gw::launch_check(ctx, "screening sweep"));
  }
  gw::prof_end(ctx, pi, "screen_sweep", (double)F * N * (double)N * N,
               (double)F * N * (double)N * 8.0 * 2.0);
  if (prec == GW_FP64)
    hipLaunchKernelGGL(finish_kernel<double>, dim3(grid_for(F * NN, 256)), dim3(256), 0,
                       ctx->stream, A, N, F, static_cast<double*>(W_hat));
  else
    hipLaunchKernelGGL(finish_kernel<float>, dim3(grid_for(F * NN, 256)), dim3(256), 0,
                       ctx->stream, A, N, F, static_cast<float*>(W_hat));
  return gw::launch_check(ctx, "finish_kernel");
}
