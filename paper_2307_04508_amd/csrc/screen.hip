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
struct AsmArgs {
  const double* M;      // [L][N][N]
  int L, N;
  const double* x;      // [L]
  const double* omega;  // [F]
  int F;
  double* A;            // [F][N][N]
};

__device__ __forceinline__ void load_coef(const AsmArgs& a, double* coef) {
  for (int i = threadIdx.x; i < a.F * a.L; i += blockDim.x) {
    const int j = i / a.L, m = i % a.L;
    coef[i] = 4.0 * exp(-a.omega[j] * a.omega[j] * a.x[m]);   // 2 s, s = 2
  }
  __syncthreads();
}

__device__ __forceinline__ void assemble_elem(const AsmArgs& a, const double* coef, int64_t idx) {
  const int64_t NN = (int64_t)a.N * a.N;
  if (idx >= NN) return;
  const int p = (int)(idx / a.N), q = (int)(idx % a.N);
  if (q > p) return;
  double mv[32];
  for (int m = 0; m < a.L; ++m) mv[m] = a.M[m * NN + idx];
  const double d = (p == q) ? 1.0 : 0.0;
  for (int j = 0; j < a.F; ++j) {
    double v = d;
    for (int m = 0; m < a.L; ++m) v += coef[j * a.L + m] * mv[m];
    a.A[j * NN + idx] = v;
  }
}

__global__ void assemble_kernel(AsmArgs a) {
  extern __shared__ double coef[];   // [F][L]
  load_coef(a, coef);
  const int64_t NN = (int64_t)a.N * a.N;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < NN;
       idx += (int64_t)gridDim.x * blockDim.x)
    assemble_elem(a, coef, idx);
}

__global__ void assemble_batched_kernel(Batch bt) {
  extern __shared__ double coef[];
  AsmArgs a;
  int64_t first;
  if (!block_of(bt, a, first)) return;
  load_coef(a, coef);
  for (int e = 0; e < kBatchElems; e += 256) assemble_elem(a, coef, first + e + threadIdx.x);
}

// Arguments of one sweep step (pivot block kt, columns kb .. kb + bw - 1)
// for one batch of F matrices.
struct SwArgs {
  double* A;            // [F][N][N] lower triangle
  double* C;            // [F][N][B] pivot column panel
  double* P;            // [F][N][B] scaled panel
  double* Dinv;         // [F][B][B]
  int N, F, kb, bw, T, kt;
  int flag_base;        // flag value offset of this batch's first matrix
  int panel_blocks;     // batched panel kernel: workgroups per matrix
};

// C[j][r][c] = A_j(r, kb + c) read from the lower triangle; zero for c >= bw.
__device__ __forceinline__ void gather_elem(const SwArgs& a, int64_t idx) {
  const int64_t NN = (int64_t)a.N * a.N;
  if (idx >= (int64_t)a.F * a.N * B) return;
  const int c = (int)(idx % B);
  const int r = (int)((idx / B) % a.N);
  const int j = (int)(idx / ((int64_t)B * a.N));
  double v = 0.0;
  if (c < a.bw) {
    const int col = a.kb + c;
    v = (r >= col) ? a.A[j * NN + (int64_t)r * a.N + col] : a.A[j * NN + (int64_t)col * a.N + r];
  }
  a.C[idx] = v;
}

__global__ void gather_panel_kernel(SwArgs a) {
  const int64_t total = (int64_t)a.F * a.N * B;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x)
    gather_elem(a, idx);
}

__global__ void gather_panel_batched_kernel(Batch bt) {
  SwArgs a;
  int64_t first;
  if (!block_of(bt, a, first)) return;
  for (int e = 0; e < kBatchElems; e += 256) gather_elem(a, first + e + threadIdx.x);
}

// One workgroup per frequency sweeps the 64 x 64 pivot block, stored in
// registers: thread (tr, tc) owns rows 4 tr .. 4 tr + 3 and columns
// 4 tc .. 4 tc + 3.  Each step the owners of pivot column k and row k publish
// them through double-buffered LDS (one barrier per step).  A partial block
// (bw < 64) is padded with the identity, which the sweep leaves as -1 and
// does not couple to the valid part.  Stores D^-1 (zero-padded).
constexpr int PIV_THREADS = 256;
__device__ __forceinline__ void pivot_unit(const SwArgs& a, int j, int* __restrict__ flags) {
  __shared__ double colb[2][B], rowb[2][B];
  const int N = a.N, kb = a.kb, bw = a.bw;
  const double* Cj = a.C + (int64_t)j * N * B;
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
  if (bad && threadIdx.x == 0) atomicCAS(flags, 0, a.flag_base + j + 1);
  double* out = a.Dinv + (int64_t)j * B * B;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int gr = 4 * tr + r, gc = 4 * tc + c;
      out[gr * B + gc] = (gr < bw && gc < bw && !bad) ? -d[r][c] : 0.0;   // d holds -D^-1
    }
}

__global__ __launch_bounds__(PIV_THREADS) void pivot_kernel(SwArgs a, int* __restrict__ flags) {
  pivot_unit(a, blockIdx.x, flags);
}

__global__ __launch_bounds__(PIV_THREADS) void pivot_batched_kernel(Batch bt,
                                                                    int* __restrict__ flags) {
  const int d = find_problem(bt.off, bt.n, blockIdx.x);
  const SwArgs a = static_cast<const SwArgs*>(bt.descs)[d];
  pivot_unit(a, (int)(blockIdx.x - bt.off[d]), flags);
}

// P[j][r][c] = sum_c' C[j][r][c'] Dinv[j][c'][c] for every row r; this
// workgroup takes row groups blk, blk + nblk, ... of 4 rows.
__device__ __forceinline__ void panel_unit(const SwArgs& a, int j, int blk, int nblk) {
  __shared__ double Ds[B][B + 1];
  __shared__ double Cs[4][B];
  const int N = a.N;
  const double* Dj = a.Dinv + (int64_t)j * B * B;
  for (int i = threadIdx.x; i < B * B; i += blockDim.x) Ds[i / B][i % B] = Dj[i];
  const int rsub = threadIdx.x / B, c = threadIdx.x % B;
  for (int r0 = blk * 4; r0 < N; r0 += nblk * 4) {
    __syncthreads();
    const int r = r0 + rsub;
    Cs[rsub][c] = (r < N) ? a.C[((int64_t)j * N + r) * B + c] : 0.0;
    __syncthreads();
    if (r < N) {
      double v = 0.0;
#pragma unroll 8
      for (int k = 0; k < B; ++k) v += Cs[rsub][k] * Ds[k][c];
      a.P[((int64_t)j * N + r) * B + c] = v;
    }
  }
}

__global__ __launch_bounds__(256) void panel_kernel(SwArgs a) {
  panel_unit(a, blockIdx.y, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void panel_batched_kernel(Batch bt) {
  const int d = find_problem(bt.off, bt.n, blockIdx.x);
  const SwArgs a = static_cast<const SwArgs*>(bt.descs)[d];
  const int u = (int)(blockIdx.x - bt.off[d]);
  panel_unit(a, u / a.panel_blocks, u % a.panel_blocks, a.panel_blocks);
}

// A[I][J] -= P[I rows] C[J rows]^T for lower tiles I >= J, I, J != pivot tile.
__global__ __launch_bounds__(256) void update_kernel(SwArgs a0, Batch bt) {
  __shared__ double Ps[B][LDP];
  __shared__ double Cs[B][LDP];
  SwArgs sa;
  int64_t lid;
  if (!unit_of(a0, bt, sa, lid)) return;
  const int N = sa.N, T = sa.T, kt = sa.kt;
  double* __restrict__ A = sa.A;
  const double* __restrict__ P = sa.P;
  const double* __restrict__ C = sa.C;
  const int n_tiles = T * (T + 1) / 2;
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
__device__ __forceinline__ void writeback_elem(const SwArgs& a, int64_t idx) {
  const int64_t NN = (int64_t)a.N * a.N;
  if (idx >= (int64_t)a.F * a.N * B) return;
  const int c = (int)(idx % B);
  const int r = (int)((idx / B) % a.N);
  const int j = (int)(idx / ((int64_t)B * a.N));
  if (c >= a.bw) return;
  const int col = a.kb + c;
  double* Aj = a.A + j * NN;
  if (r >= a.kb && r < a.kb + a.bw) {
    const int rr = r - a.kb;
    if (rr >= c) Aj[(int64_t)r * a.N + col] = -a.Dinv[((int64_t)j * B + rr) * B + c];
  } else {
    const double v = a.P[idx];
    if (r > col) Aj[(int64_t)r * a.N + col] = v;
    else Aj[(int64_t)col * a.N + r] = v;
  }
}

__global__ void writeback_kernel(SwArgs a) {
  const int64_t total = (int64_t)a.F * a.N * B;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x)
    writeback_elem(a, idx);
}

__global__ void writeback_batched_kernel(Batch bt) {
  SwArgs a;
  int64_t first;
  if (!block_of(bt, a, first)) return;
  for (int e = 0; e < kBatchElems; e += 256) writeback_elem(a, first + e + threadIdx.x);
}

// W^ = -S - 1 from the swept lower triangle S = -A^-1; both triangles.
struct FinArgs {
  const double* S;      // [F][N][N]
  int N, F;
  void* W;              // [F][N][N] FP64 or FP32
};

template <typename T>
__device__ __forceinline__ void finish_elem(const FinArgs& a, int64_t idx) {
  const int64_t NN = (int64_t)a.N * a.N;
  if (idx >= (int64_t)a.F * NN) return;
  const int64_t j = idx / NN, e = idx % NN;
  const int p = (int)(e / a.N), q = (int)(e % a.N);
  if (q > p) return;
  const double v = -a.S[j * NN + e] - (p == q ? 1.0 : 0.0);
  T* W = static_cast<T*>(a.W);
  W[j * NN + (int64_t)p * a.N + q] = (T)v;
  W[j * NN + (int64_t)q * a.N + p] = (T)v;
}

template <typename T>
__global__ void finish_kernel(FinArgs a) {
  const int64_t total = (int64_t)a.F * a.N * a.N;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x)
    finish_elem<T>(a, idx);
}

template <typename T>
__global__ void finish_batched_kernel(Batch bt) {
  FinArgs a;
  int64_t first;
  if (!block_of(bt, a, first)) return;
  for (int e = 0; e < kBatchElems; e += 256) finish_elem<T>(a, first + e + threadIdx.x);
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
                     (size_t)F * n_lt * sizeof(double), ctx->stream,
                     AsmArgs{M, n_lt, N, dx, dw, F, A});
  GW_TRY(gw::launch_check(ctx, "assemble_kernel"));
  const int T = (N + B - 1) / B;
  const int n_tiles = T * (T + 1) / 2;
  for (int kt = 0; kt < T; ++kt) {
    const int kb = kt * B, bw = std::min(B, N - kb);
    const SwArgs sa{A, C, P, Dinv, N, F, kb, bw, T, kt, 0, 0};
    hipLaunchKernelGGL(gather_panel_kernel, dim3(grid_for((int64_t)F * N * B, 256)), dim3(256),
                       0, ctx->stream, sa);
    hipLaunchKernelGGL(pivot_kernel, dim3(F), dim3(PIV_THREADS), 0, ctx->stream, sa,
                       ctx->d_flags);
    hipLaunchKernelGGL(panel_kernel, dim3(std::min(1024, (N + 3) / 4), F), dim3(256), 0,
                       ctx->stream, sa);
    if (T > 1)
      hipLaunchKernelGGL(update_kernel, dim3((unsigned)((int64_t)F * n_tiles)), dim3(256), 0,
                         ctx->stream, sa, Batch{});
    hipLaunchKernelGGL(writeback_kernel, dim3(grid_for((int64_t)F * N * B, 256)), dim3(256), 0,
                       ctx->stream, sa);
    GW_TRY(gw::launch_check(ctx, "screening sweep"));
  }
  gw::prof_end(ctx, pi, "screen_sweep", (double)F * N * (double)N * N,
               (double)F * N * (double)N * 8.0 * 2.0);
  const FinArgs fa{A, N, F, W_hat};
  if (prec == GW_FP64)
    hipLaunchKernelGGL(finish_kernel<double>, dim3(grid_for(F * NN, 256)), dim3(256), 0,
                       ctx->stream, fa);
  else
    hipLaunchKernelGGL(finish_kernel<float>, dim3(grid_for(F * NN, 256)), dim3(256), 0,
                       ctx->stream, fa);
  return gw::launch_check(ctx, "finish_kernel");
}

extern "C" gw_status gw_screen_batched(gw_ctx ctx, gw_precision prec, int n_lt, int n_jobs,
                                       const gw_screen_job* jobs) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_screen_batched: ctx is NULL");
  gw::clear_error(ctx);
  GW_REQUIRE(ctx, prec == GW_FP64 || prec == GW_FP32 || prec == GW_BF16X3,
             "gw_screen_batched: unknown precision %d", (int)prec);
  GW_REQUIRE(ctx, n_lt >= 1 && n_lt <= 32 && n_jobs >= 0 && (n_jobs == 0 || jobs),
             "gw_screen_batched: bad sizes (n_lt=%d n_jobs=%d)", n_lt, n_jobs);
  for (int d = 0; d < n_jobs; ++d) {
    const gw_screen_job& j = jobs[d];
    GW_REQUIRE(ctx, j.n_naf >= 1 && j.n_w >= 1 && j.n_w * n_lt <= 4096,
               "gw_screen_batched: job %d: bad sizes (n_naf=%d n_w=%d)", d, j.n_naf, j.n_w);
    GW_REQUIRE(ctx, j.x_lt && j.M && j.omega && j.W_hat, "gw_screen_batched: job %d: NULL argument", d);
  }
  if (n_jobs == 0) return GW_OK;
  GW_HIP(ctx, hipSetDevice(ctx->device));

  // workspace: FP64 working matrices (in place for FP64), panels, pivots
  size_t a_tot = 0, p_tot = 0, d_tot = 0;
  for (int d = 0; d < n_jobs; ++d) {
    const size_t N = jobs[d].n_naf, F = jobs[d].n_w;
    if (prec != GW_FP64) a_tot += F * N * N;
    p_tot += F * N * B;
    d_tot += F * B * B;
  }
  double* Aws = nullptr;
  if (a_tot) {
    Aws = static_cast<double*>(gw::ws_get(ctx, WS_SCREEN_A, a_tot * sizeof(double)));
    if (!Aws) return GW_ENOMEM;
  }
  double* pan = static_cast<double*>(
      gw::ws_get(ctx, WS_SCREEN_PANEL, (2 * p_tot + d_tot) * sizeof(double)));
  if (!pan) return GW_ENOMEM;

  std::vector<AsmArgs> asm_d;
  std::vector<FinArgs> fin_d;
  std::vector<SwArgs> base;
  std::vector<int64_t> n_asm, n_fin;
  size_t ao = 0, po = 0, dof = 0;
  int flag_base = 0, T_max = 0, smem = 0;
  double flops = 0, bytes = 0;
  for (int d = 0; d < n_jobs; ++d) {
    const gw_screen_job& j = jobs[d];
    const int N = j.n_naf, F = j.n_w;
    const double* dx = gw::stage_t(ctx, j.x_lt, n_lt);
    const double* dw = gw::stage_t(ctx, j.omega, F);
    if (!dx || !dw) return GW_EINVAL;
    double* A = prec == GW_FP64 ? static_cast<double*>(j.W_hat) : Aws + ao;
    if (prec != GW_FP64) ao += (size_t)F * N * N;
    SwArgs sa{A, pan + po, pan + p_tot + po, pan + 2 * p_tot + dof, N, F, 0, 0,
              (N + B - 1) / B, 0, flag_base, std::min(1024, (N + 15) / 16)};
    po += (size_t)F * N * B;
    dof += (size_t)F * B * B;
    flag_base += F;
    T_max = std::max(T_max, sa.T);
    smem = std::max(smem, F * n_lt);
    base.push_back(sa);
    asm_d.push_back(AsmArgs{j.M, n_lt, N, dx, dw, F, A});
    n_asm.push_back((int64_t)N * N);
    fin_d.push_back(FinArgs{A, N, F, j.W_hat});
    n_fin.push_back((int64_t)F * N * N);
    flops += (double)F * N * (double)N * N;
    bytes += (double)F * N * (double)N * 8.0 * 2.0;
  }

  const int pi = gw::prof_begin(ctx);
  {
    std::vector<int64_t> off(1, 0);
    for (int64_t n : n_asm) off.push_back(off.back() + (n + kBatchElems - 1) / kBatchElems);
    Batch bt;
    GW_TRY(gw::stage_batch(ctx, asm_d, off, 1, bt));
    hipLaunchKernelGGL(assemble_batched_kernel, dim3((unsigned)off.back()), dim3(256),
                       (size_t)smem * sizeof(double), ctx->stream, bt);
    GW_TRY(gw::launch_check(ctx, "assemble_batched_kernel"));
  }
  for (int kt = 0; kt < T_max; ++kt) {
    std::vector<SwArgs> st;
    std::vector<int64_t> o_el(1, 0), o_piv(1, 0), o_pan(1, 0), o_upd(1, 0);
    for (const SwArgs& b0 : base) {
      if (kt >= b0.T) continue;
      SwArgs sa = b0;
      sa.kt = kt;
      sa.kb = kt * B;
      sa.bw = std::min(B, sa.N - sa.kb);
      st.push_back(sa);
      const int64_t el = (int64_t)sa.F * sa.N * B;
      o_el.push_back(o_el.back() + (el + kBatchElems - 1) / kBatchElems);
      o_piv.push_back(o_piv.back() + sa.F);
      o_pan.push_back(o_pan.back() + (int64_t)sa.F * sa.panel_blocks);
      o_upd.push_back(o_upd.back() + (int64_t)sa.F * sa.T * (sa.T + 1) / 2);
    }
    const SwArgs* dst = static_cast<const SwArgs*>(gw::stage(ctx, st.data(), st.size() * sizeof(SwArgs)));
    const int64_t* d_el = gw::stage_t(ctx, o_el.data(), o_el.size());
    const int64_t* d_piv = gw::stage_t(ctx, o_piv.data(), o_piv.size());
    const int64_t* d_pan = gw::stage_t(ctx, o_pan.data(), o_pan.size());
    const int64_t* d_upd = gw::stage_t(ctx, o_upd.data(), o_upd.size());
    if (!dst || !d_el || !d_piv || !d_pan || !d_upd) return GW_EINVAL;
    const int n = (int)st.size();
    constexpr int CHUNK = 8;
    const Batch b_el{dst, d_el, n, 1, o_el.back()};
    const Batch b_piv{dst, d_piv, n, 1, o_piv.back()};
    const Batch b_pan{dst, d_pan, n, 1, o_pan.back()};
    const Batch b_upd{dst, d_upd, n, CHUNK, o_upd.back()};
    hipLaunchKernelGGL(gather_panel_batched_kernel, dim3((unsigned)o_el.back()), dim3(256), 0,
                       ctx->stream, b_el);
    hipLaunchKernelGGL(pivot_batched_kernel, dim3((unsigned)o_piv.back()), dim3(PIV_THREADS), 0,
                       ctx->stream, b_piv, ctx->d_flags);
    hipLaunchKernelGGL(panel_batched_kernel, dim3((unsigned)o_pan.back()), dim3(256), 0,
                       ctx->stream, b_pan);
    const int64_t g_upd = (o_upd.back() + 8 * CHUNK - 1) / (8 * CHUNK) * (8 * CHUNK);
    hipLaunchKernelGGL(update_kernel, dim3((unsigned)g_upd), dim3(256), 0, ctx->stream,
                       SwArgs{}, b_upd);
    hipLaunchKernelGGL(writeback_batched_kernel, dim3((unsigned)o_el.back()), dim3(256), 0,
                       ctx->stream, b_el);
    GW_TRY(gw::launch_check(ctx, "batched screening sweep"));
  }
  gw::prof_end(ctx, pi, "screen_sweep", flops, bytes);
  return gw::elementwise_batched(ctx, fin_d, n_fin,
                                 prec == GW_FP64 ? finish_batched_kernel<double>
                                                 : finish_batched_kernel<float>,
                                 "finish_batched_kernel");
}

namespace gw {

void screen_ws_bytes(gw_precision prec, int N, int F, size_t* a_bytes, size_t* panel_bytes) {
  *a_bytes = prec == GW_FP64 ? 0 : (size_t)F * N * N * sizeof(double);
  *panel_bytes = (2 * (size_t)F * N * B + (size_t)F * B * B) * sizeof(double);
}

}  // namespace gw
