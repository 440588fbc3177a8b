// Natural auxiliary functions (Eqs. 11-13).
//
//  * Metric: K = s (R_oo^T R_oo + 2 R_ov^T R_ov), s = 2, with the virtual-
//    virtual block omitted (Sec. 2), on the scaled-SYRK kernels with a
//    constant scale.
//  * Eigendecomposition of K in FP64 on the device: Householder reduction to
//    tridiagonal form held on chip (tridiag.hip), then bisection, the
//    twisted factorisation (inverse iteration for clusters), one
//    Newton-Schulz step and the back-transformation of the kept eigenvectors
//    in blocks of reflectors (eig.hip); past the on-chip limit the reduction
//    runs in HBM by panels until the trailing block fits on chip
//    (tridiag.hip).  The kept
//    eigenvectors (eigenvalue > eps_NAF, at most max_keep) are copied in
//    descending order into U (row p = p-th eigenvector).
//  * Transform R~ = R U (Eq. 13): a GEMM with both operands contiguous along
//    the auxiliary index; FP32 MFMA with FP64 partial sums every 256 terms,
//    or FP64 MFMA.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"

namespace gw {
// Eigenpairs from the tridiagonal form (eig.hip): eigenvalues descending in
// ev, the kept eigenvectors of the original matrix in U's first rows.
gw_status naf_tri_solve(gw_ctx ctx, double* K, int n, const double* d_d, const double* d_e,
                        const double* d_tau, double eps_naf, int max_keep, double* U,
                        std::vector<double>& ev, int* keep_out, bool all_eigs);
// Synchronises; GW_EDEVICE if a tridiagonalisation barrier timed out.
gw_status check_tridiag(gw_ctx ctx);
gw_status gemm_f32_direct(gw_ctx ctx, const std::vector<NafGemmJob>& jobs, const char* prof);
}  // namespace gw

namespace {

constexpr int BM = 128;
constexpr int NT = 256;

inline int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  return (int)std::min<int64_t>(std::max<int64_t>(g, 1), 65536);
}

struct GemmArgs {
  const void* A;      // [rows][K]
  const double* B;    // [ncols][K] FP64
  void* C;            // [rows][ldc]; columns ncols .. ldc-1 are zeroed
  int64_t rows;
  int K;
  int ncols;
  int64_t ldc;
  int row_tiles, col_tiles;
};

constexpr int BK = 32;
constexpr int LDK = BK + 1;
constexpr int NT8 = 512;

// C[r][c] = sum_k A[r][k] B[c][k] on FP32 MFMA (32x32x2), FP64 running sums
// every 256 k.  8 waves of 32 x 64 per 128 x 128 tile; double-buffered LDS
// tiles stored k-contiguous ([row][k], padded), filled from registers loaded
// one stage ahead and consumed only at the LDS store, so the global reads
// stay in flight behind the MFMA block.  Rows past the end and k past K load
// as zeros (k is the contraction index, so the tail must be exact zeros).
__global__ __launch_bounds__(NT8, 2) void nt_gemm_f32_kernel(GemmArgs g0, Batch bt) {
  __shared__ float As[2][BM][LDK];
  __shared__ float Bs[2][BM][LDK];
  GemmArgs g;
  int64_t lid;
  if (!unit_of(g0, bt, g, lid)) return;
  const int ct = (int)(lid % g.col_tiles);
  const int rt = (int)(lid / g.col_tiles);
  const int64_t row0 = (int64_t)rt * BM;
  const int col0 = ct * BM;
  const float* A = static_cast<const float*>(g.A);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wy = wave >> 1, wx = wave & 1;            // rows wy*32, cols wx*64
  f32x16 acc[2];
  double acc64[2][16];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) { acc[j][r] = 0.f; acc64[j][r] = 0.0; }

  // A loader: rows (tid >> 3) + 64 h, k offset (tid & 7) * 4 (float4)
  // B loader: rows (tid >> 4) + 32 h, k offset (tid & 15) * 2 (double2)
  const bool vecA = (g.K % 4 == 0), vecB = (g.K % 2 == 0);
  float4 ra[2];
  double2 rb[4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t r = row0 + (tid >> 3) + 64 * h;
      const int k = k0 + (tid & 7) * 4;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (r < g.rows) {
        const float* p = A + r * g.K;
        if (vecA && k + 3 < g.K) {
          v = *reinterpret_cast<const float4*>(p + k);
        } else {
          if (k + 0 < g.K) v.x = p[k + 0];
          if (k + 1 < g.K) v.y = p[k + 1];
          if (k + 2 < g.K) v.z = p[k + 2];
          if (k + 3 < g.K) v.w = p[k + 3];
        }
      }
      ra[h] = v;
    }
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int c = col0 + (tid >> 4) + 32 * h;
      const int k = k0 + (tid & 15) * 2;
      double2 v = make_double2(0.0, 0.0);
      if (c < g.ncols) {
        const double* p = g.B + (int64_t)c * g.K;
        if (vecB && k + 1 < g.K) {
          v = *reinterpret_cast<const double2*>(p + k);
        } else {
          if (k + 0 < g.K) v.x = p[k + 0];
          if (k + 1 < g.K) v.y = p[k + 1];
        }
      }
      rb[h] = v;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = (tid >> 3) + 64 * h, k = (tid & 7) * 4;
      As[buf][r][k + 0] = ra[h].x;
      As[buf][r][k + 1] = ra[h].y;
      As[buf][r][k + 2] = ra[h].z;
      As[buf][r][k + 3] = ra[h].w;
    }
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int c = (tid >> 4) + 32 * h, k = (tid & 15) * 2;
      Bs[buf][c][k + 0] = (float)rb[h].x;
      Bs[buf][c][k + 1] = (float)rb[h].y;
    }
  };

  const int nk = (g.K + BK - 1) / BK;
  constexpr int FLUSH_STAGES = 256 / BK;
  gload(0);
  sstore(0);
  __syncthreads();
  const int arow = wy * 32 + (lane & 31);
  const int bcol = wx * 64 + (lane & 31);
  const int ksub = lane >> 5;
  for (int it = 0; it < nk; ++it) {
    const int cur = it & 1;
    if (it + 1 < nk) gload((it + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK / 2; ++kk) {
      const int kr = 2 * kk + ksub;
      const float a0 = As[cur][arow][kr];
      const float b0 = Bs[cur][bcol][kr];
      const float b1 = Bs[cur][bcol + 32][kr];
      acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[1], 0, 0, 0);
    }
    if (it + 1 < nk) sstore(cur ^ 1);
    if ((it + 1) % FLUSH_STAGES == 0 || it + 1 == nk) {
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          acc64[j][r] += (double)acc[j][r];
          acc[j][r] = 0.f;
        }
    }
    __syncthreads();
  }
  float* C = static_cast<float*>(g.C);
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t row = row0 + wy * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      const int col = col0 + wx * 64 + j * 32 + (lane & 31);
      if (row < g.rows && col < g.ldc)
        C[row * g.ldc + col] = col < g.ncols ? (float)acc64[j][r] : 0.f;
    }
}

// FP32 transform with both operands k-major: A^T = R^T ([K][ldat], a copy
// of the rows made by gw::transpose_f32) and B^T = U^T in FP32 ([K][ldbt],
// made by ut_kernel), so each 32 x 128 stage of either operand is 32 rows of
// memory copied global -> LDS by global_load_lds_dwordx4 (lane l of a wave
// fills bytes 16 l .. 16 l + 15: two 128-float rows per wave and
// instruction).  8 waves of 32 x 64 on v_mfma_f32_32x32x2f32, four waves
// per SIMD, FP64 running sums every 256 k; a per-k factor (1, or 0 past K)
// masks the clamped tail rows.
struct GemmDArgs {
  const float* AT;      // [K][ldat]
  int64_t ldat;         // multiple of 4, >= rows
  const float* BT;      // [K][ldbt]
  int ldbt;             // multiple of 4, >= ncols
  float* C;             // [rows][ldc]; columns ncols .. ldc-1 are zeroed
  int64_t rows;
  int K, ncols;
  int64_t ldc;
  int row_tiles, col_tiles;
};

constexpr int BKD = 32;

__global__ __launch_bounds__(NT8, 4) void nt_gemm_f32_direct_kernel(GemmDArgs g0, Batch bt) {
  __shared__ __attribute__((aligned(16))) float As[2][BKD][BM];
  __shared__ __attribute__((aligned(16))) float Bs[2][BKD][BM];
  __shared__ float Ss[2][BKD];
  GemmDArgs g;
  int64_t lid;
  if (!unit_of(g0, bt, g, lid)) return;
  const int ct = (int)(lid % g.col_tiles);
  const int rt = (int)(lid / g.col_tiles);
  const int64_t row0 = (int64_t)rt * BM;
  const int col0 = ct * BM;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wy = wave >> 1, wx = wave & 1;            // rows wy*32, cols wx*64
  const int nk = (g.K + BKD - 1) / BKD;
  const int lrow = 2 * wave + (lane >> 5);
  const int64_t ca = min(row0 + (int64_t)(lane & 31) * 4, g.ldat - 4);
  const int cb = min(col0 + (lane & 31) * 4, g.ldbt - 4);
  f32x16 acc[2];
  double acc64[2][16];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) { acc[j][r] = 0.f; acc64[j][r] = 0.0; }
  float sreg = 0.f;
  auto issue = [&](int kb, int buf) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int kr = min(kb + lrow + 16 * h, g.K - 1);
      __builtin_amdgcn_global_load_lds(g.AT + (int64_t)kr * g.ldat + ca,
                                       &As[buf][2 * wave + 16 * h][0], 16, 0, 0);
      __builtin_amdgcn_global_load_lds(g.BT + (int64_t)kr * g.ldbt + cb,
                                       &Bs[buf][2 * wave + 16 * h][0], 16, 0, 0);
    }
    if (tid < BKD) sreg = kb + tid < g.K ? 1.f : 0.f;
  };
  auto publish = [&](int buf) {
    if (tid < BKD) Ss[buf][tid] = sreg;
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  };
  constexpr int FLUSH_STAGES = 256 / BKD;
  issue(0, 0);
  publish(0);
  const int arow = wy * 32 + (lane & 31);
  const int bcol = wx * 64 + (lane & 31);
  const int ksub = lane >> 5;
  for (int it = 0; it < nk; ++it) {
    const int cur = it & 1;
    if (it + 1 < nk) issue((it + 1) * BKD, cur ^ 1);
    // operands of step kk + 1 read during the MFMAs of step kk (see the
    // chi SYRK for the scheduling hint)
    float na = As[cur][ksub][arow], ns = Ss[cur][ksub];
    float nb0 = Bs[cur][ksub][bcol], nb1 = Bs[cur][ksub][bcol + 32];
#pragma unroll
    for (int kk = 0; kk < BKD / 2; ++kk) {
      const float av = na * ns, b0 = nb0, b1 = nb1;
      if (kk + 1 < BKD / 2) {
        const int kr = 2 * (kk + 1) + ksub;
        na = As[cur][kr][arow];
        ns = Ss[cur][kr];
        nb0 = Bs[cur][kr][bcol];
        nb1 = Bs[cur][kr][bcol + 32];
      }
      acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, b0, acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, b1, acc[1], 0, 0, 0);
      __builtin_amdgcn_iglp_opt(0);
    }
    if ((it + 1) % FLUSH_STAGES == 0 || it + 1 == nk) {
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          acc64[j][r] += (double)acc[j][r];
          acc[j][r] = 0.f;
        }
    }
    publish(cur ^ 1);
  }
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t row = row0 + wy * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      const int col = col0 + wx * 64 + j * 32 + (lane & 31);
      if (row < g.rows && col < g.ldc)
        g.C[row * g.ldc + col] = col < g.ncols ? (float)acc64[j][r] : 0.f;
    }
}

// U^T in FP32: UT[k][c] = U[c][k] for c < ncols, zero for ncols <= c < ldbt.
struct UtArgs {
  const double* U;      // [>= ncols][K]
  int K, ncols, ldbt;
  float* UT;            // [K][ldbt]
};

__device__ __forceinline__ void ut_elem(const UtArgs& a, int64_t idx) {
  if (idx >= (int64_t)a.K * a.ldbt) return;
  const int k = (int)(idx / a.ldbt), c = (int)(idx % a.ldbt);
  a.UT[idx] = c < a.ncols ? (float)a.U[(int64_t)c * a.K + k] : 0.f;
}

__global__ void ut_batched_kernel(Batch bt) {
  UtArgs a;
  int64_t first;
  if (!block_of(bt, a, first)) return;
  for (int e = 0; e < kBatchElems; e += 256) ut_elem(a, first + e + threadIdx.x);
}

constexpr int BK64 = 16;
constexpr int LDK64 = BK64 + 2;

__global__ __launch_bounds__(NT, 1) void nt_gemm_f64_kernel(GemmArgs g0, Batch bt) {
  __shared__ double As[BM][LDK64];
  __shared__ double Bs[BM][LDK64];
  GemmArgs g;
  int64_t lid;
  if (!unit_of(g0, bt, g, lid)) return;
  const int ct = (int)(lid % g.col_tiles);
  const int rt = (int)(lid / g.col_tiles);
  const int64_t row0 = (int64_t)rt * BM;
  const int col0 = ct * BM;
  const double* A = static_cast<const double*>(g.A);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wy = wave >> 1, wx = wave & 1;
  f64x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int nk = (g.K + BK64 - 1) / BK64;
  for (int it = 0; it < nk; ++it) {
    const int k0 = it * BK64;
    // 128 rows x 16 k; thread: rows (tid >> 3) + 32 h, k (tid & 7) * 2
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int r = (tid >> 3) + 32 * h, k = k0 + (tid & 7) * 2;
      const int64_t ar = row0 + r;
      const int bc = col0 + r;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        As[r][(tid & 7) * 2 + e] = (ar < g.rows && k + e < g.K) ? A[ar * g.K + k + e] : 0.0;
        Bs[r][(tid & 7) * 2 + e] = (bc < g.ncols && k + e < g.K) ? g.B[(int64_t)bc * g.K + k + e] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK64 / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      double af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        af[i] = As[wy * 64 + i * 16 + (lane & 15)][kr];
        bf[i] = Bs[wx * 64 + i * 16 + (lane & 15)][kr];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  double* C = static_cast<double*>(g.C);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = row0 + wy * 64 + i * 16 + (lane >> 4) + 4 * r;
        const int col = col0 + wx * 64 + j * 16 + (lane & 15);
        if (row < g.rows && col < g.ldc) C[row * g.ldc + col] = col < g.ncols ? acc[i][j][r] : 0.0;
      }
}

}  // namespace


extern "C" gw_status gw_naf_compress(gw_ctx ctx, gw_precision prec, int n_aux,
                                     int64_t n_oo_rows, const void* R_oo, int64_t n_ov_rows,
                                     const void* R_ov, double* K, int accumulate, int finalize,
                                     double eps_naf, int max_keep, int* n_naf, double* U,
                                     double* eigvals) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_naf_compress: ctx is NULL");
  gw::clear_error(ctx);
  GW_REQUIRE(ctx, prec == GW_FP64 || prec == GW_FP32 || prec == GW_BF16X3,
             "gw_naf_compress: unknown precision %d", (int)prec);
  GW_REQUIRE(ctx, n_aux >= 1 && n_oo_rows >= 0 && n_ov_rows >= 0 && max_keep >= 0,
             "gw_naf_compress: bad sizes");
  GW_REQUIRE(ctx, K && (n_oo_rows == 0 || R_oo) && (n_ov_rows == 0 || R_ov),
             "gw_naf_compress: NULL argument");
  GW_REQUIRE(ctx, !finalize || (n_naf && U), "gw_naf_compress: finalize needs n_naf and U");
  if (finalize && ctx->capturing)
    return gw::fail(ctx, GW_EUNSUPPORTED,
                    "gw_naf_compress: the eigensolver synchronises and cannot be captured");
  GW_HIP(ctx, hipSetDevice(ctx->device));
  // FP32- and BF16x3-path tensors are stored in FP32: FP32 MFMA metric.
  const gw_precision mp = prec == GW_FP64 ? GW_FP64 : GW_FP32;
  if (n_oo_rows > 0)
    GW_TRY(gw::syrk_launch(ctx, mp, R_oo, n_oo_rows, n_aux, n_aux, 1, nullptr, 2.0, K, accumulate,
                           "naf_syrk"));
  if (n_ov_rows > 0)
    GW_TRY(gw::syrk_launch(ctx, mp, R_ov, n_ov_rows, n_aux, n_aux, 1, nullptr, 4.0, K,
                           accumulate || n_oo_rows > 0, "naf_syrk"));
  if (n_oo_rows == 0 && n_ov_rows == 0 && !accumulate)
    GW_TRY(gw::fill_zero(ctx, K, (int64_t)n_aux * n_aux));
  if (!finalize) return GW_OK;

  GW_TRY(gw::mirror_lower(ctx, K, 1, n_aux));
  double* ws = static_cast<double*>(gw::ws_get(ctx, WS_EIG, (3 * (size_t)n_aux + 8) * sizeof(double)));
  if (!ws) return GW_ENOMEM;
  double* d_eval = ws;
  double* d_e = ws + n_aux;
  double* d_tau = ws + 2 * n_aux;
  const int pe = gw::prof_begin(ctx);
  std::vector<double> ev(n_aux);
  int keep = 0;
  // reduction to tridiagonal form: held on chip up to the register limit,
  // in HBM by panels past it; then the eigenpairs of the tridiagonal matrix
  // and only the kept eigenvectors back-transformed
  const gw::TriIn tj{K, n_aux, d_eval, d_e, d_tau};
  if (n_aux <= gw::tridiag_max_order(ctx)) {
    const int pt = gw::prof_begin(ctx);
    GW_TRY(gw::tridiag_jobs(ctx, {tj}));
    gw::prof_end(ctx, pt, "naf_tridiag", 0.0, 0.0);
  } else {
    GW_TRY(gw::tridiag_blocked(ctx, tj));
  }
  GW_TRY(gw::check_tridiag(ctx));
  GW_TRY(gw::naf_tri_solve(ctx, K, n_aux, d_eval, d_e, d_tau, eps_naf, max_keep, U, ev, &keep,
                           eigvals != nullptr));
  gw::prof_end(ctx, pe, "naf_eig", 0.0, 0.0);
  *n_naf = keep;
  if (eigvals) std::copy(ev.begin(), ev.end(), eigvals);
  return GW_OK;
}

extern "C" gw_status gw_naf_apply(gw_ctx ctx, gw_precision prec, int n_aux, int n_naf,
                                  const double* U, int64_t n_rows, const void* R_in,
                                  void* R_out, int64_t ld_out) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_naf_apply: ctx is NULL");
  gw::clear_error(ctx);
  GW_REQUIRE(ctx, prec == GW_FP64 || prec == GW_FP32 || prec == GW_BF16X3,
             "gw_naf_apply: unknown precision %d", (int)prec);
  GW_REQUIRE(ctx, n_aux >= 1 && n_naf >= 1 && n_naf <= n_aux && n_rows >= 0,
             "gw_naf_apply: bad sizes (n_aux=%d n_naf=%d)", n_aux, n_naf);
  GW_REQUIRE(ctx, U && (n_rows == 0 || (R_in && R_out)), "gw_naf_apply: NULL argument");
  if (ld_out == 0) ld_out = n_naf;
  GW_REQUIRE(ctx, ld_out >= n_naf, "gw_naf_apply: ld_out < n_naf");
  if (n_rows == 0) return GW_OK;
  GW_HIP(ctx, hipSetDevice(ctx->device));
  if (prec != GW_FP64)
    return gw::gemm_f32_direct(ctx, {gw::NafGemmJob{R_in, U, R_out, n_rows, n_aux, n_naf, ld_out}},
                               "naf_gemm_f32");
  const int rt = (int)((n_rows + BM - 1) / BM), ct = (int)((ld_out + BM - 1) / BM);
  GemmArgs g{R_in, U, R_out, n_rows, n_aux, n_naf, ld_out, rt, ct};
  const int64_t grid = (int64_t)rt * ct;
  const int pi = gw::prof_begin(ctx);
  if (prec == GW_FP64)
    hipLaunchKernelGGL(nt_gemm_f64_kernel, dim3((unsigned)grid), dim3(NT), 0, ctx->stream, g,
                       Batch{});
  else
    hipLaunchKernelGGL(nt_gemm_f32_kernel, dim3((unsigned)grid), dim3(NT8), 0, ctx->stream, g,
                       Batch{});
  gw::prof_end(ctx, pi, prec == GW_FP64 ? "naf_gemm_f64" : "naf_gemm_f32",
               2.0 * (double)n_rows * n_aux * (double)n_naf, 0.0);
  return gw::launch_check(ctx, "naf transform");
}

namespace gw {

gw_status check_tridiag(gw_ctx ctx) {
  int f = 0;
  GW_HIP(ctx, hipMemcpyAsync(&f, ctx->d_flags + 1, sizeof f, hipMemcpyDeviceToHost, ctx->stream));
  GW_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (f != 0) {
    GW_HIP(ctx, hipMemsetAsync(ctx->d_flags + 1, 0, sizeof(int), ctx->stream));
    GW_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return fail(ctx, GW_EDEVICE, "tridiagonalisation: a workgroup barrier timed out");
  }
  return GW_OK;
}

// Eigendecompositions of several metrics.  K[d] (lower triangle) is read;
// U[d] receives the needed eigenvectors as rows, descending (at least those
// above eps_naf, up to max_keep); eig[d] (host, descending) the eigenvalues:
// all of them with all_eigs, else those above eps_naf and one below, the
// rest -inf.  Every metric is copied and mirrored; those within the on-chip
// limit are reduced to tridiagonal form together (packed cooperative
// launches), the larger ones one by one by panels in HBM with their
// trailing block on chip; then bisection, the twisted eigenvectors and the
// back-transformation per metric.  Synchronises.
gw_status naf_eig_batched(gw_ctx ctx, const std::vector<NafEigJob>& jobs) {
  if (jobs.empty()) return GW_OK;
  const int lim = tridiag_max_order(ctx);
  size_t k_tot = 0, v_tot = 0;
  int a_max = 0;
  for (const NafEigJob& j : jobs) {
    k_tot += (size_t)j.A * j.A;
    v_tot += (size_t)j.A;
    a_max = std::max(a_max, j.A);
  }
  double* Kt = static_cast<double*>(ws_get(ctx, WS_B_K, k_tot * sizeof(double)));
  double* dv = static_cast<double*>(ws_get(ctx, WS_B_EIG, (3 * v_tot + 8) * sizeof(double)));
  if (!Kt || !dv) return GW_ENOMEM;
  if (!ws_get(ctx, WS_EIG_Y, tri_solve_ws_elems(a_max) * sizeof(double))) return GW_ENOMEM;
  std::vector<TriIn> tri, small;
  std::vector<MirrorJob> mir;
  size_t ko = 0, vo = 0;
  for (const NafEigJob& j : jobs) {
    GW_HIP(ctx, hipMemcpyAsync(Kt + ko, j.K, (size_t)j.A * j.A * sizeof(double),
                               hipMemcpyDeviceToDevice, ctx->stream));
    mir.push_back(MirrorJob{Kt + ko, 1, j.A});
    tri.push_back(TriIn{Kt + ko, j.A, dv + vo, dv + v_tot + vo, dv + 2 * v_tot + vo});
    if (j.A <= lim) small.push_back(tri.back());
    ko += (size_t)j.A * j.A;
    vo += (size_t)j.A;
  }
  GW_TRY(mirror_lower_batched(ctx, mir));
  const int pe = prof_begin(ctx);
  if (!small.empty()) {
    const int pt = prof_begin(ctx);
    GW_TRY(tridiag_jobs(ctx, small));
    prof_end(ctx, pt, "naf_tridiag", 0.0, 0.0);
  }
  for (const TriIn& t : tri)
    if (t.n > lim) GW_TRY(tridiag_blocked(ctx, t));
  GW_TRY(check_tridiag(ctx));
  std::vector<double> ev;
  for (size_t d = 0; d < jobs.size(); ++d) {
    const NafEigJob& j = jobs[d];
    int keep = 0;
    GW_TRY(naf_tri_solve(ctx, tri[d].K, j.A, tri[d].d, tri[d].e, tri[d].tau, j.eps_naf,
                         j.max_keep, j.U, ev, &keep, j.all_eigs));
    std::copy(ev.begin(), ev.end(), j.eig);
  }
  prof_end(ctx, pe, "naf_eig", 0.0, 0.0);
  GW_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return GW_OK;
}

// FP32 transforms C = A U^T of several jobs through k-major copies of A and
// U (one transpose launch, one conversion launch, one GEMM launch).
gw_status gemm_f32_direct(gw_ctx ctx, const std::vector<NafGemmJob>& jobs, const char* prof) {
  auto r4 = [](int64_t x) { return std::max<int64_t>(4, (x + 3) / 4 * 4); };
  size_t tot = 0;
  for (const NafGemmJob& j : jobs)
    if (j.rows > 0) tot += (size_t)j.K * (r4(j.rows) + r4(j.ncols));
  if (tot == 0) return GW_OK;
  float* ws = static_cast<float*>(ws_get(ctx, WS_NAF_T, tot * sizeof(float)));
  if (!ws) return GW_ENOMEM;
  std::vector<TransposeJob> tr;
  std::vector<UtArgs> ut;
  std::vector<int64_t> ut_n;
  std::vector<GemmDArgs> d;
  std::vector<int64_t> off(1, 0);
  double flops = 0;
  size_t o = 0;
  for (const NafGemmJob& j : jobs) {
    if (j.rows == 0) continue;
    const int64_t ldat = r4(j.rows);
    const int ldbt = (int)r4(j.ncols);
    float* AT = ws + o;
    o += (size_t)j.K * ldat;
    float* BT = ws + o;
    o += (size_t)j.K * ldbt;
    tr.push_back(TransposeJob{static_cast<const float*>(j.A), j.rows, j.K, j.K, AT, ldat});
    ut.push_back(UtArgs{j.U, j.K, j.ncols, ldbt, BT});
    ut_n.push_back((int64_t)j.K * ldbt);
    const int rt = (int)((j.rows + BM - 1) / BM), ct = (int)((j.ldc + BM - 1) / BM);
    d.push_back(GemmDArgs{AT, ldat, BT, ldbt, static_cast<float*>(j.C), j.rows, j.K, j.ncols,
                          j.ldc, rt, ct});
    off.push_back(off.back() + (int64_t)rt * ct);
    flops += 2.0 * (double)j.rows * j.K * (double)j.ncols;
  }
  GW_TRY(transpose_f32(ctx, tr));
  GW_TRY(elementwise_batched(ctx, ut, ut_n, ut_batched_kernel, "ut_batched_kernel"));
  constexpr int CHUNK = 8;
  Batch bt;
  GW_TRY(stage_batch(ctx, d, off, CHUNK, bt));
  const int64_t grid = (off.back() + 8 * CHUNK - 1) / (8 * CHUNK) * (8 * CHUNK);
  const int pi = prof_begin(ctx);
  hipLaunchKernelGGL(nt_gemm_f32_direct_kernel, dim3((unsigned)grid), dim3(NT8), 0, ctx->stream,
                     GemmDArgs{}, bt);
  prof_end(ctx, pi, prof, flops, 0.0);
  return launch_check(ctx, "naf transform");
}

gw_status naf_gemm_batched(gw_ctx ctx, gw_precision prec, const std::vector<NafGemmJob>& jobs) {
  if (prec != GW_FP64) return gemm_f32_direct(ctx, jobs, "naf_gemm_f32");
  std::vector<GemmArgs> d;
  std::vector<int64_t> off(1, 0);
  double flops = 0;
  for (const NafGemmJob& j : jobs) {
    if (j.rows == 0) continue;
    const int rt = (int)((j.rows + BM - 1) / BM), ct = (int)((j.ldc + BM - 1) / BM);
    d.push_back(GemmArgs{j.A, j.U, j.C, j.rows, j.K, j.ncols, j.ldc, rt, ct});
    off.push_back(off.back() + (int64_t)rt * ct);
    flops += 2.0 * (double)j.rows * j.K * (double)j.ncols;
  }
  if (d.empty()) return GW_OK;
  constexpr int CHUNK = 8;
  Batch bt;
  GW_TRY(stage_batch(ctx, d, off, CHUNK, bt));
  const int64_t grid = (off.back() + 8 * CHUNK - 1) / (8 * CHUNK) * (8 * CHUNK);
  const int pi = prof_begin(ctx);
  if (prec == GW_FP64)
    hipLaunchKernelGGL(nt_gemm_f64_kernel, dim3((unsigned)grid), dim3(NT), 0, ctx->stream,
                       GemmArgs{}, bt);
  else
    hipLaunchKernelGGL(nt_gemm_f32_kernel, dim3((unsigned)grid), dim3(NT8), 0, ctx->stream,
                       GemmArgs{}, bt);
  prof_end(ctx, pi, prec == GW_FP64 ? "naf_gemm_f64" : "naf_gemm_f32", flops, 0.0);
  return launch_check(ctx, "batched naf transform");
}

}  // namespace gw

extern "C" gw_status gw_naf_compress_batched(gw_ctx ctx, gw_precision prec, int n_jobs,
                                             gw_naf_job* jobs) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_naf_compress_batched: ctx is NULL");
  gw::clear_error(ctx);
  if (ctx->capturing)
    return gw::fail(ctx, GW_EUNSUPPORTED,
                    "gw_naf_compress_batched: the eigensolver synchronises and cannot be captured");
  GW_REQUIRE(ctx, prec == GW_FP64 || prec == GW_FP32 || prec == GW_BF16X3,
             "gw_naf_compress_batched: unknown precision %d", (int)prec);
  GW_REQUIRE(ctx, n_jobs >= 0 && (n_jobs == 0 || jobs), "gw_naf_compress_batched: bad n_jobs");
  for (int d = 0; d < n_jobs; ++d) {
    const gw_naf_job& j = jobs[d];
    GW_REQUIRE(ctx, j.n_aux >= 1 && j.n_oo_rows >= 0 && j.n_ov_rows >= 0 && j.max_keep >= 0,
               "gw_naf_compress_batched: job %d: bad sizes", d);
    GW_REQUIRE(ctx, j.K && j.U && (j.n_oo_rows == 0 || j.R_oo) && (j.n_ov_rows == 0 || j.R_ov),
               "gw_naf_compress_batched: job %d: NULL argument", d);
  }
  if (n_jobs == 0) return GW_OK;
  GW_HIP(ctx, hipSetDevice(ctx->device));
  const gw_precision mp = prec == GW_FP64 ? GW_FP64 : GW_FP32;
  std::vector<gw::SyrkJob> oo, ov;
  for (int d = 0; d < n_jobs; ++d) {
    const gw_naf_job& j = jobs[d];
    oo.push_back(gw::SyrkJob{j.R_oo, j.n_oo_rows, j.n_aux, j.n_aux, 1, nullptr, 2.0, j.K, 0});
    ov.push_back(gw::SyrkJob{j.R_ov, j.n_ov_rows, j.n_aux, j.n_aux, 1, nullptr, 4.0, j.K, 1});
  }
  GW_TRY(gw::syrk_batched_launch(ctx, mp, oo, "naf_syrk"));
  GW_TRY(gw::syrk_batched_launch(ctx, mp, ov, "naf_syrk"));
  std::vector<std::vector<double>> ev(n_jobs);
  std::vector<gw::NafEigJob> ej;
  for (int d = 0; d < n_jobs; ++d) {
    ev[d].resize(jobs[d].n_aux);
    ej.push_back(gw::NafEigJob{jobs[d].K, jobs[d].n_aux, jobs[d].U, ev[d].data(),
                               jobs[d].eps_naf, jobs[d].max_keep, jobs[d].eigvals != nullptr});
  }
  GW_TRY(gw::naf_eig_batched(ctx, ej));
  for (int d = 0; d < n_jobs; ++d) {
    gw_naf_job& j = jobs[d];
    int keep = 0;
    for (int p = 0; p < j.n_aux; ++p) {
      if (ev[d][p] > j.eps_naf) ++keep; else break;
    }
    if (j.max_keep > 0) keep = std::min(keep, j.max_keep);
    j.n_naf = keep;
    if (j.eigvals) std::copy(ev[d].begin(), ev[d].end(), j.eigvals);
  }
  return GW_OK;
}

extern "C" gw_status gw_naf_apply_batched(gw_ctx ctx, gw_precision prec, int n_jobs,
                                          const gw_naf_apply_job* jobs) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_naf_apply_batched: ctx is NULL");
  gw::clear_error(ctx);
  GW_REQUIRE(ctx, prec == GW_FP64 || prec == GW_FP32 || prec == GW_BF16X3,
             "gw_naf_apply_batched: unknown precision %d", (int)prec);
  GW_REQUIRE(ctx, n_jobs >= 0 && (n_jobs == 0 || jobs), "gw_naf_apply_batched: bad n_jobs");
  std::vector<gw::NafGemmJob> gj;
  for (int d = 0; d < n_jobs; ++d) {
    const gw_naf_apply_job& j = jobs[d];
    GW_REQUIRE(ctx, j.n_aux >= 1 && j.n_naf >= 1 && j.n_naf <= j.n_aux && j.n_rows >= 0,
               "gw_naf_apply_batched: job %d: bad sizes", d);
    GW_REQUIRE(ctx, j.U && (j.n_rows == 0 || (j.R_in && j.R_out)),
               "gw_naf_apply_batched: job %d: NULL argument", d);
    const int64_t ld = j.ld_out ? j.ld_out : j.n_naf;
    GW_REQUIRE(ctx, ld >= j.n_naf, "gw_naf_apply_batched: job %d: ld_out < n_naf", d);
    gj.push_back(gw::NafGemmJob{j.R_in, j.U, j.R_out, j.n_rows, j.n_aux, j.n_naf, ld});
  }
  if (n_jobs == 0) return GW_OK;
  GW_HIP(ctx, hipSetDevice(ctx->device));
  return gw::naf_gemm_batched(ctx, prec, gj);
}
