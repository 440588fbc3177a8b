// Diagonal self-energy: W_nm(i w_j) = R_nm^T W^_j R_nm (Eq. 2) on MFMA, then
// the imaginary-axis quadrature of Eq. 7 in FP64.
//
// The contraction is a GEMM Y = R_qp W^_j (rows: the Q*M pairs (n, m);
// columns: the auxiliary index) whose epilogue takes the row-wise dot
// product of each output tile with the matching columns of R_qp, so Y never
// reaches memory.  Because W^_j is symmetric, a column block J only needs
// the rows P >= J of W^ (off-diagonal blocks counted twice), which halves
// the work: rows * N (N + 1) flops per frequency.  Each 64-column slice of a
// tile writes one FP64 partial per row; a second kernel sums the partials
// in a fixed order.
//
//  FP32:   v_mfma_f32_32x32x2f32, operands FP32 and k-major (R~ transposed once
//          per call), copied global -> LDS directly; tile 128 x 128 x 32.
//  FP64:   v_mfma_f64_16x16x4f64, operands FP64, tile 128 x 128 x 16.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "bf16x3.hpp"
#include "common.hpp"

namespace {

constexpr int BM = 128;
constexpr int NT = 256;

inline int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  return (int)std::min<int64_t>(std::max<int64_t>(g, 1), 65536);
}

// Row stride of the k-major copy of the QP rows: a multiple of 4 floats.
inline int64_t rt_ld(int64_t rows) { return std::max<int64_t>(4, (rows + 3) / 4 * 4); }

struct BwbArgs {
  const void* R;      // [rows][ldr]
  const void* W;      // [F][N][N]
  int64_t rows;
  int N;
  int64_t ldr;
  int F;
  int row_tiles;
  int col_tiles;
  double* part;       // [F][2 * col_tiles][rows]
  const float* RT;    // FP32 k-major copy of R: [N][ldt] (bwb_f32_direct_kernel)
  int64_t ldt;        // multiple of 4, >= rows
};

// Work-unit order of the BF16x3 contraction: blocks of 8 frequencies
// outermost, then the column tile, then the row tile with the frequency of
// the block fastest.  The 32 units an XCD runs at once are then 4 row tiles
// x 8 frequencies of one column tile: per k step they read 4 slices of R
// and 8 of W^ (12 distinct slices per 32 units; row tile fastest gives 33),
// and every XCD's share of the launch spans all column tiles, whose k
// ranges differ.  (The FP32 and FP64 kernels keep the row tile fastest: the
// blocked order made the FP32 contraction at the large workload slower,
// 441 -> 500 ms.)
__device__ __forceinline__ void bwb_unit(int64_t lid, int row_tiles, int col_tiles, int F, int& j,
                                         int& ct, int& rt) {
  constexpr int JB = 8;
  const int64_t per_blk = (int64_t)row_tiles * col_tiles * JB;
  const int jblk = (int)(lid / per_blk);
  const int j0 = jblk * JB, jn = min(JB, F - j0);
  const int64_t rem = lid - (int64_t)jblk * per_blk;
  const int64_t per_ct = (int64_t)row_tiles * jn;
  ct = (int)(rem / per_ct);
  const int64_t in = rem - (int64_t)ct * per_ct;
  rt = (int)(in / jn);
  j = j0 + (int)(in - (int64_t)rt * jn);
}

__device__ __forceinline__ void decode(const BwbArgs& a, int64_t lid, int& j, int& ct, int& rt) {
  rt = (int)(lid % a.row_tiles);
  ct = (int)((lid / a.row_tiles) % a.col_tiles);
  j = (int)(lid / ((int64_t)a.row_tiles * a.col_tiles));
}

// ------------------------------------------------------------------ FP32
constexpr int BK32 = 32;

// FP32 with both operands k-major: A = R^T (a copy of R made by
// transpose_kernel, [N][ldt]) and B = W^_j ([N][N], rows are k), so each
// 32 x 128 stage of either operand is 32 rows of memory copied global -> LDS
// by global_load_lds (lane l of a wave fills bytes 16 l .. 16 l + 15, or
// 4 l .. 4 l + 3 when the rows of W^ are not 16-byte aligned): no loader
// registers, no transposing LDS stores.  8 waves of 32 x 64 on
// v_mfma_f32_32x32x2f32, four waves per SIMD.  The symmetric weighting of the
// k blocks (1 for the diagonal block, 2 below it, 0 past N) is a per-k
// factor on the A operand, kept in LDS next to the tiles.
constexpr int NTD = 512;

template <bool VEC>
__global__ __launch_bounds__(NTD, 4) void bwb_f32_direct_kernel(BwbArgs a0, Batch bt) {
  __shared__ __attribute__((aligned(16))) float As[2][BK32][BM];
  __shared__ __attribute__((aligned(16))) float Bs[2][BK32][BM];
  __shared__ float Ss[2][BK32];
  int j, ct, rt;
  BwbArgs a;
  int64_t lid;
  if (!unit_of(a0, bt, a, lid)) return;
  decode(a, lid, j, ct, rt);
  const int N = a.N;
  const float* RT = a.RT;
  const float* W = static_cast<const float*>(a.W) + (int64_t)j * N * N;
  const int64_t row0 = (int64_t)rt * BM;
  const int col0 = ct * BM;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wy = wave >> 1, wx = wave & 1;            // rows wy*32, cols wx*64
  const int kstart = col0;
  const int nk = (N - kstart + BK32 - 1) / BK32;
  const int kdiag = col0 + BM;                        // first k of the doubled blocks
  // loader: wave w fills stage rows 2w + (lane >> 5) and 16 + 2w + (lane >> 5)
  const int lrow = 2 * wave + (lane >> 5);
  const int64_t ca = min(row0 + (int64_t)(lane & 31) * 4, a.ldt - 4);
  const int cb = min(col0 + (lane & 31) * 4, N - 4);  // VEC: N >= 4

  f32x16 acc[2];
#pragma unroll
  for (int jj = 0; jj < 2; ++jj)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[jj][r] = 0.f;

  float sreg = 0.f;
  auto issue = [&](int kb, int buf) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int kr = min(kb + lrow + 16 * h, N - 1);
      __builtin_amdgcn_global_load_lds(RT + (int64_t)kr * a.ldt + ca,
                                       &As[buf][2 * wave + 16 * h][0], 16, 0, 0);
      if (VEC) {
        __builtin_amdgcn_global_load_lds(W + (int64_t)kr * N + cb, &Bs[buf][2 * wave + 16 * h][0],
                                         16, 0, 0);
      }
    }
    if (!VEC) {
      // 4-byte copies: one instruction fills 64 consecutive floats (half a row)
#pragma unroll
      for (int h = 0; h < 8; ++h) {
        const int q = wave + 8 * h;                   // 64 halves of 32 rows x 128 columns
        const int kr = min(kb + (q >> 1), N - 1);
        const int c = min(col0 + (q & 1) * 64 + lane, N - 1);
        __builtin_amdgcn_global_load_lds(W + (int64_t)kr * N + c, &Bs[buf][q >> 1][(q & 1) * 64],
                                         4, 0, 0);
      }
    }
    if (tid < BK32) {
      const int k = kb + tid;
      sreg = k < N ? (k < kdiag ? 1.f : 2.f) : 0.f;
    }
  };
  auto publish = [&](int buf) {
    if (tid < BK32) Ss[buf][tid] = sreg;
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  };

  issue(kstart, 0);
  publish(0);
  const int arow = wy * 32 + (lane & 31);
  const int bcol = wx * 64 + (lane & 31);
  const int ksub = lane >> 5;
  for (int it = 0; it < nk; ++it) {
    const int cur = it & 1;
    if (it + 1 < nk) issue(kstart + (it + 1) * BK32, cur ^ 1);
    // operands of step kk + 1 read during the MFMAs of step kk (see the
    // chi SYRK for the scheduling hint)
    float na = As[cur][ksub][arow], ns = Ss[cur][ksub];
    float nb0 = Bs[cur][ksub][bcol], nb1 = Bs[cur][ksub][bcol + 32];
#pragma unroll
    for (int kk = 0; kk < BK32 / 2; ++kk) {
      const float av = na * ns, b0 = nb0, b1 = nb1;
      if (kk + 1 < BK32 / 2) {
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
    publish(cur ^ 1);
  }

  // epilogue: per-row dot product with R[row][col] over this wave's 64 columns
  const float* R = static_cast<const float*>(a.R);
  double* part = a.part + ((int64_t)j * 2 * a.col_tiles + 2 * ct + wx) * a.rows;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t row = row0 + wy * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    double sum = 0.0;
    if (row < a.rows) {
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const int col = col0 + wx * 64 + jj * 32 + (lane & 31);
        if (col < N) sum += (double)acc[jj][r] * (double)R[row * a.ldr + col];
      }
    }
    sum = half_wave_sum(sum);
    if ((lane & 31) == 31 && row < a.rows) part[row] = sum;
  }
}

// ------------------------------------------------------- BF16x3, pre-split
// Both operands split once per call into workspace (bf16x3.hpp): the QP rows
// ([rows_pad][Npad]) and each W^_j ([Npad][Npad]), hi and lo, zero padded,
// stored in blocks of 32 k: block b holds [rows][32] of k 32 b .. 32 b + 31,
// so one pipeline stage of any tile is one contiguous range.  W^_j is
// symmetric, so row c of W^_j is column c along k, and both tiles are copied
// global -> LDS directly.  The symmetric
// weighting (1 for the diagonal block, 2 below it) scales the accumulators:
// after the diagonal block they are halved, at the end doubled (exact).
struct Split3Args {
  const float* src;     // [batch][rows][ld] with batch stride sstride
  int64_t rows, ld, sstride;
  int cols;
  __bf16* hi;           // [batch][cols_pad / 32][rows_pad][32]
  __bf16* lo;
  int64_t rows_pad, cols_pad;
  int batch;
};

__global__ __launch_bounds__(256) void split3_kernel(Split3Args a) {
  const int64_t per = a.rows_pad * a.cols_pad;
  const int64_t total = per * a.batch;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = i / per, e = i % per;
    const int64_t r = e / a.cols_pad;
    const int c = (int)(e % a.cols_pad);
    const float v = (r < a.rows && c < a.cols) ? a.src[b * a.sstride + r * a.ld + c] : 0.f;
    __bf16 h, l;
    b3::split(v, h, l);
    const int64_t o = b * per + (int64_t)(c >> 5) * (a.rows_pad * 32) + r * 32 + (c & 31);
    a.hi[o] = h;
    a.lo[o] = l;
  }
}

struct Bwb3Args {
  const __bf16* rh;     // [Npad / 32][rows_pad][32]
  const __bf16* rl;
  const __bf16* wh;     // [F][Npad / 32][Npad][32]
  const __bf16* wl;
  const float* R;       // FP32 rows for the row-dot epilogue, [rows][ldr]
  int64_t ldr;
  int64_t rows;
  int N, Npad, F, row_tiles, col_tiles;
  double* part;         // [F][2 * col_tiles][rows]
  int64_t rows_pad;
};

// NW = 4: waves of 64 rows x 64 columns; NW = 8: waves of 32 rows x 64
// columns (four waves per SIMD with two workgroups per CU).  Either way a
// wave's columns are one 64-column slice, so each row's slice partial comes
// from one wave.
template <int NW>
__global__ __launch_bounds__(NW * 64, 2) void bwb_bf16x3_direct_kernel(Bwb3Args a) {
  constexpr int WI = NW == 4 ? 2 : 1, WJ = 2;
  __shared__ __attribute__((aligned(16))) b3::Stage st[2];
  const int64_t lid = xcd_remap(blockIdx.x, gridDim.x);
  int j, ct, rt;
  bwb_unit(lid, a.row_tiles, a.col_tiles, a.F, j, ct, rt);
  const int64_t row0 = (int64_t)rt * BM;
  const int col0 = ct * BM;
  const __bf16* wh = a.wh + (int64_t)j * a.Npad * a.Npad;
  const __bf16* wl = a.wl + (int64_t)j * a.Npad * a.Npad;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wx = wave & 1;
  const int ar = (wave >> 1) * (WI * 32);          // first tile row of the wave
  const int br = wx * 64;                          // first tile column

  f32x16 acc[WI][WJ];
#pragma unroll
  for (int i = 0; i < WI; ++i)
#pragma unroll
    for (int jj = 0; jj < WJ; ++jj)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][jj][r] = 0.f;

  static_assert(b3::BK == 32, "one stage is one k block of the split layout");
  auto issue = [&](int64_t kb, int buf) {   // kb: a multiple of 32
    b3::load_tile<b3::BK, NW>(a.rh + kb * a.rows_pad, b3::BK, row0, 0, st[buf].t[0], wave, lane);
    b3::load_tile<b3::BK, NW>(a.rl + kb * a.rows_pad, b3::BK, row0, 0, st[buf].t[1], wave, lane);
    b3::load_tile<b3::BK, NW>(wh + kb * a.Npad, b3::BK, col0, 0, st[buf].t[2], wave, lane);
    b3::load_tile<b3::BK, NW>(wl + kb * a.Npad, b3::BK, col0, 0, st[buf].t[3], wave, lane);
  };
  auto publish = [&]() {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  };
  const int kstart = col0;
  const int nk = (a.Npad - kstart) / b3::BK;
  constexpr int DIAG_STAGES = BM / b3::BK;
  issue(kstart, 0);
  publish();
  for (int it = 0; it < nk; ++it) {
    const int cur = it & 1;
    if (it + 1 < nk) issue(kstart + (int64_t)(it + 1) * b3::BK, cur ^ 1);
    b3::stage_mfma<b3::BK, WI, WJ>(st[cur], acc, ar, br, lane);
    if (it + 1 == DIAG_STAGES && nk > DIAG_STAGES) {
#pragma unroll
      for (int i = 0; i < WI; ++i)
#pragma unroll
        for (int jj = 0; jj < WJ; ++jj) acc[i][jj] *= 0.5f;
    }
    publish();
  }
  if (nk > DIAG_STAGES) {
#pragma unroll
    for (int i = 0; i < WI; ++i)
#pragma unroll
      for (int jj = 0; jj < WJ; ++jj) acc[i][jj] *= 2.0f;
  }

  // epilogue: per-row dot product with R over this wave's 64 columns
  double* part = a.part + ((int64_t)j * 2 * a.col_tiles + 2 * ct + wx) * a.rows;
#pragma unroll
  for (int i = 0; i < WI; ++i) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t row = row0 + ar + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      double sum = 0.0;
      if (row < a.rows) {
#pragma unroll
        for (int jj = 0; jj < WJ; ++jj) {
          const int col = col0 + br + jj * 32 + (lane & 31);
          if (col < a.N) sum += (double)acc[i][jj][r] * (double)a.R[row * a.ldr + col];
        }
      }
      // lanes 0-31 and 32-63 hold different rows: sum within each half
      sum = half_wave_sum(sum);
      if ((lane & 31) == 31 && row < a.rows) part[row] = sum;
    }
  }
}

// ------------------------------------------------------------------ FP64
constexpr int BK64 = 16;
constexpr int LDA64 = BK64 + 2;

__global__ __launch_bounds__(NT, 1) void bwb_f64_kernel(BwbArgs a0, Batch bt) {
  __shared__ double As[2][BM][LDA64];
  __shared__ double Bs[2][BK64][BM];
  int j, ct, rt;
  BwbArgs a;
  int64_t lid;
  if (!unit_of(a0, bt, a, lid)) return;
  decode(a, lid, j, ct, rt);
  const double* R = static_cast<const double*>(a.R);
  const double* W = static_cast<const double*>(a.W) + (int64_t)j * a.N * a.N;
  const int64_t row0 = (int64_t)rt * BM;
  const int col0 = ct * BM;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wy = wave >> 1, wx = wave & 1;

  f64x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) acc[i][jj] = f64x4{0.0, 0.0, 0.0, 0.0};

  // A loader: 128 rows x 16 doubles = 1024 double2 -> 4 per thread:
  //   rows (tid >> 3) + 32 h, k offset (tid & 7) * 2
  // B loader: 16 rows x 128 doubles = 1024 double2 -> 4 per thread:
  //   rows (tid >> 6) + 4 h, col offset (tid & 63) * 2
  double2 ra[4], rb[4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int64_t row = row0 + (tid >> 3) + 32 * h;
      const int k = k0 + (tid & 7) * 2;
      double2 v = make_double2(0.0, 0.0);
      if (row < a.rows) {
        const int64_t off = row * a.ldr + k;
        const double* p = R + off;
        if (k + 1 < a.N && (off & 1) == 0) v = *reinterpret_cast<const double2*>(p);
        else {
          if (k < a.N) v.x = p[0];
          if (k + 1 < a.N) v.y = p[1];
        }
      }
      ra[h] = v;
      const int kr = k0 + (tid >> 6) + 4 * h;
      const int c = col0 + (tid & 63) * 2;
      double2 u = make_double2(0.0, 0.0);
      if (kr < a.N) {
        const int64_t off = (int64_t)kr * a.N + c;
        const double* p = W + off;
        if (c + 1 < a.N && (off & 1) == 0) u = *reinterpret_cast<const double2*>(p);
        else {
          if (c < a.N) u.x = p[0];
          if (c + 1 < a.N) u.y = p[1];
        }
      }
      rb[h] = u;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      *reinterpret_cast<double2*>(&As[buf][(tid >> 3) + 32 * h][(tid & 7) * 2]) = ra[h];
      *reinterpret_cast<double2*>(&Bs[buf][(tid >> 6) + 4 * h][(tid & 63) * 2]) = rb[h];
    }
  };

  // symmetric W^: rows P >= col0 only (see the FP32 kernel)
  const int kstart = col0;
  const int nk = (a.N - kstart + BK64 - 1) / BK64;
  constexpr int DIAG_STAGES = BM / BK64;
  gload(kstart);
  sstore(0);
  __syncthreads();
  for (int it = 0; it < nk; ++it) {
    const int cur = it & 1;
    if (it + 1 < nk) gload(kstart + (it + 1) * BK64);
#pragma unroll
    for (int kk = 0; kk < BK64 / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      double af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        af[i] = As[cur][wy * 64 + i * 16 + (lane & 15)][kr];
        bf[i] = Bs[cur][kr][wx * 64 + i * 16 + (lane & 15)];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
          acc[i][jj] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[jj], acc[i][jj], 0, 0, 0);
    }
    if (it + 1 == DIAG_STAGES && nk > DIAG_STAGES) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) acc[i][jj] *= 0.5;
    }
    if (it + 1 < nk) sstore(cur ^ 1);
    __syncthreads();
  }
  if (nk > DIAG_STAGES) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) acc[i][jj] *= 2.0;
  }

  double* part = a.part + ((int64_t)j * 2 * a.col_tiles + 2 * ct + wx) * a.rows;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int lrow = wy * 64 + i * 16 + (lane >> 4) + 4 * r;
      const int64_t row = row0 + lrow;
      double s = 0.0;
      if (row < a.rows) {
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int col = col0 + wx * 64 + jj * 16 + (lane & 15);
          if (col < a.N) s += acc[i][jj][r] * R[row * a.ldr + col];
        }
      }
      s = row16_sum(s);
      if ((lane & 15) == 0 && row < a.rows) part[row] = s;
    }
  }
}

// ------------------------------------------------------------------ BF16x3
// Same contraction as hi*hi + hi*lo + lo*hi BF16 MFMA products
// (v_mfma_f32_32x32x16_bf16), FP32 accumulation.  W^_j is symmetric, so the
// B operand W^[p][q] is read as row q of W^ (contiguous along p = k) and
// both tiles stage into k-contiguous LDS rows without a transpose; the split
// into hi/lo happens in the LDS store.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
constexpr int BKB = 32;
// k stride (bf16) of an LDS row: unpadded, with the 16-byte k-chunks of a row
// XOR-swizzled by the row so the 16-byte operand reads of 32 consecutive rows
// stay conflict-free (64 KB of tiles: two workgroups per CU)
constexpr int LDB = BKB;
__device__ __forceinline__ int swz(int row, int k) {
  return (((k >> 3) ^ ((row >> 2) & 3)) << 3) | (k & 7);
}

__device__ __forceinline__ void split4(const float4 v, bf16x4& hi, bf16x4& lo) {
  const float x[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const __bf16 h = (__bf16)x[e];
    hi[e] = h;
    lo[e] = (__bf16)(x[e] - (float)h);
  }
}

__device__ __forceinline__ float4 load4_guarded(const float* base, int64_t off, int k, int n) {
  const float* p = base + off;
  if (k + 3 < n && (off & 3) == 0) return *reinterpret_cast<const float4*>(p);
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (k + 0 < n) v.x = p[0];
  if (k + 1 < n) v.y = p[1];
  if (k + 2 < n) v.z = p[2];
  if (k + 3 < n) v.w = p[3];
  return v;
}

__global__ __launch_bounds__(NT, 2) void bwb_bf16x3_kernel(BwbArgs a0, Batch bt) {
  __shared__ __attribute__((aligned(16))) __bf16 Ah[2][BM][LDB];
  __shared__ __attribute__((aligned(16))) __bf16 Al[2][BM][LDB];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[2][BM][LDB];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[2][BM][LDB];
  int j, ct, rt;
  BwbArgs a;
  int64_t lid;
  if (!unit_of(a0, bt, a, lid)) return;
  decode(a, lid, j, ct, rt);
  const float* R = static_cast<const float*>(a.R);
  const float* W = static_cast<const float*>(a.W) + (int64_t)j * a.N * a.N;
  const int64_t row0 = (int64_t)rt * BM;
  const int col0 = ct * BM;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wy = wave >> 1, wx = wave & 1;

  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][jj][r] = 0.f;

  // loader: rows (tid >> 3) + 32 h, k offset (tid & 7) * 4, for both tiles
  float4 ra[4], rb[4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int lr = (tid >> 3) + 32 * h;
      const int k = k0 + (tid & 7) * 4;
      const int64_t row = row0 + lr;
      ra[h] = row < a.rows ? load4_guarded(R, row * a.ldr + k, k, a.N)
                           : make_float4(0.f, 0.f, 0.f, 0.f);
      const int q = col0 + lr;
      rb[h] = q < a.N ? load4_guarded(W, (int64_t)q * a.N + k, k, a.N)
                      : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int lr = (tid >> 3) + 32 * h, kk = swz(lr, (tid & 7) * 4);
      bf16x4 hi, lo;
      split4(ra[h], hi, lo);
      *reinterpret_cast<bf16x4*>(&Ah[buf][lr][kk]) = hi;
      *reinterpret_cast<bf16x4*>(&Al[buf][lr][kk]) = lo;
      split4(rb[h], hi, lo);
      *reinterpret_cast<bf16x4*>(&Bh[buf][lr][kk]) = hi;
      *reinterpret_cast<bf16x4*>(&Bl[buf][lr][kk]) = lo;
    }
  };

  // symmetric W^: rows P >= col0 only (see the FP32 kernel)
  const int kstart = col0;
  const int nk = (a.N - kstart + BKB - 1) / BKB;
  constexpr int DIAG_STAGES = BM / BKB;
  gload(kstart);
  sstore(0);
  __syncthreads();
  const int kl = 8 * (lane >> 5);
  for (int it = 0; it < nk; ++it) {
    const int cur = it & 1;
    if (it + 1 < nk) gload(kstart + (it + 1) * BKB);
#pragma unroll
    for (int ks = 0; ks < BKB; ks += 16) {
      bf16x8 ahf[2], alf[2], bhf[2], blf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int pr = wy * 64 + i * 32 + (lane & 31);
        const int qc = wx * 64 + i * 32 + (lane & 31);
        const int kp = swz(pr, ks + kl), kq = swz(qc, ks + kl);
        ahf[i] = *reinterpret_cast<const bf16x8*>(&Ah[cur][pr][kp]);
        alf[i] = *reinterpret_cast<const bf16x8*>(&Al[cur][pr][kp]);
        bhf[i] = *reinterpret_cast<const bf16x8*>(&Bh[cur][qc][kq]);
        blf[i] = *reinterpret_cast<const bf16x8*>(&Bl[cur][qc][kq]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
          acc[i][jj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahf[i], bhf[jj], acc[i][jj], 0, 0, 0);
          acc[i][jj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahf[i], blf[jj], acc[i][jj], 0, 0, 0);
          acc[i][jj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alf[i], bhf[jj], acc[i][jj], 0, 0, 0);
        }
    }
    if (it + 1 == DIAG_STAGES && nk > DIAG_STAGES) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) acc[i][jj] *= 0.5f;
    }
    if (it + 1 < nk) sstore(cur ^ 1);
    __syncthreads();
  }
  if (nk > DIAG_STAGES) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) acc[i][jj] *= 2.0f;
  }

  double* part = a.part + ((int64_t)j * 2 * a.col_tiles + 2 * ct + wx) * a.rows;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int lrow = wy * 64 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      const int64_t row = row0 + lrow;
      double sum = 0.0;
      if (row < a.rows) {
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
          const int col = col0 + wx * 64 + jj * 32 + (lane & 31);
          if (col < a.N) sum += (double)acc[i][jj][r] * (double)R[row * a.ldr + col];
        }
      }
      sum = half_wave_sum(sum);
      if ((lane & 31) == 31 && row < a.rows) part[row] = sum;
    }
  }
}

// W[j][row] = sum over column partials (fixed order); optional user copy.
struct WRedArgs {
  const double* part;   // [F][n_part][rows]
  int n_part;
  int64_t rows;
  int F;
  double* W;            // [F][rows]
  double* W_user;       // optional copy
};

__device__ __forceinline__ void w_reduce_elem(const WRedArgs& a, int64_t idx) {
  if (idx >= (int64_t)a.F * a.rows) return;
  const int64_t j = idx / a.rows, r = idx % a.rows;
  double v = 0.0;
  for (int p = 0; p < a.n_part; ++p) v += a.part[(j * a.n_part + p) * a.rows + r];
  a.W[idx] = v;
  if (a.W_user) a.W_user[idx] = v;
}

__global__ void w_reduce_kernel(WRedArgs a) {
  const int64_t total = (int64_t)a.F * a.rows;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x)
    w_reduce_elem(a, idx);
}

__global__ void w_reduce_batched_kernel(Batch bt) {
  WRedArgs a;
  int64_t first;
  if (!block_of(bt, a, first)) return;
  for (int e = 0; e < kBatchElems; e += 256) w_reduce_elem(a, first + e + threadIdx.x);
}

// One workgroup per (QP state q, Pade node k):
//   Sigma = -(1/pi) sum_j w_j sum_m a / (a^2 + w_j^2) W[j][q][m],
//   a = i wp_k + e_F - e_m.
struct QuadArgs {
  const double* W;      // [F][Q][M]
  int F, Q, M;
  const double* eps_m;  // [M]
  double eps_f;
  const double* omega;
  const double* w_omega;
  const double* omega_p;
  int Pd;
  int accumulate;
  double* sigma;        // [Q][Pd][2]
};

__device__ __forceinline__ void sigma_quad_unit(const QuadArgs& a, int unit) {
  __shared__ double sre[256], sim[256];
  const int q = unit / a.Pd, k = unit % a.Pd;
  const double wk = a.omega_p[k];
  double re = 0.0, im = 0.0;
  for (int idx = threadIdx.x; idx < a.F * a.M; idx += blockDim.x) {
    const int j = idx / a.M, m = idx % a.M;
    const double ar = a.eps_f - a.eps_m[m], ai = wk;      // a = ar + i ai
    const double wj = a.omega[j];
    // a^2 + w_j^2 = (ar^2 - ai^2 + wj^2) + i (2 ar ai)
    const double dr = ar * ar - ai * ai + wj * wj, di = 2.0 * ar * ai;
    const double den = dr * dr + di * di;
    const double gr = (ar * dr + ai * di) / den, gi = (ai * dr - ar * di) / den;
    const double f = a.w_omega[j] * a.W[((int64_t)j * a.Q + q) * a.M + m];
    re += f * gr;
    im += f * gi;
  }
  sre[threadIdx.x] = re;
  sim[threadIdx.x] = im;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sre[threadIdx.x] += sre[threadIdx.x + s];
      sim[threadIdx.x] += sim[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double c = -1.0 / 3.14159265358979323846;
    double* out = a.sigma + 2 * ((int64_t)q * a.Pd + k);
    if (a.accumulate) {
      out[0] += c * sre[0];
      out[1] += c * sim[0];
    } else {
      out[0] = c * sre[0];
      out[1] = c * sim[0];
    }
  }
}

__global__ __launch_bounds__(256) void sigma_quad_kernel(QuadArgs a) {
  sigma_quad_unit(a, blockIdx.x);
}

__global__ __launch_bounds__(256) void sigma_quad_batched_kernel(Batch bt) {
  const int d = find_problem(bt.off, bt.n, blockIdx.x);
  const QuadArgs a = static_cast<const QuadArgs*>(bt.descs)[d];
  sigma_quad_unit(a, (int)(blockIdx.x - bt.off[d]));
}

// FP32: rows of W^_j 16-byte aligned (N % 4 == 0, aligned base) take the
// vector copies of bwb_f32_direct_kernel, other N its 4-byte copies.
bool w_rows_aligned(const void* W, int N) {
  return N >= 4 && N % 4 == 0 && reinterpret_cast<uintptr_t>(W) % 16 == 0;
}

void launch_bwb(gw_ctx ctx, gw_precision prec, const BwbArgs& a, const Batch& bt,
                int64_t grid, bool vec) {
  if (prec == GW_FP64)
    hipLaunchKernelGGL(bwb_f64_kernel, dim3((unsigned)grid), dim3(NT), 0, ctx->stream, a, bt);
  else if (prec == GW_BF16X3)
    hipLaunchKernelGGL(bwb_bf16x3_kernel, dim3((unsigned)grid), dim3(NT), 0, ctx->stream, a, bt);
  else if (vec)
    hipLaunchKernelGGL(bwb_f32_direct_kernel<true>, dim3((unsigned)grid), dim3(NTD), 0,
                       ctx->stream, a, bt);
  else
    hipLaunchKernelGGL(bwb_f32_direct_kernel<false>, dim3((unsigned)grid), dim3(NTD), 0,
                       ctx->stream, a, bt);
}

gw::TransposeJob tr_job(const void* R, int64_t rows, int64_t ldr, int N, float* RT) {
  return gw::TransposeJob{static_cast<const float*>(R), rows, ldr, N, RT, rt_ld(rows)};
}

}  // namespace

namespace {

// Device buffers of one gw_sigma_diag call.
struct SigmaBufs {
  double* part;   // [F][2 * col_tiles][rows]
  double* W;      // [F][rows]
  float* RT;      // [N][rt_ld(rows)], FP32 path only
  __bf16* R3;     // BF16x3 path: split QP rows, hi then lo, k-blocked [rows_pad][Npad]
  __bf16* W3;     // BF16x3 path: split W^, hi then lo, k-blocked [F][Npad][Npad]
};

// Bytes of each buffer of one call, each rounded up to 256 bytes.
struct SigmaSizes {
  size_t part, w, rt, r3, w3;
  size_t total() const { return part + w + rt + r3 + w3; }
};

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

inline int64_t pad128(int64_t n) { return (n + BM - 1) / BM * BM; }

SigmaSizes sigma_sizes(gw_precision prec, int N, int64_t rows, int F) {
  SigmaSizes z;
  z.part = round256((size_t)F * 2 * ((N + BM - 1) / BM) * rows * sizeof(double));
  z.w = round256((size_t)F * rows * sizeof(double));
  z.rt = prec == GW_FP32 ? round256((size_t)N * rt_ld(rows) * sizeof(float)) : 0;
  z.r3 = prec == GW_BF16X3 ? round256((size_t)2 * pad128(rows) * pad128(N) * sizeof(__bf16)) : 0;
  z.w3 = prec == GW_BF16X3 ? round256((size_t)2 * F * pad128(N) * pad128(N) * sizeof(__bf16)) : 0;
  return z;
}

gw_status sigma_check(gw_ctx ctx, const char* who, gw_precision prec, int n_naf, int n_qp,
                      int n_mo, const double* eps_mo, const void* R_qp, int64_t ld_R, int n_w,
                      const double* omega, const double* w_omega, const void* W_hat,
                      int n_pade, const double* omega_pade, double* sigma_iw) {
  GW_REQUIRE(ctx, prec == GW_FP64 || prec == GW_FP32 || prec == GW_BF16X3,
             "%s: unknown precision %d", who, (int)prec);
  GW_REQUIRE(ctx, n_naf >= 1 && n_qp >= 1 && n_mo >= 1 && n_w >= 1 && n_pade >= 1,
             "%s: bad sizes", who);
  GW_REQUIRE(ctx, eps_mo && R_qp && omega && w_omega && W_hat && omega_pade && sigma_iw,
             "%s: NULL argument", who);
  GW_REQUIRE(ctx, ld_R == 0 || ld_R >= n_naf, "%s: ld_R < n_naf", who);
  return GW_OK;
}

// The contraction, the reduction of its partials and the quadrature, with
// the call's buffers supplied by the caller of this function.
gw_status sigma_diag_run(gw_ctx ctx, gw_precision prec, int n_naf, int n_qp, int n_mo,
                         const double* eps_mo, double eps_F, const void* R_qp, int64_t ld_R,
                         int n_w, const double* omega, const double* w_omega,
                         const void* W_hat, int n_pade, const double* omega_pade,
                         int accumulate, double* sigma_iw, double* W_nm, const SigmaBufs& b) {
  const int N = n_naf, F = n_w;
  const int64_t rows = (int64_t)n_qp * n_mo;
  const double* d_eps = gw::stage_t(ctx, eps_mo, n_mo);
  const double* d_om = gw::stage_t(ctx, omega, n_w);
  const double* d_wt = gw::stage_t(ctx, w_omega, n_w);
  const double* d_op = gw::stage_t(ctx, omega_pade, n_pade);
  if (!d_eps || !d_om || !d_wt || !d_op) return GW_EINVAL;
  const int row_tiles = (int)((rows + BM - 1) / BM);
  const int col_tiles = (N + BM - 1) / BM;
  const int n_part = 2 * col_tiles;
  BwbArgs a{R_qp, W_hat, rows, N, ld_R, F, row_tiles, col_tiles, b.part, nullptr, 0};
  if (prec == GW_FP32) {
    const gw::TransposeJob t = tr_job(R_qp, rows, ld_R, N, b.RT);
    GW_TRY(gw::transpose_f32(ctx, {t}));
    a.RT = b.RT;
    a.ldt = t.ld_dst;
  }
  const int64_t grid = (int64_t)F * row_tiles * col_tiles;
  if (prec == GW_BF16X3) {
    // split both operands once, then the direct BF16x3 contraction
    const int64_t rp = pad128(rows), np = pad128(N);
    const Split3Args sr{static_cast<const float*>(R_qp), rows, ld_R, 0, N, b.R3,
                        b.R3 + rp * np, rp, np, 1};
    const Split3Args sw{static_cast<const float*>(W_hat), N, N, (int64_t)N * N, N, b.W3,
                        b.W3 + (int64_t)F * np * np, np, np, F};
    const int ps = gw::prof_begin(ctx);
    hipLaunchKernelGGL(split3_kernel, dim3(grid_for(rp * np, 256)), dim3(256), 0, ctx->stream,
                       sr);
    hipLaunchKernelGGL(split3_kernel, dim3(grid_for((int64_t)F * np * np, 256)), dim3(256), 0,
                       ctx->stream, sw);
    gw::prof_end(ctx, ps, "bwb_split_bf16x3", 0.0,
                 4.0 * ((double)rows * N + (double)F * N * N) +
                     4.0 * ((double)rp * np + (double)F * np * np));
    GW_TRY(gw::launch_check(ctx, "split3_kernel"));
    const Bwb3Args a3{b.R3, b.R3 + rp * np, b.W3, b.W3 + (int64_t)F * np * np,
                      static_cast<const float*>(R_qp), ld_R, rows, N, (int)np, F, row_tiles,
                      col_tiles, b.part, rp};
    // 4 or 8 waves per workgroup, autotuned per shape (trials write only partials)
    auto launch = [&](int nw) {
      if (nw == 8)
        hipLaunchKernelGGL(bwb_bf16x3_direct_kernel<8>, dim3((unsigned)grid), dim3(512), 0,
                           ctx->stream, a3);
      else
        hipLaunchKernelGGL(bwb_bf16x3_direct_kernel<4>, dim3((unsigned)grid), dim3(256), 0,
                           ctx->stream, a3);
      return gw::launch_check(ctx, "bwb_bf16x3_direct_kernel");
    };
    const int nw = gw::tune(ctx, "bwb3:" + std::to_string(N) + ":" + std::to_string(rows) + ":" +
                                     std::to_string(F),
                            {4, 8}, launch);
    const int pi = gw::prof_begin(ctx);
    GW_TRY(launch(nw));
    gw::prof_end(ctx, pi, "bwb_bf16x3", (double)F * (double)rows * N * (N + 1.0),
                 4.0 * ((double)rp * np + (double)F * np * np));
    GW_TRY(gw::launch_check(ctx, "bwb_bf16x3_direct_kernel"));
  } else {
  const int pi = gw::prof_begin(ctx);
  launch_bwb(ctx, prec, a, Batch{}, grid, w_rows_aligned(W_hat, N));
  {
    const double esz = prec == GW_FP64 ? 8.0 : 4.0;
    // algorithmic work of the symmetric form: rows * N (N + 1) per frequency
    gw::prof_end(ctx, pi, prec == GW_FP64 ? "bwb_f64" : (prec == GW_BF16X3 ? "bwb_bf16x3" : "bwb_f32"),
                 (double)F * (double)rows * N * (N + 1.0),
                 (double)rows * N * esz + (double)F * N * (double)N * esz);
  }
  GW_TRY(gw::launch_check(ctx, "bwb kernel"));
  }
  hipLaunchKernelGGL(w_reduce_kernel, dim3(grid_for((int64_t)F * rows, 256)), dim3(256), 0,
                     ctx->stream, WRedArgs{b.part, n_part, rows, F, b.W, W_nm});
  GW_TRY(gw::launch_check(ctx, "w_reduce_kernel"));
  hipLaunchKernelGGL(sigma_quad_kernel, dim3(n_qp * n_pade), dim3(256), 0, ctx->stream,
                     QuadArgs{b.W, F, n_qp, n_mo, d_eps, eps_F, d_om, d_wt, d_op, n_pade,
                              accumulate, sigma_iw});
  return gw::launch_check(ctx, "sigma_quad_kernel");
}

// Fixed scratch of gw_sigma_diag_noalloc: one array per GPU, present from
// the loading of the code object until the process ends.  Host code never
// passes `scratch` itself (its host-side name is not a device address); it
// uses the device address looked up once per device by sigma_scratch_init.
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

namespace gw {

// Looks up this device's copy of `scratch` (the device must be current).
// Called by gw_create; repeated calls for a device are no-ops.
gw_status sigma_scratch_init(gw_ctx ctx, int device) {
  if (device < 0 || device >= kMaxDevices)
    return fail(ctx, GW_EUNSUPPORTED, "device index %d beyond the scratch table (%d)", device,
                kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return GW_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return fail(ctx, GW_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", device,
                hipGetErrorString(e));
  }
  g_scratch_ptr[device] = ptr;
  return GW_OK;
}

}  // namespace gw

extern "C" gw_status gw_sigma_diag(gw_ctx ctx, gw_precision prec, int n_naf, int n_qp,
                                   int n_mo, const double* eps_mo, double eps_F,
                                   const void* R_qp, int64_t ld_R, int n_w,
                                   const double* omega,
                                   const double* w_omega, const void* W_hat, int n_pade,
                                   const double* omega_pade, int accumulate,
                                   double* sigma_iw, double* W_nm) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_sigma_diag: ctx is NULL");
  gw::clear_error(ctx);
  GW_TRY(sigma_check(ctx, "gw_sigma_diag", prec, n_naf, n_qp, n_mo, eps_mo, R_qp, ld_R, n_w,
                     omega, w_omega, W_hat, n_pade, omega_pade, sigma_iw));
  if (ld_R == 0) ld_R = n_naf;
  GW_HIP(ctx, hipSetDevice(ctx->device));
  const int64_t rows = (int64_t)n_qp * n_mo;
  const SigmaSizes z = sigma_sizes(prec, n_naf, rows, n_w);
  SigmaBufs b{};
  b.part = static_cast<double*>(gw::ws_get(ctx, WS_SIGMA_PART, z.part));
  b.W = static_cast<double*>(gw::ws_get(ctx, WS_SIGMA_W, z.w));
  if (!b.part || !b.W) return GW_ENOMEM;
  if (prec == GW_FP32) {
    b.RT = static_cast<float*>(gw::ws_get(ctx, WS_SIGMA_RT, z.rt));
    if (!b.RT) return GW_ENOMEM;
  }
  if (prec == GW_BF16X3) {
    b.R3 = static_cast<__bf16*>(gw::ws_get(ctx, WS_B3_R, z.r3));
    b.W3 = static_cast<__bf16*>(gw::ws_get(ctx, WS_B3_W, z.w3));
    if (!b.R3 || !b.W3) return GW_ENOMEM;
  }
  return sigma_diag_run(ctx, prec, n_naf, n_qp, n_mo, eps_mo, eps_F, R_qp, ld_R, n_w, omega,
                        w_omega, W_hat, n_pade, omega_pade, accumulate, sigma_iw, W_nm, b);
}

extern "C" gw_status gw_sigma_diag_noalloc(gw_ctx ctx, gw_precision prec, int n_naf, int n_qp,
                                           int n_mo, const double* eps_mo, double eps_F,
                                           const void* R_qp, int64_t ld_R, int n_w,
                                           const double* omega, const double* w_omega,
                                           const void* W_hat, int n_pade,
                                           const double* omega_pade, int accumulate,
                                           double* sigma_iw, double* W_nm) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_sigma_diag_noalloc: ctx is NULL");
  gw::clear_error(ctx);
  GW_TRY(sigma_check(ctx, "gw_sigma_diag_noalloc", prec, n_naf, n_qp, n_mo, eps_mo, R_qp, ld_R,
                     n_w, omega, w_omega, W_hat, n_pade, omega_pade, sigma_iw));
  if (ld_R == 0) ld_R = n_naf;
  const int64_t rows = (int64_t)n_qp * n_mo;
  const SigmaSizes z = sigma_sizes(prec, n_naf, rows, n_w);
  GW_REQUIRE(ctx, z.total() <= kNoallocScratchBytes,
             "gw_sigma_diag_noalloc: the call needs %zu bytes of scratch, the fixed buffer holds "
             "%zu; split the frequencies or the QP states over several calls",
             z.total(), kNoallocScratchBytes);
  GW_HIP(ctx, hipSetDevice(ctx->device));
  GW_TRY(gw::sigma_scratch_init(ctx, ctx->device));   // no-op once looked up
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    base = g_scratch_ptr[ctx->device];
  }
  unsigned char* p = static_cast<unsigned char*>(base);
  SigmaBufs b{};
  b.part = reinterpret_cast<double*>(p);
  b.W = reinterpret_cast<double*>(p + z.part);
  b.RT = prec == GW_FP32 ? reinterpret_cast<float*>(p + z.part + z.w) : nullptr;
  b.R3 = prec == GW_BF16X3 ? reinterpret_cast<__bf16*>(p + z.part + z.w + z.rt) : nullptr;
  b.W3 = prec == GW_BF16X3 ? reinterpret_cast<__bf16*>(p + z.part + z.w + z.rt + z.r3) : nullptr;
  return sigma_diag_run(ctx, prec, n_naf, n_qp, n_mo, eps_mo, eps_F, R_qp, ld_R, n_w, omega,
                        w_omega, W_hat, n_pade, omega_pade, accumulate, sigma_iw, W_nm, b);
}

extern "C" gw_status gw_sigma_diag_batched(gw_ctx ctx, gw_precision prec, int n_jobs,
                                           const gw_sigma_job* jobs, int accumulate) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_sigma_diag_batched: ctx is NULL");
  gw::clear_error(ctx);
  GW_REQUIRE(ctx, prec == GW_FP64 || prec == GW_FP32 || prec == GW_BF16X3,
             "gw_sigma_diag_batched: unknown precision %d", (int)prec);
  GW_REQUIRE(ctx, n_jobs >= 0 && (n_jobs == 0 || jobs), "gw_sigma_diag_batched: bad n_jobs");
  for (int d = 0; d < n_jobs; ++d) {
    const gw_sigma_job& j = jobs[d];
    GW_REQUIRE(ctx, j.n_naf >= 1 && j.n_qp >= 1 && j.n_mo >= 1 && j.n_w >= 1 && j.n_pade >= 1,
               "gw_sigma_diag_batched: job %d: bad sizes", d);
    GW_REQUIRE(ctx, j.eps_mo && j.R_qp && j.omega && j.w_omega && j.W_hat && j.omega_pade &&
                        j.sigma_iw,
               "gw_sigma_diag_batched: job %d: NULL argument", d);
    GW_REQUIRE(ctx, j.ld_R == 0 || j.ld_R >= j.n_naf, "gw_sigma_diag_batched: job %d: ld_R < n_naf", d);
  }
  if (n_jobs == 0) return GW_OK;
  GW_HIP(ctx, hipSetDevice(ctx->device));
  size_t part_tot = 0, w_tot = 0;
  for (int d = 0; d < n_jobs; ++d) {
    const gw_sigma_job& j = jobs[d];
    const size_t rows = (size_t)j.n_qp * j.n_mo;
    part_tot += (size_t)j.n_w * 2 * ((j.n_naf + BM - 1) / BM) * rows;
    w_tot += (size_t)j.n_w * rows;
  }
  double* part = static_cast<double*>(gw::ws_get(ctx, WS_SIGMA_PART, part_tot * sizeof(double)));
  double* W = static_cast<double*>(gw::ws_get(ctx, WS_SIGMA_W, w_tot * sizeof(double)));
  if (!part || !W) return GW_ENOMEM;
  float* RT = nullptr;
  bool vec = true;
  if (prec == GW_FP32) {
    size_t rt_tot = 0;
    for (int d = 0; d < n_jobs; ++d)
      rt_tot += (size_t)jobs[d].n_naf * rt_ld((int64_t)jobs[d].n_qp * jobs[d].n_mo);
    RT = static_cast<float*>(gw::ws_get(ctx, WS_SIGMA_RT, rt_tot * sizeof(float)));
    if (!RT) return GW_ENOMEM;
  }
  std::vector<gw::TransposeJob> trs;
  size_t rto = 0;
  std::vector<BwbArgs> bw;
  std::vector<WRedArgs> red;
  std::vector<QuadArgs> quad;
  std::vector<int64_t> n_red;
  size_t po = 0, wo = 0;
  double flops = 0, bytes = 0;
  const double esz = prec == GW_FP64 ? 8.0 : 4.0;
  for (int d = 0; d < n_jobs; ++d) {
    const gw_sigma_job& j = jobs[d];
    const int N = j.n_naf, F = j.n_w;
    const int64_t rows = (int64_t)j.n_qp * j.n_mo;
    const double* d_eps = gw::stage_t(ctx, j.eps_mo, j.n_mo);
    const double* d_om = gw::stage_t(ctx, j.omega, F);
    const double* d_wt = gw::stage_t(ctx, j.w_omega, F);
    const double* d_op = gw::stage_t(ctx, j.omega_pade, j.n_pade);
    if (!d_eps || !d_om || !d_wt || !d_op) return GW_EINVAL;
    const int row_tiles = (int)((rows + BM - 1) / BM);
    const int col_tiles = (N + BM - 1) / BM;
    const int n_part = 2 * col_tiles;
    BwbArgs b{j.R_qp, j.W_hat, rows, N, j.ld_R ? j.ld_R : N, F, row_tiles, col_tiles,
              part + po, nullptr, 0};
    if (prec == GW_FP32) {
      const gw::TransposeJob t = tr_job(j.R_qp, rows, b.ldr, N, RT + rto);
      trs.push_back(t);
      b.RT = t.dst;
      b.ldt = t.ld_dst;
      rto += (size_t)N * t.ld_dst;
      vec = vec && w_rows_aligned(j.W_hat, N);
    }
    bw.push_back(b);
    red.push_back(WRedArgs{part + po, n_part, rows, F, W + wo, j.W_nm});
    n_red.push_back((int64_t)F * rows);
    quad.push_back(QuadArgs{W + wo, F, j.n_qp, j.n_mo, d_eps, j.eps_F, d_om, d_wt, d_op,
                            j.n_pade, accumulate, j.sigma_iw});
    po += (size_t)F * n_part * rows;
    wo += (size_t)F * rows;
    flops += (double)F * (double)rows * N * (N + 1.0);
    bytes += (double)rows * N * esz + (double)F * N * (double)N * esz;
  }
  // longest work units first: rows of a unit are fixed, its length grows with N
  std::vector<BwbArgs> order = bw;
  std::stable_sort(order.begin(), order.end(),
                   [](const BwbArgs& x, const BwbArgs& y) { return x.N > y.N; });
  std::vector<int64_t> off(1, 0);
  for (const BwbArgs& a : order) off.push_back(off.back() + (int64_t)a.F * a.row_tiles * a.col_tiles);
  constexpr int CHUNK = 8;
  Batch bt;
  GW_TRY(gw::stage_batch(ctx, order, off, CHUNK, bt));
  const int64_t grid = (off.back() + 8 * CHUNK - 1) / (8 * CHUNK) * (8 * CHUNK);
  if (prec == GW_FP32) GW_TRY(gw::transpose_f32(ctx, trs));
  const int pi = gw::prof_begin(ctx);
  launch_bwb(ctx, prec, BwbArgs{}, bt, grid, vec);
  gw::prof_end(ctx, pi, prec == GW_FP64 ? "bwb_f64" : (prec == GW_BF16X3 ? "bwb_bf16x3" : "bwb_f32"),
               flops, bytes);
  GW_TRY(gw::launch_check(ctx, "batched bwb kernel"));
  GW_TRY(gw::elementwise_batched(ctx, red, n_red, w_reduce_batched_kernel, "w_reduce_batched"));
  std::vector<int64_t> qoff(1, 0);
  for (const QuadArgs& q : quad) qoff.push_back(qoff.back() + (int64_t)q.Q * q.Pd);
  Batch bq;
  GW_TRY(gw::stage_batch(ctx, quad, qoff, 1, bq));
  hipLaunchKernelGGL(sigma_quad_batched_kernel, dim3((unsigned)qoff.back()), dim3(256), 0,
                     ctx->stream, bq);
  return gw::launch_check(ctx, "sigma_quad_batched_kernel");
}

namespace gw {

void sigma_ws_bytes(int N, int64_t rows, int F, size_t* part_bytes, size_t* w_bytes,
                    size_t* rt_bytes) {
  *part_bytes = (size_t)F * 2 * ((N + BM - 1) / BM) * rows * sizeof(double);
  *w_bytes = (size_t)F * rows * sizeof(double);
  *rt_bytes = (size_t)N * rt_ld(rows) * sizeof(float);
}

}  // namespace gw

namespace {

// dst[c][r] = src[r][c] for c < cols, r < rows; rows .. ld_dst-1 zero.
// 64 x 64 tiles through LDS, one workgroup each.
__device__ __forceinline__ void transpose_tile(const gw::TransposeJob& t, int64_t tile) {
  __shared__ float sh[64][65];
  const int64_t ktiles = (t.cols + 63) / 64;
  const int64_t r0 = (tile / ktiles) * 64;
  const int c0 = (int)(tile % ktiles) * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;      // 256 threads: 4 rows a pass
  for (int y = ty; y < 64; y += 4) {
    const int64_t r = r0 + y;
    const int c = c0 + tx;
    sh[y][tx] = (r < t.rows && c < t.cols) ? t.src[r * t.ld_src + c] : 0.f;
  }
  __syncthreads();
  for (int y = ty; y < 64; y += 4) {
    const int c = c0 + y;
    const int64_t r = r0 + tx;
    if (c < t.cols && r < t.ld_dst) t.dst[(int64_t)c * t.ld_dst + r] = sh[tx][y];
  }
}

__global__ __launch_bounds__(256) void transpose_batched_kernel(Batch bt) {
  const int64_t u = blockIdx.x;
  if (u >= bt.units) return;
  const int d = find_problem(bt.off, bt.n, u);
  transpose_tile(static_cast<const gw::TransposeJob*>(bt.descs)[d], u - bt.off[d]);
}

}  // namespace

namespace gw {

gw_status transpose_f32(gw_ctx ctx, const std::vector<TransposeJob>& jobs) {
  std::vector<int64_t> off(1, 0);
  for (const TransposeJob& t : jobs)
    off.push_back(off.back() + ((t.ld_dst + 63) / 64) * (int64_t)((t.cols + 63) / 64));
  if (off.back() == 0) return GW_OK;
  Batch bt;
  GW_TRY(stage_batch(ctx, jobs, off, 1, bt));
  hipLaunchKernelGGL(transpose_batched_kernel, dim3((unsigned)off.back()), dim3(256), 0,
                     ctx->stream, bt);
  return launch_check(ctx, "transpose_batched_kernel");
}

}  // namespace gw
