// Scaled SYRK on MFMA: the Laplace-transformed polarizability matrices
//   M^m_PQ = sum_r X_rP s_m(r) X_rQ,  s_m(ia) = w_m D_ia exp(-D_ia^2 x_m)
// (Eq. 10) and, with a constant scale, the NAF metric of Eq. 11.
//
// X is [k_rows][N] row-major (rows = occupied-virtual pairs, aux contiguous).
// Each workgroup computes one 128 x 128 lower-triangle tile of one matrix m
// over one slice of rows (split-K); the per-row scale is multiplied into the
// A operand while the tile is staged into LDS.  Partial tiles are written in
// FP64 and summed in a fixed order by a second kernel, so results are
// bitwise reproducible.
//
//  FP32 / BF16x3: v_mfma_f32_32x32x2f32 / v_mfma_f32_32x32x16_bf16, FP32
//                 accumulators added into FP64 registers every 256 rows.
//  FP64:          v_mfma_f64_16x16x4f64.
#include <algorithm>
#include <cmath>

#include "common.hpp"

namespace {

constexpr int BM = 128;             // tile edge (P and Q)
constexpr int NT = 256;             // threads per workgroup (4 waves, 2 x 2)
constexpr int FLUSH_ROWS = 256;     // FP32 -> FP64 flush interval (rows)

struct SyrkArgs {
  const void* X;
  int64_t k_rows;
  int N;
  int64_t ld;           // row stride of X in elements (>= N)
  int L;
  const void* scale;    // [L][k_rows] (element type) or nullptr
  double cscale;
  int tiles_side;
  int n_tiles;
  int splits;
  int64_t rows_per_split;
  double* part;         // [splits][L][n_tiles][BM*BM]
};

__device__ __forceinline__ void tile_coords(int t, int& ti, int& tj) {
  int i = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  ti = i;
  tj = t - i * (i + 1) / 2;
}

// ------------------------------------------------------------------ FP32 MFMA
// 8 waves (4 x 2), each owning a 32 x 64 slice of the 128 x 128 tile, so the
// FP32 accumulators (32 AGPRs) and their FP64 running sums (64 VGPRs) leave
// room for two waves per SIMD.  FAST: rows 16-byte aligned (row stride a
// multiple of 4).  Tile loads then need no column guards: a float4 start
// past the row end is clamped back inside the row, and lanes past column N
// only feed outputs that are discarded.  Rows past the end are clamped and
// zeroed with a select, keeping the loads branch-free.
constexpr int NT32 = 512;
constexpr int BK32 = 32;

template <bool FAST, bool SCALED>
__global__ __launch_bounds__(NT32, 2) void syrk_f32_kernel(SyrkArgs a) {
  __shared__ float As[2][BK32][BM];
  __shared__ float Bs[2][BK32][BM];

  const int64_t lid = xcd_remap(blockIdx.x, gridDim.x);
  const int m = (int)(lid % a.L);
  const int t = (int)((lid / a.L) % a.n_tiles);
  const int s = (int)(lid / ((int64_t)a.L * a.n_tiles));
  int ti, tj;
  tile_coords(t, ti, tj);
  const int p0 = ti * BM, q0 = tj * BM;
  const int64_t r0 = (int64_t)s * a.rows_per_split;
  const int64_t r1 = min(r0 + a.rows_per_split, a.k_rows);

  const float* X = static_cast<const float*>(a.X);
  const float* scale = SCALED ? static_cast<const float*>(a.scale) + (int64_t)m * a.k_rows : nullptr;
  const float csc = (float)a.cscale;

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wy = wave >> 1, wx = wave & 1;            // rows wy*32, cols wx*64
  const int lrow = tid >> 5, lcol = (tid & 31) * 4;   // loader rows lrow, lrow + 16

  f32x16 acc[2];
  double acc64[2][16];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) { acc[j][r] = 0.f; acc64[j][r] = 0.0; }

  // Tile loads only issue the global reads; the scale and the row mask are
  // applied when the registers are written to LDS after the MFMA block, so
  // the reads stay in flight behind the block.
  float4 ra[2], rb[2];
  float rs[2], rm[2];
  auto gload = [&](int64_t kb) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t r = kb + lrow + 16 * h;
      if (FAST) {
        const bool ok = r < r1;
        const int64_t rr = ok ? r : r1 - 1;
        if (SCALED) rs[h] = scale[rr]; else rs[h] = csc;
        rm[h] = ok ? 1.f : 0.f;
        const float* row = X + rr * a.ld;
        ra[h] = *reinterpret_cast<const float4*>(row + min(p0 + lcol, (int)a.ld - 4));
        rb[h] = *reinterpret_cast<const float4*>(row + min(q0 + lcol, (int)a.ld - 4));
      } else {
        float4 va = make_float4(0.f, 0.f, 0.f, 0.f), vb = va;
        rs[h] = 0.f;
        rm[h] = 0.f;
        if (r < r1) {
          if (SCALED) rs[h] = scale[r]; else rs[h] = csc;
          rm[h] = 1.f;
          const float* row = X + r * a.ld;
          const int pa = p0 + lcol, pb = q0 + lcol;
          if (pa + 0 < a.N) va.x = row[pa + 0];
          if (pa + 1 < a.N) va.y = row[pa + 1];
          if (pa + 2 < a.N) va.z = row[pa + 2];
          if (pa + 3 < a.N) va.w = row[pa + 3];
          if (pb + 0 < a.N) vb.x = row[pb + 0];
          if (pb + 1 < a.N) vb.y = row[pb + 1];
          if (pb + 2 < a.N) vb.z = row[pb + 2];
          if (pb + 3 < a.N) vb.w = row[pb + 3];
        }
        ra[h] = va;
        rb[h] = vb;
      }
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const float sa = rs[h] * rm[h], sb = rm[h];
      *reinterpret_cast<float4*>(&As[buf][lrow + 16 * h][lcol]) =
          make_float4(ra[h].x * sa, ra[h].y * sa, ra[h].z * sa, ra[h].w * sa);
      *reinterpret_cast<float4*>(&Bs[buf][lrow + 16 * h][lcol]) =
          make_float4(rb[h].x * sb, rb[h].y * sb, rb[h].z * sb, rb[h].w * sb);
    }
  };

  const int nk = (int)((r1 - r0 + BK32 - 1) / BK32);
  constexpr int FLUSH_STAGES = FLUSH_ROWS / BK32;
  if (nk > 0) {
    gload(r0);
    sstore(0);
  }
  __syncthreads();
  const int arow = wy * 32 + (lane & 31);
  const int bcol = wx * 64 + (lane & 31);
  const int ksub = lane >> 5;
  for (int it = 0; it < nk; ++it) {
    const int cur = it & 1;
    if (it + 1 < nk) gload(r0 + (int64_t)(it + 1) * BK32);
    float a_c = As[cur][ksub][arow];
    float b0_c = Bs[cur][ksub][bcol];
    float b1_c = Bs[cur][ksub][bcol + 32];
#pragma unroll
    for (int kk = 0; kk < BK32 / 2; ++kk) {
      float a_n = 0.f, b0_n = 0.f, b1_n = 0.f;
      if (kk + 1 < BK32 / 2) {
        const int kr = 2 * (kk + 1) + ksub;
        a_n = As[cur][kr][arow];
        b0_n = Bs[cur][kr][bcol];
        b1_n = Bs[cur][kr][bcol + 32];
      }
      acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a_c, b0_c, acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a_c, b1_c, acc[1], 0, 0, 0);
      a_c = a_n;
      b0_c = b0_n;
      b1_c = b1_n;
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

  double* out = a.part + (((int64_t)s * a.L + m) * a.n_tiles + t) * (BM * BM);
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = wy * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      const int col = wx * 64 + j * 32 + (lane & 31);
      out[row * BM + col] = acc64[j][r];
    }
}

// ------------------------------------------------------------------ BF16x3
// x = hi + lo with hi = bf16(x), lo = bf16(x - hi); each product is formed
// as hi*hi + hi*lo + lo*hi on v_mfma_f32_32x32x16_bf16 (the lo*lo term,
// ~2^-16 relative, is dropped).  The split happens in the LDS store; the LDS
// tiles are k-contiguous ([column][row of X]) so each MFMA operand (8
// consecutive k for one column) is one 16-byte read.  4 waves, 64 x 64 each;
// FP32 accumulation over the split-K slice, FP64 across slices.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
constexpr int NTB = 256;
constexpr int BKB = 32;
constexpr int LDB = BKB + 8;        // padded k stride (bf16) of an LDS row

__device__ __forceinline__ void split4(const float4 v, float s, bf16x4& hi, bf16x4& lo) {
  const float x[4] = {v.x * s, v.y * s, v.z * s, v.w * s};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const __bf16 h = (__bf16)x[e];
    hi[e] = h;
    lo[e] = (__bf16)(x[e] - (float)h);
  }
}

template <bool FAST, bool SCALED>
__global__ __launch_bounds__(NTB, 2) void syrk_bf16x3_kernel(SyrkArgs a) {
  __shared__ __attribute__((aligned(16))) __bf16 Ah[2][BM][LDB];
  __shared__ __attribute__((aligned(16))) __bf16 Al[2][BM][LDB];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[2][BM][LDB];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[2][BM][LDB];

  const int64_t lid = xcd_remap(blockIdx.x, gridDim.x);
  const int m = (int)(lid % a.L);
  const int t = (int)((lid / a.L) % a.n_tiles);
  const int s = (int)(lid / ((int64_t)a.L * a.n_tiles));
  int ti, tj;
  tile_coords(t, ti, tj);
  const int p0 = ti * BM, q0 = tj * BM;
  const int64_t r0 = (int64_t)s * a.rows_per_split;
  const int64_t r1 = min(r0 + a.rows_per_split, a.k_rows);

  const float* X = static_cast<const float*>(a.X);
  const float* scale = SCALED ? static_cast<const float*>(a.scale) + (int64_t)m * a.k_rows : nullptr;
  const float csc = (float)a.cscale;

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wy = wave >> 1, wx = wave & 1;
  // loader: 4 consecutive rows (krow..krow+3) x 4 consecutive columns (lcol)
  const int lcol = (tid & 31) * 4, krow = (tid >> 5) * 4;

  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  float4 ra[4], rb[4];
  float rs[4];
  auto gload = [&](int64_t kb) {
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int64_t r = kb + krow + h;
      if (FAST) {
        const bool ok = r < r1;
        const int64_t rr = ok ? r : r1 - 1;
        const float sc = SCALED ? scale[rr] : csc;
        rs[h] = ok ? sc : 0.f;
        const float* row = X + rr * a.ld;
        ra[h] = *reinterpret_cast<const float4*>(row + min(p0 + lcol, (int)a.ld - 4));
        rb[h] = *reinterpret_cast<const float4*>(row + min(q0 + lcol, (int)a.ld - 4));
        if (!ok) rb[h] = make_float4(0.f, 0.f, 0.f, 0.f);
      } else {
        float4 va = make_float4(0.f, 0.f, 0.f, 0.f), vb = va;
        rs[h] = 0.f;
        if (r < r1) {
          rs[h] = SCALED ? scale[r] : csc;
          const float* row = X + r * a.ld;
          const int pa = p0 + lcol, pb = q0 + lcol;
          if (pa + 0 < a.N) va.x = row[pa + 0];
          if (pa + 1 < a.N) va.y = row[pa + 1];
          if (pa + 2 < a.N) va.z = row[pa + 2];
          if (pa + 3 < a.N) va.w = row[pa + 3];
          if (pb + 0 < a.N) vb.x = row[pb + 0];
          if (pb + 1 < a.N) vb.y = row[pb + 1];
          if (pb + 2 < a.N) vb.z = row[pb + 2];
          if (pb + 3 < a.N) vb.w = row[pb + 3];
        }
        ra[h] = va;
        rb[h] = vb;
      }
    }
  };
  // registers hold 4 rows x 4 columns; LDS wants, per column, 4 consecutive rows
  auto sstore = [&](int buf) {
    bf16x4 ah[4], al[4], bh[4], bl[4];   // [row h] -> 4 columns
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      split4(ra[h], rs[h], ah[h], al[h]);
      split4(rb[h], 1.f, bh[h], bl[h]);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      bf16x4 v;
      v = bf16x4{ah[0][c], ah[1][c], ah[2][c], ah[3][c]};
      *reinterpret_cast<bf16x4*>(&Ah[buf][lcol + c][krow]) = v;
      v = bf16x4{al[0][c], al[1][c], al[2][c], al[3][c]};
      *reinterpret_cast<bf16x4*>(&Al[buf][lcol + c][krow]) = v;
      v = bf16x4{bh[0][c], bh[1][c], bh[2][c], bh[3][c]};
      *reinterpret_cast<bf16x4*>(&Bh[buf][lcol + c][krow]) = v;
      v = bf16x4{bl[0][c], bl[1][c], bl[2][c], bl[3][c]};
      *reinterpret_cast<bf16x4*>(&Bl[buf][lcol + c][krow]) = v;
    }
  };

  const int nk = (int)((r1 - r0 + BKB - 1) / BKB);
  if (nk > 0) {
    gload(r0);
    sstore(0);
  }
  __syncthreads();
  const int kl = 8 * (lane >> 5);
  for (int it = 0; it < nk; ++it) {
    const int cur = it & 1;
    if (it + 1 < nk) gload(r0 + (int64_t)(it + 1) * BKB);
#pragma unroll
    for (int ks = 0; ks < BKB; ks += 16) {
      bf16x8 ahf[2], alf[2], bhf[2], blf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int pr = wy * 64 + i * 32 + (lane & 31);
        const int qc = wx * 64 + i * 32 + (lane & 31);
        ahf[i] = *reinterpret_cast<const bf16x8*>(&Ah[cur][pr][ks + kl]);
        alf[i] = *reinterpret_cast<const bf16x8*>(&Al[cur][pr][ks + kl]);
        bhf[i] = *reinterpret_cast<const bf16x8*>(&Bh[cur][qc][ks + kl]);
        blf[i] = *reinterpret_cast<const bf16x8*>(&Bl[cur][qc][ks + kl]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahf[i], bhf[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahf[i], blf[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alf[i], bhf[j], acc[i][j], 0, 0, 0);
        }
    }
    if (it + 1 < nk) sstore(cur ^ 1);
    __syncthreads();
  }

  double* out = a.part + (((int64_t)s * a.L + m) * a.n_tiles + t) * (BM * BM);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wy * 64 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int col = wx * 64 + j * 32 + (lane & 31);
        out[row * BM + col] = (double)acc[i][j][r];
      }
}

// ------------------------------------------------------------------ FP64 MFMA
constexpr int BK64 = 16;

__global__ __launch_bounds__(NT, 1) void syrk_f64_kernel(SyrkArgs a) {
  __shared__ double As[2][BK64][BM];
  __shared__ double Bs[2][BK64][BM];

  const int64_t lid = xcd_remap(blockIdx.x, gridDim.x);
  const int m = (int)(lid % a.L);
  const int t = (int)((lid / a.L) % a.n_tiles);
  const int s = (int)(lid / ((int64_t)a.L * a.n_tiles));
  int ti, tj;
  tile_coords(t, ti, tj);
  const int p0 = ti * BM, q0 = tj * BM;
  const int64_t r0 = (int64_t)s * a.rows_per_split;
  const int64_t r1 = min(r0 + a.rows_per_split, a.k_rows);

  const double* X = static_cast<const double*>(a.X);
  const double* scale = a.scale ? static_cast<const double*>(a.scale) + (int64_t)m * a.k_rows : nullptr;

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wy = wave >> 1, wx = wave & 1;
  // loader: 16 rows x 128 doubles per operand = 1024 double2; 4 per thread
  const int lrow = tid >> 6, lcol = (tid & 63) * 2;   // rows lrow + 4h

  f64x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};

  double2 ra[4], rb[4];
  auto gload = [&](int64_t kb) {
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int64_t r = kb + lrow + 4 * h;
      double2 va = make_double2(0.0, 0.0), vb = va;
      if (r < r1) {
        const double sc = scale ? scale[r] : a.cscale;
        const int64_t rb = r * a.ld;
        const double* row = X + rb;
        const int pa = p0 + lcol, pb = q0 + lcol;
        if (pa + 1 < a.N && ((rb + pa) & 1) == 0) {
          va = *reinterpret_cast<const double2*>(row + pa);
        } else {
          if (pa < a.N) va.x = row[pa];
          if (pa + 1 < a.N) va.y = row[pa + 1];
        }
        if (pb + 1 < a.N && ((rb + pb) & 1) == 0) {
          vb = *reinterpret_cast<const double2*>(row + pb);
        } else {
          if (pb < a.N) vb.x = row[pb];
          if (pb + 1 < a.N) vb.y = row[pb + 1];
        }
        va.x *= sc; va.y *= sc;
      }
      ra[h] = va;
      rb[h] = vb;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      *reinterpret_cast<double2*>(&As[buf][lrow + 4 * h][lcol]) = ra[h];
      *reinterpret_cast<double2*>(&Bs[buf][lrow + 4 * h][lcol]) = rb[h];
    }
  };

  const int nk = (int)((r1 - r0 + BK64 - 1) / BK64);
  if (nk > 0) {
    gload(r0);
    sstore(0);
  }
  __syncthreads();
  for (int it = 0; it < nk; ++it) {
    const int cur = it & 1;
    if (it + 1 < nk) gload(r0 + (int64_t)(it + 1) * BK64);
#pragma unroll
    for (int kk = 0; kk < BK64 / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      double af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        af[i] = As[cur][kr][wy * 64 + i * 16 + (lane & 15)];
        bf[i] = Bs[cur][kr][wx * 64 + i * 16 + (lane & 15)];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    if (it + 1 < nk) sstore(cur ^ 1);
    __syncthreads();
  }

  double* out = a.part + (((int64_t)s * a.L + m) * a.n_tiles + t) * (BM * BM);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wy * 64 + i * 16 + (lane >> 4) + 4 * r;
        const int col = wx * 64 + j * 16 + (lane & 15);
        out[row * BM + col] = acc[i][j][r];
      }
}

// Sum the split-K partials in a fixed order into the lower triangle of out.
__global__ void syrk_reduce_kernel(const double* __restrict__ part, int splits,
                                   int L, int n_tiles, int N, double* __restrict__ out,
                                   int accumulate) {
  const int64_t per_tile = BM * BM;
  const int64_t total = (int64_t)L * n_tiles * per_tile;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int e = (int)(idx % per_tile);
    const int t = (int)((idx / per_tile) % n_tiles);
    const int m = (int)(idx / (per_tile * n_tiles));
    int ti, tj;
    tile_coords(t, ti, tj);
    const int p = ti * BM + e / BM, q = tj * BM + e % BM;
    if (p >= N || q >= N || q > p) continue;
    double v = 0.0;
    for (int s = 0; s < splits; ++s)
      v += part[(((int64_t)s * L + m) * n_tiles + t) * per_tile + e];
    double* dst = out + ((int64_t)m * N + p) * N + q;
    *dst = accumulate ? *dst + v : v;
  }
}

__global__ void mirror_kernel(double* M, int L, int N) {
  const int64_t total = (int64_t)L * N * N;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int q = (int)(idx % N);
    const int p = (int)((idx / N) % N);
    const int64_t m = idx / ((int64_t)N * N);
    if (q > p) M[(m * N + p) * N + q] = M[(m * N + q) * N + p];
  }
}

template <typename T>
__global__ void lt_scale_kernel(int L, const double* __restrict__ x,
                                const double* __restrict__ w, int n_i, int n_virt,
                                const double* __restrict__ eps_i,
                                const double* __restrict__ eps_a, T* __restrict__ out) {
  const int64_t k = (int64_t)n_i * n_virt;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < k * L;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx % k;
    const int m = (int)(idx / k);
    const int i = (int)(r / n_virt), aa = (int)(r % n_virt);
    const double d = eps_a[aa] - eps_i[i];
    out[idx] = (T)(w[m] * d * exp(-d * d * x[m]));
  }
}

inline int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  return (int)std::min<int64_t>(std::max<int64_t>(g, 1), 65536);
}

}  // namespace

namespace gw {

gw_status lt_scale_launch(gw_ctx ctx, gw_precision prec, int L, const double* d_x,
                          const double* d_w, int n_i, int n_virt,
                          const double* d_eps_i, const double* d_eps_a, void* scale) {
  const int64_t n = (int64_t)L * n_i * n_virt;
  if (prec == GW_FP64)
    hipLaunchKernelGGL(lt_scale_kernel<double>, dim3(grid_for(n, 256)), dim3(256), 0,
                       ctx->stream, L, d_x, d_w, n_i, n_virt, d_eps_i, d_eps_a,
                       static_cast<double*>(scale));
  else
    hipLaunchKernelGGL(lt_scale_kernel<float>, dim3(grid_for(n, 256)), dim3(256), 0,
                       ctx->stream, L, d_x, d_w, n_i, n_virt, d_eps_i, d_eps_a,
                       static_cast<float*>(scale));
  return launch_check(ctx, "lt_scale_kernel");
}

// Choose the split-K factor so the grid fills the 256 CUs evenly.
static int choose_splits(int64_t k_rows, int64_t units) {
  int best = 1;
  double best_eff = 0;
  for (int s = 1; s <= 16; ++s) {
    if (s > 1 && k_rows / s < 1024) break;
    const int64_t wg = units * s;
    const double eff = (double)wg / (256.0 * (double)((wg + 255) / 256));
    if (eff > best_eff + 0.02) { best_eff = eff; best = s; }
  }
  return best;
}

gw_status syrk_launch(gw_ctx ctx, gw_precision prec, const void* X, int64_t k_rows,
                      int N, int64_t ld, int L, const void* scale, double cscale,
                      double* out, int accumulate, const char* prof_name) {
  const int T = (N + BM - 1) / BM;
  const int n_tiles = T * (T + 1) / 2;
  const int S = k_rows > 0 ? choose_splits(k_rows, (int64_t)n_tiles * L) : 1;
  const int64_t align = prec == GW_FP64 ? BK64 : (prec == GW_BF16X3 ? BKB : FLUSH_ROWS);
  int64_t rps = (k_rows + S - 1) / S;
  rps = (rps + align - 1) / align * align;
  const size_t part_bytes = (size_t)S * L * n_tiles * BM * BM * sizeof(double);
  double* part = static_cast<double*>(ws_get(ctx, WS_SYRK_PART, part_bytes));
  if (!part) return GW_ENOMEM;
  SyrkArgs a{X, k_rows, N, ld, L, scale, cscale, T, n_tiles, S, rps, part};
  const int64_t grid = (int64_t)S * L * n_tiles;
  const int pi = prof_begin(ctx);
  const bool fast = prec != GW_FP64 && (ld % 4 == 0) && ld >= 4 &&
                    (reinterpret_cast<uintptr_t>(X) % 16 == 0);
  if (prec == GW_FP64) {
    hipLaunchKernelGGL(syrk_f64_kernel, dim3((unsigned)grid), dim3(NT), 0, ctx->stream, a);
  } else if (prec == GW_BF16X3) {
    auto kern = fast ? (scale ? syrk_bf16x3_kernel<true, true> : syrk_bf16x3_kernel<true, false>)
                     : (scale ? syrk_bf16x3_kernel<false, true> : syrk_bf16x3_kernel<false, false>);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(NTB), 0, ctx->stream, a);
  } else {
    auto kern = fast ? (scale ? syrk_f32_kernel<true, true> : syrk_f32_kernel<true, false>)
                     : (scale ? syrk_f32_kernel<false, true> : syrk_f32_kernel<false, false>);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(NT32), 0, ctx->stream, a);
  }
  // algorithmic work: L lower-triangle products of 2 k flops each; X read
  // once, the triangle written once
  const double esz = prec == GW_FP64 ? 8.0 : 4.0;
  prof_end(ctx, pi, prof_name,
           (double)L * N * (N + 1.0) * (double)k_rows,
           (double)k_rows * N * esz + (double)L * N * (N + 1.0) / 2.0 * 8.0);
  GW_TRY(launch_check(ctx, "syrk kernel"));
  const int64_t tot = (int64_t)L * n_tiles * BM * BM;
  hipLaunchKernelGGL(syrk_reduce_kernel, dim3(grid_for(tot, 256)), dim3(256), 0,
                     ctx->stream, part, S, L, n_tiles, N, out, accumulate);
  return launch_check(ctx, "syrk_reduce_kernel");
}

gw_status mirror_lower(gw_ctx ctx, double* M, int L, int N) {
  const int64_t tot = (int64_t)L * N * N;
  hipLaunchKernelGGL(mirror_kernel, dim3(grid_for(tot, 256)), dim3(256), 0, ctx->stream,
                     M, L, N);
  return launch_check(ctx, "mirror_kernel");
}

}  // namespace gw

extern "C" gw_status gw_polarizability_lt(gw_ctx ctx, gw_precision prec, int n_naf,
                                          int n_lt, const double* x_lt,
                                          const double* w_lt, int n_i, int n_virt,
                                          const double* eps_i, const double* eps_a,
                                          const void* R_chunk, int64_t ld_R,
                                          int accumulate, int finalize, double* M) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_polarizability_lt: ctx is NULL");
  gw::clear_error(ctx);
  GW_REQUIRE(ctx, prec == GW_FP64 || prec == GW_FP32 || prec == GW_BF16X3,
             "gw_polarizability_lt: unknown precision %d", (int)prec);

  GW_REQUIRE(ctx, n_naf >= 1 && n_lt >= 1 && n_lt <= 32 && n_i >= 0 && n_virt >= 1,
             "gw_polarizability_lt: bad sizes (n_naf=%d n_lt=%d n_i=%d n_virt=%d)",
             n_naf, n_lt, n_i, n_virt);
  GW_REQUIRE(ctx, x_lt && w_lt && M && eps_a && (n_i == 0 || (eps_i && R_chunk)),
             "gw_polarizability_lt: NULL argument");
  if (ld_R == 0) ld_R = n_naf;
  GW_REQUIRE(ctx, ld_R >= n_naf, "gw_polarizability_lt: ld_R < n_naf");
  GW_HIP(ctx, hipSetDevice(ctx->device));
  const int64_t k = (int64_t)n_i * n_virt;
  const double* dx = gw::stage_t(ctx, x_lt, n_lt);
  const double* dw = gw::stage_t(ctx, w_lt, n_lt);
  const double* dei = n_i ? gw::stage_t(ctx, eps_i, n_i) : nullptr;
  const double* dea = gw::stage_t(ctx, eps_a, n_virt);
  if (!dx || !dw || !dea || (n_i && !dei)) return GW_EINVAL;
  void* scale = nullptr;
  if (k > 0) {
    const size_t esz = prec == GW_FP64 ? 8 : 4;
    scale = gw::ws_get(ctx, WS_SYRK_SCALE, (size_t)n_lt * k * esz);
    if (!scale) return GW_ENOMEM;
    GW_TRY(gw::lt_scale_launch(ctx, prec, n_lt, dx, dw, n_i, n_virt, dei, dea, scale));
  }
  GW_TRY(gw::syrk_launch(ctx, prec, R_chunk, k, n_naf, ld_R, n_lt, scale, 1.0, M, accumulate,
                         prec == GW_FP64 ? "chi_syrk_f64"
                                         : (prec == GW_BF16X3 ? "chi_syrk_bf16x3" : "chi_syrk_f32")));
  if (finalize) GW_TRY(gw::mirror_lower(ctx, M, n_lt, n_naf));
  return GW_OK;
}
