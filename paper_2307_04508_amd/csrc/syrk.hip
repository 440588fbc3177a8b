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
//                 accumulators added into FP64 registers every 256 rows
//                 (FP32: per-lane FP64 sums; BF16x3: per split-K slice).
//                 Aligned FP32 rows are copied global -> LDS directly.
//  FP64:          v_mfma_f64_16x16x4f64.
#include <algorithm>
#include <cmath>
#include <string>

#include "bf16x3.hpp"
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
// 8 waves (4 x 2), each owning a 32 x 64 slice of the 128 x 128 tile: 32
// FP32 accumulators and their 32 FP64 running sums per lane.  This kernel
// takes rows of any stride and alignment (element loads with column
// guards); rows whose stride is a multiple of 4 floats at a 16-byte aligned
// base go to syrk_f32_direct_kernel below.
constexpr int NT32 = 512;
constexpr int BK32 = 32;

template <bool SCALED>
__global__ __launch_bounds__(NT32, 2) void syrk_f32_kernel(SyrkArgs a0, Batch bt) {
  __shared__ float As[2][BK32][BM];
  __shared__ float Bs[2][BK32][BM];

  SyrkArgs a;
  int64_t lid;
  if (!unit_of(a0, bt, a, lid)) return;
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

// FP32, rows 16-byte aligned: the same 128 x 128 tile and wave layout, with
// the X tiles copied global -> LDS by global_load_lds_dwordx4 (lane l of a
// wave writes bytes 16 l .. 16 l + 15 after the wave's LDS base, i.e. two
// 128-float rows per wave and instruction), so no loader registers are held
// across the MFMA block.  The per-row scale (zero for rows past the slice,
// whose loads are clamped to the last row) goes to a small LDS vector and
// multiplies the A operand as it is read.  About 120 VGPRs: four waves per
// SIMD, two workgroups per CU.
template <bool SCALED>
__global__ __launch_bounds__(NT32, 4) void syrk_f32_direct_kernel(SyrkArgs a0, Batch bt) {
  __shared__ __attribute__((aligned(16))) float As[2][BK32][BM];
  __shared__ __attribute__((aligned(16))) float Bs[2][BK32][BM];
  __shared__ float Ss[2][BK32];

  SyrkArgs a;
  int64_t lid;
  if (!unit_of(a0, bt, a, lid)) return;
  const int m = (int)(lid % a.L);
  const int t = (int)((lid / a.L) % a.n_tiles);
  const int s = (int)(lid / ((int64_t)a.L * a.n_tiles));
  int ti, tj;
  tile_coords(t, ti, tj);
  const int p0 = ti * BM, q0 = tj * BM;
  const int64_t r0 = (int64_t)s * a.rows_per_split;
  const int64_t r1 = min(r0 + a.rows_per_split, a.k_rows);
  const int nk = r1 > r0 ? (int)((r1 - r0 + BK32 - 1) / BK32) : 0;

  const float* X = static_cast<const float*>(a.X);
  const float* scale = SCALED ? static_cast<const float*>(a.scale) + (int64_t)m * a.k_rows : nullptr;
  const float csc = (float)a.cscale;

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wy = wave >> 1, wx = wave & 1;            // rows wy*32, cols wx*64
  // loader: wave w fills tile rows 2w + (lane >> 5) and 16 + 2w + (lane >> 5),
  // columns 4 (lane & 31) .. + 3 (clamped inside the row)
  const int lrow = 2 * wave + (lane >> 5);
  const int64_t ca = min(p0 + (lane & 31) * 4, (int)a.ld - 4);
  const int64_t cb = min(q0 + (lane & 31) * 4, (int)a.ld - 4);

  f32x16 acc[2];
  double acc64[2][16];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) { acc[j][r] = 0.f; acc64[j][r] = 0.0; }

  // Issue the copies of stage kb into buffer buf; threads 0..31 also fetch
  // the row scales into sreg (written to LDS before the next barrier).
  float sreg = 0.f;
  auto issue = [&](int64_t kb, int buf) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t rr = min(kb + lrow + 16 * h, r1 - 1);
      const float* row = X + rr * a.ld;
      __builtin_amdgcn_global_load_lds(row + ca, &As[buf][2 * wave + 16 * h][0], 16, 0, 0);
      __builtin_amdgcn_global_load_lds(row + cb, &Bs[buf][2 * wave + 16 * h][0], 16, 0, 0);
    }
    if (tid < BK32) {
      // a global (not flat) load, so it need not wait for the LDS copies
      const int64_t r = kb + tid;
      sreg = r < r1 ? (SCALED ? ((const __attribute__((address_space(1))) float*)scale)[r]
                              : csc)
                    : 0.f;
    }
  };
  auto publish = [&](int buf) {
    if (tid < BK32) Ss[buf][tid] = sreg;
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  };

  constexpr int FLUSH_STAGES = FLUSH_ROWS / BK32;
  if (nk > 0) {
    issue(r0, 0);
    publish(0);
  }
  const int arow = wy * 32 + (lane & 31);
  const int bcol = wx * 64 + (lane & 31);
  const int ksub = lane >> 5;
  for (int it = 0; it < nk; ++it) {
    const int cur = it & 1;
    if (it + 1 < nk) issue(r0 + (int64_t)(it + 1) * BK32, cur ^ 1);
    // operands of step kk + 1 are read while the MFMAs of step kk run; the
    // scheduling hint interleaves the LDS reads with the MFMA issue (the
    // default schedule waits on each read right before its MFMA)
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
constexpr int LDB = BKB;            // k stride (bf16) of an LDS row; 16-byte chunks XOR-swizzled
__device__ __forceinline__ int swz(int col, int k) { return (((k >> 3) ^ ((col >> 2) & 3)) << 3) | (k & 7); }

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
__global__ __launch_bounds__(NTB, 2) void syrk_bf16x3_kernel(SyrkArgs a0, Batch bt) {
  __shared__ __attribute__((aligned(16))) __bf16 Ah[2][BM][LDB];
  __shared__ __attribute__((aligned(16))) __bf16 Al[2][BM][LDB];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[2][BM][LDB];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[2][BM][LDB];

  SyrkArgs a;
  int64_t lid;
  if (!unit_of(a0, bt, a, lid)) return;
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
      const int ks = swz(lcol + c, krow);
      *reinterpret_cast<bf16x4*>(&Ah[buf][lcol + c][ks]) = v;
      v = bf16x4{al[0][c], al[1][c], al[2][c], al[3][c]};
      *reinterpret_cast<bf16x4*>(&Al[buf][lcol + c][ks]) = v;
      v = bf16x4{bh[0][c], bh[1][c], bh[2][c], bh[3][c]};
      *reinterpret_cast<bf16x4*>(&Bh[buf][lcol + c][ks]) = v;
      v = bf16x4{bl[0][c], bl[1][c], bl[2][c], bl[3][c]};
      *reinterpret_cast<bf16x4*>(&Bl[buf][lcol + c][ks]) = v;
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
        const int ka = swz(pr, ks + kl), kb2 = swz(qc, ks + kl);
        ahf[i] = *reinterpret_cast<const bf16x8*>(&Ah[cur][pr][ka]);
        alf[i] = *reinterpret_cast<const bf16x8*>(&Al[cur][pr][ka]);
        bhf[i] = *reinterpret_cast<const bf16x8*>(&Bh[cur][qc][kb2]);
        blf[i] = *reinterpret_cast<const bf16x8*>(&Bl[cur][qc][kb2]);
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

// ------------------------------------------------------- BF16x3, pre-split
// The scaled rows are split once per call into workspace: Y_m[P][r] =
// sqrt(s_m(r)) X[r][P] as BF16 hi and lo, transposed into blocks of 32 k
// (rows r of X), each block [Npad][32], so the pipeline stage of any tile is
// one contiguous range of the block (whole DRAM pages, few TLB entries);
// then M^m = Y_m Y_m^T is a plain BF16x3 SYRK over tiles copied global ->
// LDS directly (bf16x3.hpp).  The square root splits the positive scale
// evenly over both operands.
struct ChiSplitArgs {
  const float* X;       // rows r_base .. r_base + k_rows - 1 of [k_total][ld]
  int64_t ld;
  int64_t k_rows;       // rows of this chunk
  int N;
  int L;
  const float* scale;   // [L][k_total] or nullptr (constant cscale)
  float cscale;
  int64_t k_total;
  int64_t r_base;
  __bf16* hi;           // [L][kp / 32][Npad][32]: k blocks of 32, each [row][k]
  __bf16* lo;
  int64_t kp;           // k extent of Y (rows of the chunk rounded up to 32)
  int Npad;
};

// 64 rows x 64 columns of X per workgroup, read once, written for every m
// (Y rows start 16-byte aligned: Npad and kp are multiples of 32).
__global__ __launch_bounds__(256) void chi_split_kernel(ChiSplitArgs a) {
  __shared__ float tile[64][65];
  __shared__ float sq[32][64];
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int p0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int y = ty; y < 64; y += 4) {
    const int64_t r = r0 + y;
    const int P = p0 + tx;
    tile[y][tx] = (r < a.k_rows && P < a.N) ? a.X[(a.r_base + r) * a.ld + P] : 0.f;
  }
  const int64_t mstride = (int64_t)a.Npad * a.kp;
  // the square-rooted scales of 32 points at a time
  for (int m0 = 0; m0 < a.L; m0 += 32) {
    const int nm = min(32, a.L - m0);
    __syncthreads();
    for (int idx = threadIdx.x; idx < nm * 64; idx += 256) {
      const int m = idx >> 6, y = idx & 63;
      const int64_t r = r0 + y;
      float v = 0.f;
      if (r < a.k_rows)
        v = a.scale ? a.scale[(int64_t)(m0 + m) * a.k_total + a.r_base + r] : a.cscale;
      sq[m][y] = sqrtf(v);
    }
    __syncthreads();
    // 16-byte stores of 8 consecutive k: thread t writes row P = t / 4, k
    // r0 + 32 h + 8 (t % 4) .. + 7 of k block h, so a wave writes 1 KB of
    // one block contiguously
    const int P = threadIdx.x >> 2, q = threadIdx.x & 3;
    for (int m = 0; m < nm; ++m) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int y0 = 32 * h + 8 * q;
        const int64_t r = r0 + y0;
        if (r >= a.kp) continue;
        b3::bf16x8 vh, vl;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          __bf16 hh, ll;
          b3::split(tile[y0 + e][P] * sq[m][y0 + e], hh, ll);
          vh[e] = hh;
          vl[e] = ll;
        }
        const int64_t o = (m0 + m) * mstride + (r >> 5) * ((int64_t)a.Npad * 32) +
                          (int64_t)(p0 + P) * 32 + (r & 31);
        *reinterpret_cast<b3::bf16x8*>(a.hi + o) = vh;
        *reinterpret_cast<b3::bf16x8*>(a.lo + o) = vl;
      }
    }
  }
}

struct Syrk3Args {
  const __bf16* hi;     // [L][kp / 32][Npad][32]
  const __bf16* lo;
  int64_t kp;
  int Npad;
  int L, n_tiles, splits;
  int64_t rows_per_split;   // multiple of FLUSH_ROWS
  double* part;         // [splits][L][n_tiles][BM*BM]
  int T;                // 128-row tiles of N (n_tiles = T (T + 1) / 2)
};

// Work units: tile fastest, then Laplace point, then split-K slice, so the
// tiles that read one slice of one Y_m run together on one XCD.
// Accumulation is blocked: the MFMA accumulators sum FLUSH_ROWS rows, then
// are added into a second FP32 sum per element, so an entry's rounding
// error is bounded by gamma(FLUSH_ROWS + blocks) (blocked summation).
// Shapes (the autotuner picks one): 4 waves of 64 x 64 with 2 stages of LDS
// (two workgroups per CU) or 3 stages (one workgroup per CU, the copies of
// stage it + 2 in flight while stage it is multiplied), or 8 waves of
// 64 x 32 with 2 stages (two workgroups, four waves per SIMD).  Stage
// hand-over: wait for this wave's copies of the next stage (those of later
// stages may stay in flight) and its LDS reads, then a plain s_barrier (a
// __syncthreads() would also wait for every copy still in flight).
template <int NBUF, int MINB, int NW>
__global__ __launch_bounds__(NW * 64, MINB) void syrk_bf16x3_direct_kernel(Syrk3Args a) {
  constexpr int BKT = 32;
  constexpr int WI = 2, WJ = NW == 4 ? 2 : 1;          // 32 x 32 blocks per wave
  constexpr int LOADS = 4 * BM / (64 / (BKT / 8)) / NW;  // copies per wave per stage
  static_assert(NBUF == 2 || (NBUF == 3 && LOADS == 8), "three stages: 4 waves only");
  __shared__ __attribute__((aligned(16))) b3::StageT<BKT> st[NBUF];
  const int64_t lid = xcd_remap(blockIdx.x, gridDim.x);
  const int t = (int)(lid % a.n_tiles);
  const int m = (int)((lid / a.n_tiles) % a.L);
  const int s = (int)(lid / ((int64_t)a.n_tiles * a.L));
  int ti, tj;
  tile_coords(t, ti, tj);
  const int64_t p0 = (int64_t)ti * BM, q0 = (int64_t)tj * BM;
  const int64_t r0 = (int64_t)s * a.rows_per_split;
  const int64_t r1 = min(r0 + a.rows_per_split, a.kp);
  const int nk = r1 > r0 ? (int)((r1 - r0) / BKT) : 0;
  const int64_t mo = (int64_t)m * a.Npad * a.kp;
  const __bf16* hi = a.hi + mo;
  const __bf16* lo = a.lo + mo;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int ar = (NW == 4 ? (wave >> 1) : (wave >> 2)) * 64;   // first A (P) row of the wave
  const int br = NW == 4 ? (wave & 1) * 64 : (wave & 3) * 32;  // first B (Q) row

  f32x16 acc[WI][WJ], sum[WI][WJ];
#pragma unroll
  for (int i = 0; i < WI; ++i)
#pragma unroll
    for (int j = 0; j < WJ; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) { acc[i][j][r] = 0.f; sum[i][j][r] = 0.f; }

  auto issue = [&](int it) {
    const int64_t kb = r0 + (int64_t)it * BKT;
    const __bf16* his = hi + kb * a.Npad;          // k block kb / BKT: [Npad][BKT]
    const __bf16* los = lo + kb * a.Npad;
    b3::StageT<BKT>& d = st[it % NBUF];
    b3::load_tile<BKT, NW>(his, BKT, p0, 0, d.t[0], wave, lane);
    b3::load_tile<BKT, NW>(los, BKT, p0, 0, d.t[1], wave, lane);
    b3::load_tile<BKT, NW>(his, BKT, q0, 0, d.t[2], wave, lane);
    b3::load_tile<BKT, NW>(los, BKT, q0, 0, d.t[3], wave, lane);
  };
  auto handover = [&](int it) {   // after stage it: stage it + 1 visible to all waves
    if (NBUF == 3 && it + 2 < nk)
      asm volatile("s_waitcnt vmcnt(8) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    else
      asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
  };
  constexpr int FLUSH_STAGES = FLUSH_ROWS / BKT;
  for (int it = 0; it < NBUF - 1 && it < nk; ++it) issue(it);
  handover(-1);
  for (int blk = 0; blk < nk; blk += FLUSH_STAGES) {
    const int end = min(blk + FLUSH_STAGES, nk);
    for (int it = blk; it < end; ++it) {
      if (it + NBUF - 1 < nk) issue(it + NBUF - 1);
      b3::stage_mfma<BKT, WI, WJ>(st[it % NBUF], acc, ar, br, lane);
      handover(it);
    }
#pragma unroll
    for (int i = 0; i < WI; ++i)
#pragma unroll
      for (int j = 0; j < WJ; ++j) {
        sum[i][j] += acc[i][j];
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
      }
  }

  double* out = a.part + (((int64_t)s * a.L + m) * a.n_tiles + t) * (BM * BM);
#pragma unroll
  for (int i = 0; i < WI; ++i)
#pragma unroll
    for (int j = 0; j < WJ; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = ar + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int col = br + j * 32 + (lane & 31);
        out[row * BM + col] = (double)sum[i][j][r];
      }
}

// Wide shape: 256 rows of P x 128 rows of Q per workgroup, 8 waves of
// 64 x 64 (two per SIMD), one workgroup per CU, three LDS stages of 48 KB.
// The CU copies 48 KB of operands into LDS per 2^21 MFMA flops, against
// 64 KB in the 128 x 128 shapes (two workgroups of 32 KB per 2^20).  The
// operand fragments are software-pipelined through two register sets: the
// LDS reads of k step t + 1 are issued before the MFMAs of step t, and the
// stage hand-over sits between the last reads of a stage and the first reads
// of the next.
// Units per (slice, point): 256-row tile rows I2 and 128-column tile
// columns J < min(2 I2 + 2, T); the two 128 x 128 halves of a unit are the
// lower tiles (2 I2, J) (when J <= 2 I2) and (2 I2 + 1, J) (when
// 2 I2 + 1 < T) of the partial layout.  The waves of a half that is not a
// lower tile, and the wave of the upper 64 x 64 block of a diagonal tile,
// only take part in the copies and barriers, so the other wave on their
// SIMD runs alone.  Each accumulator sees the same product order as in the
// 128 x 128 shapes.  Needs the split rows padded to a multiple of 256.
__global__ __launch_bounds__(512, 1) void syrk_bf16x3_wide_kernel(Syrk3Args a) {
  constexpr int NBUF = 3, BKT = 32, WI = 2, WJ = 2;
  struct WideStage {
    __bf16 a[2][2 * BM * BKT];   // hi, lo of 256 P rows (two swizzled 128-row tiles)
    __bf16 b[2][BM * BKT];       // hi, lo of 128 Q rows
  };
  struct Frag {
    b3::bf16x8 ah[WI], al[WI], bh[WJ], bl[WJ];
  };
  __shared__ __attribute__((aligned(16))) WideStage st[NBUF];
  const int T = a.T, T2 = (a.T + 1) / 2;
  int per = 0;                                   // units per (slice, point)
  for (int i = 0; i < T2; ++i) per += min(2 * i + 2, T);
  const int64_t lid = xcd_remap(blockIdx.x, gridDim.x);
  const int u = (int)(lid % per);
  const int m = (int)((lid / per) % a.L);
  const int s = (int)(lid / ((int64_t)per * a.L));
  int I2 = 0, J = u;
  while (J >= min(2 * I2 + 2, T)) {
    J -= min(2 * I2 + 2, T);
    ++I2;
  }
  const int64_t p0 = (int64_t)I2 * 2 * BM, q0 = (int64_t)J * BM;
  const int64_t r0 = (int64_t)s * a.rows_per_split;
  const int64_t r1 = min(r0 + a.rows_per_split, a.kp);
  const int nk = r1 > r0 ? (int)((r1 - r0) / BKT) : 0;
  const int64_t mo = (int64_t)m * a.Npad * a.kp;
  const __bf16* hi = a.hi + mo;
  const __bf16* lo = a.lo + mo;
  // the wave index as a scalar, so the idle-half branches are scalar branches
  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1;       // P rows 64 wr .., Q rows 64 wc ..
  const int half = wr >> 1;                      // the 128-row half of P of the wave
  const int ti = 2 * I2 + half;                  // its tile row
  // idle: not a lower tile, or the wholly upper 64 x 64 block of a diagonal
  // tile (the reduction reads only the lower triangle)
  const bool idle = ti >= T || J > ti || (J == ti && (wr & 1) == 0 && wc == 1);

  f32x16 acc[WI][WJ], sum[WI][WJ];
#pragma unroll
  for (int i = 0; i < WI; ++i)
#pragma unroll
    for (int j = 0; j < WJ; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) { acc[i][j][r] = 0.f; sum[i][j][r] = 0.f; }

  // one copy instruction per wave per 128-row tile, 6 per stage
  auto issue = [&](int it) {
    const int64_t kb = r0 + (int64_t)it * BKT;
    const __bf16* his = hi + kb * a.Npad;          // k block kb / BKT: [Npad][BKT]
    const __bf16* los = lo + kb * a.Npad;
    WideStage& d = st[it % NBUF];
    b3::load_tile<BKT, 8>(his, BKT, p0, 0, d.a[0], wave, lane);
    b3::load_tile<BKT, 8>(his, BKT, p0 + BM, 0, d.a[0] + BM * BKT, wave, lane);
    b3::load_tile<BKT, 8>(los, BKT, p0, 0, d.a[1], wave, lane);
    b3::load_tile<BKT, 8>(los, BKT, p0 + BM, 0, d.a[1] + BM * BKT, wave, lane);
    b3::load_tile<BKT, 8>(his, BKT, q0, 0, d.b[0], wave, lane);
    b3::load_tile<BKT, 8>(los, BKT, q0, 0, d.b[1], wave, lane);
  };
  // at the hand-over of stage it + 1 the copies of stage it + 2 may stay in
  // flight
  auto handover = [&](int it) {
    if (it + 2 < nk)
      asm volatile("s_waitcnt vmcnt(6) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    else
      asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
  };
  if (idle) {   // copies and the same barriers as the other waves, nothing else
    if (nk > 0) {
      issue(0);
      if (nk > 1) issue(1);
      handover(-1);
    }
    for (int it = 0; it + 1 < nk; ++it) {
      if (it + 2 < nk) issue(it + 2);
      handover(it);
    }
    return;
  }
  auto read = [&](Frag& f, const WideStage& d, int ks) {
    const int kc = 2 * ks + (lane >> 5);
#pragma unroll
    for (int i = 0; i < WI; ++i) {
      f.ah[i] = b3::frag<BKT>(d.a[0] + wr * 64 * BKT, i * 32 + (lane & 31), kc);
      f.al[i] = b3::frag<BKT>(d.a[1] + wr * 64 * BKT, i * 32 + (lane & 31), kc);
    }
#pragma unroll
    for (int j = 0; j < WJ; ++j) {
      f.bh[j] = b3::frag<BKT>(d.b[0], wc * 64 + j * 32 + (lane & 31), kc);
      f.bl[j] = b3::frag<BKT>(d.b[1], wc * 64 + j * 32 + (lane & 31), kc);
    }
  };
  // hi*hi, then hi*lo, then lo*hi into every accumulator
  auto mma = [&](const Frag& f) {
#pragma unroll
    for (int i = 0; i < WI; ++i)
#pragma unroll
      for (int j = 0; j < WJ; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.ah[i], f.bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < WI; ++i)
#pragma unroll
      for (int j = 0; j < WJ; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.ah[i], f.bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < WI; ++i)
#pragma unroll
      for (int j = 0; j < WJ; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.al[i], f.bh[j], acc[i][j], 0, 0, 0);
  };
  auto flush = [&]() {
#pragma unroll
    for (int i = 0; i < WI; ++i)
#pragma unroll
      for (int j = 0; j < WJ; ++j) {
        sum[i][j] += acc[i][j];
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
      }
  };
  constexpr int FLUSH_STAGES = FLUSH_ROWS / BKT;
  Frag f0, f1;
  if (nk > 0) {
    issue(0);
    if (nk > 1) issue(1);
    handover(-1);
    read(f0, st[0], 0);
  }
  // all stages but the last: no branch between the reads of the next stage
  // and the MFMAs of this one, so the waits before those MFMAs cover only
  // their own reads
  for (int it = 0; it + 1 < nk; ++it) {
    if (it + 2 < nk) issue(it + 2);     // buffer of stage it - 1: free since its hand-over
    read(f1, st[it % NBUF], 1);
    mma(f0);
    handover(it);
    read(f0, st[(it + 1) % NBUF], 0);
    mma(f1);
    if ((it + 1) % FLUSH_STAGES == 0) flush();
  }
  if (nk > 0) {
    read(f1, st[(nk - 1) % NBUF], 1);
    mma(f0);
    mma(f1);
    flush();
  }
  const int t = ti * (ti + 1) / 2 + J;
  double* out = a.part + (((int64_t)s * a.L + m) * a.n_tiles + t) * (BM * BM);
#pragma unroll
  for (int i = 0; i < WI; ++i)
#pragma unroll
    for (int j = 0; j < WJ; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = (wr & 1) * 64 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int col = wc * 64 + j * 32 + (lane & 31);
        out[row * BM + col] = (double)sum[i][j][r];
      }
}

// ------------------------------------------------------------------ FP64 MFMA
constexpr int BK64 = 16;

__global__ __launch_bounds__(NT, 1) void syrk_f64_kernel(SyrkArgs a0, Batch bt) {
  __shared__ double As[2][BK64][BM];
  __shared__ double Bs[2][BK64][BM];

  SyrkArgs a;
  int64_t lid;
  if (!unit_of(a0, bt, a, lid)) return;
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
struct RedArgs {
  const double* part;   // [splits][L][n_tiles][BM*BM]
  int splits, L, n_tiles, N;
  double* out;          // [L][N][N]
  int accumulate;
};

__device__ __forceinline__ void reduce_elem(const RedArgs& r, int64_t idx) {
  const int64_t per_tile = BM * BM;
  if (idx >= (int64_t)r.L * r.n_tiles * per_tile) return;
  const int e = (int)(idx % per_tile);
  const int t = (int)((idx / per_tile) % r.n_tiles);
  const int m = (int)(idx / (per_tile * r.n_tiles));
  int ti, tj;
  tile_coords(t, ti, tj);
  const int p = ti * BM + e / BM, q = tj * BM + e % BM;
  if (p >= r.N || q >= r.N || q > p) return;
  double v = 0.0;
  for (int s = 0; s < r.splits; ++s)
    v += r.part[(((int64_t)s * r.L + m) * r.n_tiles + t) * per_tile + e];
  double* dst = r.out + ((int64_t)m * r.N + p) * r.N + q;
  *dst = r.accumulate ? *dst + v : v;
}

__global__ void syrk_reduce_kernel(RedArgs r) {
  const int64_t total = (int64_t)r.L * r.n_tiles * BM * BM;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x)
    reduce_elem(r, idx);
}

__global__ void syrk_reduce_batched_kernel(Batch bt) {
  RedArgs r;
  int64_t first;
  if (!block_of(bt, r, first)) return;
  for (int e = 0; e < kBatchElems; e += 256) reduce_elem(r, first + e + threadIdx.x);
}

struct MirArgs {
  double* M;
  int L, N;
};

__device__ __forceinline__ void mirror_elem(const MirArgs& a, int64_t idx) {
  if (idx >= (int64_t)a.L * a.N * a.N) return;
  const int q = (int)(idx % a.N);
  const int p = (int)((idx / a.N) % a.N);
  const int64_t m = idx / ((int64_t)a.N * a.N);
  if (q > p) a.M[(m * a.N + p) * a.N + q] = a.M[(m * a.N + q) * a.N + p];
}

__global__ void mirror_kernel(MirArgs a) {
  const int64_t total = (int64_t)a.L * a.N * a.N;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x)
    mirror_elem(a, idx);
}

__global__ void mirror_batched_kernel(Batch bt) {
  MirArgs a;
  int64_t first;
  if (!block_of(bt, a, first)) return;
  for (int e = 0; e < kBatchElems; e += 256) mirror_elem(a, first + e + threadIdx.x);
}

// s_m(ia) = w_m D_ia exp(-D_ia^2 x_m) for every Laplace point and pair.
struct ScaleArgs {
  int L;
  const double* x;
  const double* w;
  int n_i, n_virt;
  const double* eps_i;
  const double* eps_a;
  void* out;            // [L][n_i * n_virt], FP64 or FP32
  int sos;              // 0: Laplace factors (x, w); 1: D / (x^2 + D^2), x = frequencies
};

template <typename T>
__device__ __forceinline__ void scale_elem(const ScaleArgs& s, int64_t idx) {
  const int64_t k = (int64_t)s.n_i * s.n_virt;
  if (idx >= k * s.L) return;
  const int64_t r = idx % k;
  const int m = (int)(idx / k);
  const int i = (int)(r / s.n_virt), aa = (int)(r % s.n_virt);
  const double d = s.eps_a[aa] - s.eps_i[i];
  const double v = s.sos ? d / (s.x[m] * s.x[m] + d * d) : s.w[m] * d * exp(-d * d * s.x[m]);
  static_cast<T*>(s.out)[idx] = (T)v;
}

template <typename T>
__global__ void lt_scale_kernel(ScaleArgs s) {
  const int64_t total = (int64_t)s.n_i * s.n_virt * s.L;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x)
    scale_elem<T>(s, idx);
}

template <typename T>
__global__ void lt_scale_batched_kernel(Batch bt) {
  ScaleArgs s;
  int64_t first;
  if (!block_of(bt, s, first)) return;
  for (int e = 0; e < kBatchElems; e += 256) scale_elem<T>(s, first + e + threadIdx.x);
}

inline int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  return (int)std::min<int64_t>(std::max<int64_t>(g, 1), 65536);
}

}  // namespace

namespace gw {

gw_status lt_scale_launch(gw_ctx ctx, gw_precision prec, int L, const double* d_x,
                          const double* d_w, int n_i, int n_virt,
                          const double* d_eps_i, const double* d_eps_a, void* scale,
                          int sos) {
  const int64_t n = (int64_t)L * n_i * n_virt;
  const ScaleArgs sa{L, d_x, d_w, n_i, n_virt, d_eps_i, d_eps_a, scale, sos};
  if (prec == GW_FP64)
    hipLaunchKernelGGL(lt_scale_kernel<double>, dim3(grid_for(n, 256)), dim3(256), 0,
                       ctx->stream, sa);
  else
    hipLaunchKernelGGL(lt_scale_kernel<float>, dim3(grid_for(n, 256)), dim3(256), 0,
                       ctx->stream, sa);
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

static int64_t split_align(gw_precision prec) {
  return prec == GW_FP64 ? BK64 : (prec == GW_BF16X3 ? BKB : FLUSH_ROWS);
}

static void launch_syrk_kernel(gw_ctx ctx, gw_precision prec, bool fast, bool scaled,
                               const SyrkArgs& a, const Batch& bt, int64_t grid) {
  if (prec == GW_FP64) {
    hipLaunchKernelGGL(syrk_f64_kernel, dim3((unsigned)grid), dim3(NT), 0, ctx->stream, a, bt);
  } else if (prec == GW_BF16X3) {
    auto kern = fast ? (scaled ? syrk_bf16x3_kernel<true, true> : syrk_bf16x3_kernel<true, false>)
                     : (scaled ? syrk_bf16x3_kernel<false, true> : syrk_bf16x3_kernel<false, false>);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(NTB), 0, ctx->stream, a, bt);
  } else {
    auto kern = fast ? (scaled ? syrk_f32_direct_kernel<true> : syrk_f32_direct_kernel<false>)
                     : (scaled ? syrk_f32_kernel<true> : syrk_f32_kernel<false>);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(NT32), 0, ctx->stream, a, bt);
  }
}

static bool fast_rows(gw_precision prec, const void* X, int64_t ld) {
  return prec != GW_FP64 && (ld % 4 == 0) && ld >= 4 &&
         (reinterpret_cast<uintptr_t>(X) % 16 == 0);
}

// Bytes of split rows one chunk of the BF16x3 path may hold (hi + lo of all
// Laplace points); longer row ranges are processed in chunks.
constexpr size_t kSplitChunkBytes = size_t(16) << 30;

static int64_t split_chunk_rows(int64_t k_rows, int Npad, int L) {
  const int64_t per_row = (int64_t)L * Npad * 2 * (int64_t)sizeof(__bf16);
  int64_t kc = (int64_t)(kSplitChunkBytes / per_row) / FLUSH_ROWS * FLUSH_ROWS;
  kc = std::max<int64_t>(kc, FLUSH_ROWS);
  return std::min<int64_t>(kc, (k_rows + b3::BK - 1) / b3::BK * b3::BK);
}

// BF16x3 scaled SYRK with the operand split once per chunk of rows.
static gw_status syrk_bf16x3_split(gw_ctx ctx, const float* X, int64_t k_rows, int N,
                                   int64_t ld, int L, const float* scale, double cscale,
                                   double* out, int accumulate, const char* prof_name) {
  static_assert(b3::BK == 32, "the split layout blocks k by 32, one stage of every shape");
  const int T = (N + BM - 1) / BM;
  const int Npad = (N + 2 * BM - 1) / (2 * BM) * (2 * BM);   // the wide shapes' 256-row tiles
  const int n_tiles = T * (T + 1) / 2;
  int wide_units = 0;
  for (int i = 0; i < (T + 1) / 2; ++i) wide_units += std::min(2 * i + 2, T);
  const int64_t kc = split_chunk_rows(k_rows, Npad, L);
  const size_t y_elems = (size_t)L * Npad * kc;
  __bf16* Y = static_cast<__bf16*>(ws_get(ctx, WS_B3_CHI, 2 * y_elems * sizeof(__bf16)));
  if (!Y) return GW_ENOMEM;
  const int S0 = choose_splits(kc, (int64_t)n_tiles * L);
  std::vector<int> cand{S0};
  if (S0 > 1) cand.push_back(std::max(1, S0 / 2));
  if (2 * S0 <= 16 && kc / (2 * S0) >= 1024) cand.push_back(2 * S0);
  const int S_max = *std::max_element(cand.begin(), cand.end());
  double* part = static_cast<double*>(
      ws_get(ctx, WS_SYRK_PART, (size_t)S_max * L * n_tiles * BM * BM * sizeof(double)));
  if (!part) return GW_ENOMEM;
  for (int64_t c0 = 0; c0 < k_rows; c0 += kc) {
    const int64_t kr = std::min(kc, k_rows - c0);
    const int64_t kp = (kr + b3::BK - 1) / b3::BK * b3::BK;
    const ChiSplitArgs sa{X, ld, kr, N, L, scale, (float)cscale, k_rows, c0, Y,
                          Y + (size_t)L * Npad * kp, kp, Npad};
    const int ps = prof_begin(ctx);
    hipLaunchKernelGGL(chi_split_kernel, dim3((unsigned)((kp + 63) / 64), (unsigned)(Npad / 64)),
                       dim3(256), 0, ctx->stream, sa);
    prof_end(ctx, ps, "chi_split_bf16x3", 0.0,
             (double)kr * N * 4.0 + (double)L * Npad * kp * 4.0);
    GW_TRY(launch_check(ctx, "chi_split_kernel"));
    auto args = [&](int S) {
      int64_t rps = (kp + S - 1) / S;
      rps = (rps + FLUSH_ROWS - 1) / FLUSH_ROWS * FLUSH_ROWS;
      const int Se = (int)((kp + rps - 1) / rps);
      return Syrk3Args{sa.hi, sa.lo, kp, Npad, L, n_tiles, Se, rps, part, T};
    };
    // candidates: split-K factor x kernel shape, encoded as 4 S + shape
    // (128 x 128 tiles: 0: 4 waves, 2 stages; 1: 4 waves, 3 stages; 2: 8
    // waves, 2 stages; 3: 256 x 128 tiles, 8 waves, 3 stages)
    auto launch = [&](int code) {
      const Syrk3Args a = args(code / 4);
      const dim3 grid((unsigned)((int64_t)a.splits * L * n_tiles));
      const dim3 wgrid((unsigned)((int64_t)a.splits * L * wide_units));
      switch (code % 4) {
        case 3:
          hipLaunchKernelGGL(syrk_bf16x3_wide_kernel, wgrid, dim3(512), 0, ctx->stream, a);
          break;
        case 1:
          hipLaunchKernelGGL((syrk_bf16x3_direct_kernel<3, 1, 4>), grid, dim3(256), 0,
                             ctx->stream, a);
          break;
        case 2:
          hipLaunchKernelGGL((syrk_bf16x3_direct_kernel<2, 2, 8>), grid, dim3(512), 0,
                             ctx->stream, a);
          break;
        default:
          hipLaunchKernelGGL((syrk_bf16x3_direct_kernel<2, 2, 4>), grid, dim3(256), 0,
                             ctx->stream, a);
      }
      return launch_check(ctx, "syrk_bf16x3_direct_kernel");
    };
    std::vector<int> codes;
    for (int c : cand)
      for (int shape = 0; shape < 4; ++shape) codes.push_back(4 * c + shape);
    const std::string key = "syrk3:" + std::to_string(N) + ":" + std::to_string(L) + ":" +
                            std::to_string(kp);
    const int code = tune(ctx, key, codes, launch);
    const Syrk3Args a = args(code / 4);
    const int pi = prof_begin(ctx);
    GW_TRY(launch(code));
    prof_end(ctx, pi, prof_name, (double)L * N * (N + 1.0) * (double)kr,
             (double)L * Npad * kp * 4.0 + (double)L * N * (N + 1.0) / 2.0 * 8.0);
    const int64_t tot = (int64_t)L * n_tiles * BM * BM;
    const RedArgs r{part, a.splits, L, n_tiles, N, out, (accumulate || c0 > 0) ? 1 : 0};
    hipLaunchKernelGGL(syrk_reduce_kernel, dim3(grid_for(tot, 256)), dim3(256), 0, ctx->stream,
                       r);
    GW_TRY(launch_check(ctx, "syrk_reduce_kernel"));
  }
  return GW_OK;
}

gw_status syrk_launch(gw_ctx ctx, gw_precision prec, const void* X, int64_t k_rows,
                      int N, int64_t ld, int L, const void* scale, double cscale,
                      double* out, int accumulate, const char* prof_name) {
  if (prec == GW_BF16X3 && k_rows > 0)
    return syrk_bf16x3_split(ctx, static_cast<const float*>(X), k_rows, N, ld, L,
                             static_cast<const float*>(scale), cscale, out, accumulate,
                             prof_name);
  const int T = (N + BM - 1) / BM;
  const int n_tiles = T * (T + 1) / 2;
  const int S0 = k_rows > 0 ? choose_splits(k_rows, (int64_t)n_tiles * L) : 1;
  // split-K candidates around the occupancy-based choice (autotuned per shape)
  std::vector<int> cand{S0};
  if (S0 > 1) cand.push_back(std::max(1, S0 / 2));
  if (2 * S0 <= 16 && k_rows / (2 * S0) >= 1024) cand.push_back(2 * S0);
  const int S_max = *std::max_element(cand.begin(), cand.end());
  const int64_t align = split_align(prec);
  double* part = static_cast<double*>(
      ws_get(ctx, WS_SYRK_PART, (size_t)S_max * L * n_tiles * BM * BM * sizeof(double)));
  if (!part) return GW_ENOMEM;
  const bool fast = fast_rows(prec, X, ld);
  auto args = [&](int S) {
    int64_t rps = (k_rows + S - 1) / S;
    rps = (rps + align - 1) / align * align;
    return SyrkArgs{X, k_rows, N, ld, L, scale, cscale, T, n_tiles, S, rps, part};
  };
  const std::string key = "syrk:" + std::to_string((int)prec) + ":" + std::to_string(N) + ":" +
                          std::to_string(L) + ":" + std::to_string(k_rows) + ":" +
                          std::to_string(scale != nullptr) + std::to_string(fast);
  const int S = k_rows > 0 ? tune(ctx, key, cand, [&](int c) {
    launch_syrk_kernel(ctx, prec, fast, scale != nullptr, args(c), Batch{},
                       (int64_t)c * L * n_tiles);
    return launch_check(ctx, "syrk kernel");
  }) : 1;
  const SyrkArgs a = args(S);
  const int64_t grid = (int64_t)S * L * n_tiles;
  const int pi = prof_begin(ctx);
  launch_syrk_kernel(ctx, prec, fast, scale != nullptr, a, Batch{}, grid);
  // algorithmic work: L lower-triangle products of 2 k flops each; X read
  // once, the triangle written once
  const double esz = prec == GW_FP64 ? 8.0 : 4.0;
  prof_end(ctx, pi, prof_name,
           (double)L * N * (N + 1.0) * (double)k_rows,
           (double)k_rows * N * esz + (double)L * N * (N + 1.0) / 2.0 * 8.0);
  GW_TRY(launch_check(ctx, "syrk kernel"));
  const int64_t tot = (int64_t)L * n_tiles * BM * BM;
  const RedArgs r{part, S, L, n_tiles, N, out, accumulate};
  hipLaunchKernelGGL(syrk_reduce_kernel, dim3(grid_for(tot, 256)), dim3(256), 0, ctx->stream, r);
  return launch_check(ctx, "syrk_reduce_kernel");
}

gw_status mirror_lower(gw_ctx ctx, double* M, int L, int N) {
  const int64_t tot = (int64_t)L * N * N;
  hipLaunchKernelGGL(mirror_kernel, dim3(grid_for(tot, 256)), dim3(256), 0, ctx->stream,
                     MirArgs{M, L, N});
  return launch_check(ctx, "mirror_kernel");
}

// ------------------------------------------------------------------ batched

gw_status lt_scale_batched(gw_ctx ctx, gw_precision prec, const std::vector<ScaleJob>& jobs) {
  std::vector<ScaleArgs> d;
  std::vector<int64_t> n;
  for (const ScaleJob& j : jobs) {
    d.push_back(ScaleArgs{j.L, j.x, j.w, j.n_i, j.n_virt, j.eps_i, j.eps_a, j.out, 0});
    n.push_back((int64_t)j.L * j.n_i * j.n_virt);
  }
  return elementwise_batched(ctx, d, n, prec == GW_FP64 ? lt_scale_batched_kernel<double>
                                                        : lt_scale_batched_kernel<float>,
                             "lt_scale_batched_kernel");
}

gw_status mirror_lower_batched(gw_ctx ctx, const std::vector<MirrorJob>& jobs) {
  std::vector<MirArgs> d;
  std::vector<int64_t> n;
  for (const MirrorJob& j : jobs) {
    d.push_back(MirArgs{j.M, j.L, j.N});
    n.push_back((int64_t)j.L * j.N * j.N);
  }
  return elementwise_batched(ctx, d, n, mirror_batched_kernel, "mirror_batched_kernel");
}

// All jobs' tiles in one launch.  Jobs must agree on whether they carry a
// per-row scale.  Split-K: a job's rows are split so that no work unit is
// much longer than twice the mean, and the descriptors are ordered by unit
// length, longest first, so the long units start first.
gw_status syrk_batched_launch(gw_ctx ctx, gw_precision prec, const std::vector<SyrkJob>& jobs,
                              const char* prof_name) {
  if (jobs.empty()) return GW_OK;
  const bool scaled = jobs[0].scale != nullptr;
  double w_units = 0, w_rows = 0;
  for (const SyrkJob& j : jobs) {
    if ((j.scale != nullptr) != scaled)
      return fail(ctx, GW_EINVAL, "batched SYRK: jobs mix scaled and unscaled rows");
    const int T = (j.N + BM - 1) / BM;
    const double u = (double)j.L * T * (T + 1) / 2;
    w_units += u;
    w_rows += u * (double)j.k_rows;
  }
  const int64_t align = split_align(prec);
  const int64_t target = std::max<int64_t>(4096, (int64_t)(2.0 * w_rows / std::max(w_units, 1.0)));
  struct Item { SyrkArgs a; RedArgs r; int64_t units; };
  std::vector<Item> items;
  size_t part_total = 0;
  bool fast = true;
  for (const SyrkJob& j : jobs) {
    const int T = (j.N + BM - 1) / BM;
    const int n_tiles = T * (T + 1) / 2;
    const int S = (int)std::min<int64_t>(16, std::max<int64_t>(1, (j.k_rows + target - 1) / target));
    int64_t rps = (j.k_rows + S - 1) / S;
    rps = std::max<int64_t>(align, (rps + align - 1) / align * align);
    Item it;
    it.a = SyrkArgs{j.X, j.k_rows, j.N, j.ld, j.L, j.scale, j.cscale, T, n_tiles, S, rps,
                    reinterpret_cast<double*>(part_total)};
    it.r = RedArgs{nullptr, S, j.L, n_tiles, j.N, j.out, j.accumulate};
    it.units = (int64_t)S * j.L * n_tiles;
    part_total += (size_t)it.units * BM * BM;
    fast = fast && (j.k_rows == 0 || fast_rows(prec, j.X, j.ld));
    items.push_back(it);
  }
  double* part = static_cast<double*>(ws_get(ctx, WS_SYRK_PART, part_total * sizeof(double)));
  if (!part) return GW_ENOMEM;
  for (Item& it : items) {
    it.a.part = part + reinterpret_cast<size_t>(it.a.part);
    it.r.part = it.a.part;
  }
  std::vector<SyrkArgs> order;
  for (const Item& it : items) order.push_back(it.a);
  std::stable_sort(order.begin(), order.end(), [](const SyrkArgs& x, const SyrkArgs& y) {
    return x.rows_per_split > y.rows_per_split;
  });
  std::vector<int64_t> off(1, 0);
  double flops = 0, bytes = 0;
  const double esz = prec == GW_FP64 ? 8.0 : 4.0;
  for (const SyrkArgs& a : order) {
    off.push_back(off.back() + (int64_t)a.splits * a.L * a.n_tiles);
    flops += (double)a.L * a.N * (a.N + 1.0) * (double)a.k_rows;
    bytes += (double)a.k_rows * a.N * esz + (double)a.L * a.N * (a.N + 1.0) / 2.0 * 8.0;
  }
  constexpr int CHUNK = 8;
  Batch bt;
  GW_TRY(stage_batch(ctx, order, off, CHUNK, bt));
  const int64_t grid = (off.back() + 8 * CHUNK - 1) / (8 * CHUNK) * (8 * CHUNK);
  const int pi = prof_begin(ctx);
  launch_syrk_kernel(ctx, prec, fast, scaled, SyrkArgs{}, bt, grid);
  prof_end(ctx, pi, prof_name, flops, bytes);
  GW_TRY(launch_check(ctx, "batched syrk kernel"));
  std::vector<RedArgs> red;
  std::vector<int64_t> n;
  for (const Item& it : items) {
    red.push_back(it.r);
    n.push_back((int64_t)it.r.L * it.r.n_tiles * BM * BM);
  }
  return elementwise_batched(ctx, red, n, syrk_reduce_batched_kernel, "syrk_reduce_batched");
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
    GW_TRY(gw::lt_scale_launch(ctx, prec, n_lt, dx, dw, n_i, n_virt, dei, dea, scale, 0));
  }
  GW_TRY(gw::syrk_launch(ctx, prec, R_chunk, k, n_naf, ld_R, n_lt, scale, 1.0, M, accumulate,
                         prec == GW_FP64 ? "chi_syrk_f64"
                                         : (prec == GW_BF16X3 ? "chi_syrk_bf16x3" : "chi_syrk_f32")));
  if (finalize) GW_TRY(gw::mirror_lower(ctx, M, n_lt, n_naf));
  return GW_OK;
}

extern "C" gw_status gw_polarizability_sos(gw_ctx ctx, gw_precision prec, int n_naf, int n_w,
                                           const double* omega, int n_i, int n_virt,
                                           const double* eps_i, const double* eps_a,
                                           const void* R_chunk, int64_t ld_R, int accumulate,
                                           int finalize, double* P) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_polarizability_sos: ctx is NULL");
  gw::clear_error(ctx);
  GW_REQUIRE(ctx, prec == GW_FP64 || prec == GW_FP32 || prec == GW_BF16X3,
             "gw_polarizability_sos: unknown precision %d", (int)prec);
  GW_REQUIRE(ctx, n_naf >= 1 && n_w >= 1 && n_i >= 0 && n_virt >= 1,
             "gw_polarizability_sos: bad sizes (n_naf=%d n_w=%d n_i=%d n_virt=%d)", n_naf, n_w,
             n_i, n_virt);
  GW_REQUIRE(ctx, omega && P && eps_a && (n_i == 0 || (eps_i && R_chunk)),
             "gw_polarizability_sos: NULL argument");
  if (ld_R == 0) ld_R = n_naf;
  GW_REQUIRE(ctx, ld_R >= n_naf, "gw_polarizability_sos: ld_R < n_naf");
  GW_HIP(ctx, hipSetDevice(ctx->device));
  const int64_t k = (int64_t)n_i * n_virt;
  const double* dom = gw::stage_t(ctx, omega, n_w);
  const double* dei = n_i ? gw::stage_t(ctx, eps_i, n_i) : nullptr;
  const double* dea = gw::stage_t(ctx, eps_a, n_virt);
  if (!dom || !dea || (n_i && !dei)) return GW_EINVAL;
  void* scale = nullptr;
  if (k > 0) {
    const size_t esz = prec == GW_FP64 ? 8 : 4;
    scale = gw::ws_get(ctx, WS_SYRK_SCALE, (size_t)n_w * k * esz);
    if (!scale) return GW_ENOMEM;
    GW_TRY(gw::lt_scale_launch(ctx, prec, n_w, dom, dom, n_i, n_virt, dei, dea, scale, 1));
  }
  GW_TRY(gw::syrk_launch(ctx, prec, R_chunk, k, n_naf, ld_R, n_w, scale, 1.0, P, accumulate,
                         prec == GW_FP64 ? "chi_sos_f64"
                                         : (prec == GW_BF16X3 ? "chi_sos_bf16x3" : "chi_sos_f32")));
  if (finalize) GW_TRY(gw::mirror_lower(ctx, P, n_w, n_naf));
  return GW_OK;
}

namespace {

__global__ void fill_zero_kernel(double* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

}  // namespace

namespace gw {

gw_status fill_zero(gw_ctx ctx, double* p, int64_t n) {
  if (n <= 0) return GW_OK;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(n, 256)), dim3(256), 0, ctx->stream, p, n);
  return launch_check(ctx, "fill_zero_kernel");
}

}  // namespace gw

extern "C" gw_status gw_polarizability_lt_batched(gw_ctx ctx, gw_precision prec, int n_lt,
                                                  int n_jobs, const gw_chi_job* jobs,
                                                  int accumulate, int finalize) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_polarizability_lt_batched: ctx is NULL");
  gw::clear_error(ctx);
  GW_REQUIRE(ctx, prec == GW_FP64 || prec == GW_FP32 || prec == GW_BF16X3,
             "gw_polarizability_lt_batched: unknown precision %d", (int)prec);
  GW_REQUIRE(ctx, n_lt >= 1 && n_lt <= 32 && n_jobs >= 0 && (n_jobs == 0 || jobs),
             "gw_polarizability_lt_batched: bad sizes (n_lt=%d n_jobs=%d)", n_lt, n_jobs);
  for (int d = 0; d < n_jobs; ++d) {
    const gw_chi_job& j = jobs[d];
    GW_REQUIRE(ctx, j.n_naf >= 1 && j.n_i >= 0 && j.n_virt >= 1,
               "gw_polarizability_lt_batched: job %d: bad sizes", d);
    GW_REQUIRE(ctx, j.x_lt && j.w_lt && j.M && j.eps_a && (j.n_i == 0 || (j.eps_i && j.R_chunk)),
               "gw_polarizability_lt_batched: job %d: NULL argument", d);
    GW_REQUIRE(ctx, j.ld_R == 0 || j.ld_R >= j.n_naf,
               "gw_polarizability_lt_batched: job %d: ld_R < n_naf", d);
  }
  if (n_jobs == 0) return GW_OK;
  GW_HIP(ctx, hipSetDevice(ctx->device));
  const size_t esz = prec == GW_FP64 ? 8 : 4;
  size_t scale_total = 0;
  for (int d = 0; d < n_jobs; ++d)
    scale_total += (size_t)n_lt * jobs[d].n_i * jobs[d].n_virt;
  unsigned char* scale = static_cast<unsigned char*>(
      gw::ws_get(ctx, WS_SYRK_SCALE, std::max<size_t>(scale_total, 1) * esz));
  if (!scale) return GW_ENOMEM;
  std::vector<gw::ScaleJob> sj;
  std::vector<gw::SyrkJob> kj;
  std::vector<gw::MirrorJob> mj;
  size_t so = 0;
  for (int d = 0; d < n_jobs; ++d) {
    const gw_chi_job& j = jobs[d];
    const int64_t k = (int64_t)j.n_i * j.n_virt;
    void* sc = scale + so * esz;
    if (k > 0) {
      const double* dx = gw::stage_t(ctx, j.x_lt, n_lt);
      const double* dw = gw::stage_t(ctx, j.w_lt, n_lt);
      const double* dei = gw::stage_t(ctx, j.eps_i, j.n_i);
      const double* dea = gw::stage_t(ctx, j.eps_a, j.n_virt);
      if (!dx || !dw || !dei || !dea) return GW_EINVAL;
      sj.push_back(gw::ScaleJob{n_lt, dx, dw, j.n_i, j.n_virt, dei, dea, sc});
    }
    // jobs without rows still zero (or keep) their output; their scale
    // pointer is never read
    kj.push_back(gw::SyrkJob{j.R_chunk, k, j.n_naf, j.ld_R ? j.ld_R : j.n_naf, n_lt, sc, 1.0,
                             j.M, accumulate});
    mj.push_back(gw::MirrorJob{j.M, n_lt, j.n_naf});
    so += (size_t)n_lt * k;
  }
  GW_TRY(gw::lt_scale_batched(ctx, prec, sj));
  GW_TRY(gw::syrk_batched_launch(ctx, prec, kj,
                                 prec == GW_FP64 ? "chi_syrk_f64"
                                 : (prec == GW_BF16X3 ? "chi_syrk_bf16x3" : "chi_syrk_f32")));
  if (finalize) GW_TRY(gw::mirror_lower_batched(ctx, mj));
  return GW_OK;
}

namespace gw {

size_t syrk_part_bytes(gw_precision prec, int64_t k_rows, int N, int L) {
  (void)prec;
  const int T = (N + BM - 1) / BM;
  const int n_tiles = T * (T + 1) / 2;
  int S = k_rows > 0 ? choose_splits(k_rows, (int64_t)n_tiles * L) : 1;
  if (2 * S <= 16 && k_rows / (2 * S) >= 1024) S *= 2;   // largest autotuning candidate
  return (size_t)S * L * n_tiles * BM * BM * sizeof(double);
}

}  // namespace gw
