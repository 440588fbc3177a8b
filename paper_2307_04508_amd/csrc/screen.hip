// Screening: Pi_j = -2 s sum_m exp(-w_j^2 x_m) M^m (Eq. 10), A_j = 1 - Pi_j,
// W^_j = A_j^-1 - 1 (Eq. 2), in FP64, batched over frequencies.
//
// The inverse uses the symmetric sweep (block Gauss-Jordan) form: for each
// pivot block K, with D = A_KK and the rest R,
//     A_RR <- A_RR - A_RK D^-1 A_KR,   A_RK <- A_RK D^-1,   A_KK <- -D^-1,
// which keeps every intermediate symmetric, so only the lower triangle is
// stored and updated; after the last block A holds -A^-1.  Sweeping a block
// equals sweeping its columns in turn, so each 256 x 256 pivot block D is
// inverted by a column-by-column sweep held in the registers of one
// workgroup per matrix.  The pivots are Schur complements of the symmetric positive
// definite 1 - Pi, so no pivoting is needed; a non-positive pivot raises the
// deferred GW_ENOTSPD flag.  The rank-256 trailing update (the whole O(N^3)
// cost, N^3 flops per matrix on the triangle) and the panel product run on
// v_mfma_f64_16x16x4f64; the matrices are streamed once per 256 columns.
#include <algorithm>
#include <cstring>
#include <cmath>
#include <string>

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
  const double* M;      // [L][N][N]; sum-over-states: [F][N][N] sums P_j
  int L, N;
  const double* x;      // [L]
  const double* omega;  // [F]
  int F;
  double* A;            // [F][N][N]
  int sos;              // 1: A_j = 1 + 2 s P_j (Eq. 3 without the Laplace transform)
};

__device__ __forceinline__ void load_coef(const AsmArgs& a, double* coef) {
  if (a.sos) return;
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
  const double d = (p == q) ? 1.0 : 0.0;
  if (a.sos) {
    for (int j = 0; j < a.F; ++j) a.A[j * NN + idx] = d + 4.0 * a.M[j * NN + idx];   // 2 s, s = 2
    return;
  }
  // fully unrolled over the at most 32 Laplace points, so mv stays in
  // registers (a loop bounded by L alone indexes it dynamically: scratch)
  double mv[32];
#pragma unroll
  for (int m = 0; m < 32; ++m) mv[m] = m < a.L ? a.M[m * NN + idx] : 0.0;
  for (int j = 0; j < a.F; ++j) {
    double v = d;
#pragma unroll
    for (int m = 0; m < 32; ++m)
      if (m < a.L) v += coef[j * a.L + m] * mv[m];
    a.A[j * NN + idx] = v;
  }
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
// for one set of F matrices.  Width pw = 64 inverts each 64 x 64 pivot in
// registers (Dinv) and updates 64-tiles; pw = 128 or 256 sweeps each pivot
// block whole in one workgroup (-D^-1 into Dw), so the O(N^3) trailing
// update is a rank-pw MFMA product and the matrices are streamed through
// HBM once per pw columns.
struct SwArgs {
  double* A;            // [F][N][N] lower triangle
  double* C;            // [F][N][pw] pivot column panel
  double* P;            // [F][N][pw] scaled panel
  double* Dinv;         // pw = B: [F][B][B] D^-1
  double* Dw;           // pw > B: [F][bw][bw], -D^-1 (lower triangle)
  int N, F, kb, bw, T, kt;
  int pw;               // panel width (B, BI or BO)
  int flag_base;        // flag value offset of this set's first matrix
  int panel_blocks;     // inner panel kernel: workgroups per matrix
  double* Cn;           // fused update (pw = 128): the next step's panel, [F][N][pw]
  int kbn, bwn;         //   its first column and width (bwn = 0: no next step)
  int mode;             // fused update: 0 every lower tile; 1 the tiles of row and
                        // column kbn / 128 (the next panel); 2 the others
};

// C[j][r][c] = A_j(r, kb + c) read from the lower triangle; zero for c >= bw.
__device__ __forceinline__ void gather_elem(const SwArgs& a, int64_t idx) {
  const int64_t NN = (int64_t)a.N * a.N;
  if (idx >= (int64_t)a.F * a.N * a.pw) return;
  const int c = (int)(idx % a.pw);
  const int r = (int)((idx / a.pw) % a.N);
  const int j = (int)(idx / ((int64_t)a.pw * a.N));
  double v = 0.0;
  if (c < a.bw) {
    const int col = a.kb + c;
    v = (r >= col) ? a.A[j * NN + (int64_t)r * a.N + col] : a.A[j * NN + (int64_t)col * a.N + r];
  }
  a.C[idx] = v;
}

__global__ void gather_panel_batched_kernel(Batch bt) {
  SwArgs a;
  int64_t first;
  if (!block_of(bt, a, first)) return;
  for (int e = 0; e < kBatchElems; e += 256) gather_elem(a, first + e + threadIdx.x);
}

// Dw[j][p][q] = D[p][q] (the pivot block, from the panel rows).
__device__ __forceinline__ void extract_elem(const SwArgs& a, int64_t idx) {
  const int64_t bb = (int64_t)a.bw * a.bw;
  if (idx >= (int64_t)a.F * bb) return;
  const int j = (int)(idx / bb);
  const int p = (int)((idx % bb) / a.bw), q = (int)(idx % a.bw);
  a.Dw[idx] = a.C[((int64_t)j * a.N + a.kb + p) * a.pw + q];
}

__global__ void extract_pivot_batched_kernel(Batch bt) {
  SwArgs a;
  int64_t first;
  if (!block_of(bt, a, first)) return;
  for (int e = 0; e < kBatchElems; e += 256) extract_elem(a, first + e + threadIdx.x);
}

// Inner level: one workgroup per matrix sweeps the 64 x 64 pivot block,
// stored in registers: thread (tr, tc) owns rows 4 tr .. 4 tr + 3 and
// columns 4 tc .. 4 tc + 3.  Each step the owners of pivot column k and row
// k publish them through double-buffered LDS (one barrier per step).  A
// partial block (bw < 64) is padded with the identity, which the sweep
// leaves as -1 and does not couple to the valid part.  Stores D^-1
// (zero-padded).
constexpr int PIV_THREADS = 256;
__device__ __forceinline__ void pivot_unit(const SwArgs& a, int j, int* __restrict__ flags) {
  __shared__ double colb[2][B], rowb[2][B];
  const int N = a.N, kb = a.kb, bw = a.bw;
  const double* Cj = a.C + (int64_t)j * N * a.pw;
  const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
  double d[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int gr = 4 * tr + r, gc = 4 * tc + c;
      d[r][c] = (gr < bw && gc < bw) ? Cj[(int64_t)(kb + gr) * a.pw + gc] : (gr == gc ? 1.0 : 0.0);
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

__global__ __launch_bounds__(PIV_THREADS) void pivot_batched_kernel(Batch bt,
                                                                    int* __restrict__ flags) {
  const int d = find_problem(bt.off, bt.n, blockIdx.x);
  const SwArgs a = static_cast<const SwArgs*>(bt.descs)[d];
  pivot_unit(a, (int)(blockIdx.x - bt.off[d]), flags);
}

// One workgroup per matrix sweeps its bw x bw pivot block D (PB >= bw;
// padded with the identity), read from the panel rows kb .. of C.  The
// lower triangle is held in registers as E x E blocks, thread u owning
// lower block (tr, tc), tr >= tc (the diagonal blocks whole).  Each step
// the owners of row k and of column k publish column k of the symmetric
// block through double-buffered LDS (one barrier per step), then every block
// takes the update a_ij -= a_ik a_kj / p and the owners rescale row and
// column k.  Leaves -D^-1 (lower triangle) in Dw; a non-positive or
// non-finite pivot raises the deferred flag and leaves zeros.
template <int PB, int E>
struct PivDense {
  static constexpr int NB = PB / E;                       // blocks per side
  static constexpr int BLOCKS = NB * (NB + 1) / 2;        // lower blocks
  static constexpr int THREADS = (BLOCKS + 63) / 64 * 64;
};

template <int PB, int E>
__global__ __launch_bounds__((PivDense<PB, E>::THREADS), 1) void pivot_dense_kernel(
    Batch bt, int* __restrict__ flags) {
  constexpr int NB = PivDense<PB, E>::NB;
  __shared__ double v[2][PB];
  const int dd = find_problem(bt.off, bt.n, blockIdx.x);
  const SwArgs a = static_cast<const SwArgs*>(bt.descs)[dd];
  const int j = (int)(blockIdx.x - bt.off[dd]);
  const int u = threadIdx.x;
  const bool own = u < PivDense<PB, E>::BLOCKS;
  int tr = 0, tc = 0;
  if (own) {
    tr = (int)((sqrtf(8.0f * u + 1.0f) - 1.0f) * 0.5f);
    while ((tr + 1) * (tr + 2) / 2 <= u) ++tr;
    while (tr * (tr + 1) / 2 > u) --tr;
    tc = u - tr * (tr + 1) / 2;
  }
  const int bw = a.bw, pw = a.pw;
  const double* Cj = a.C + (int64_t)j * a.N * pw + (int64_t)a.kb * pw;   // D[p][q] = Cj[p pw + q]
  double d[E][E];
#pragma unroll
  for (int r = 0; r < E; ++r)
#pragma unroll
    for (int c = 0; c < E; ++c) {
      const int gr = E * tr + r, gc = E * tc + c;
      d[r][c] = (own && gr < bw && gc < bw) ? Cj[(int64_t)gr * pw + gc] : (gr == gc ? 1.0 : 0.0);
    }
  bool bad = false;
  for (int kq = 0; kq < NB; ++kq) {
#pragma unroll
    for (int kk = 0; kk < E; ++kk) {
      const int k = E * kq + kk, buf = k & 1;
      if (own && tc == kq) {
#pragma unroll
        for (int r = 0; r < E; ++r) v[buf][E * tr + r] = d[r][kk];
      }
      if (own && tr == kq) {
#pragma unroll
        for (int c = 0; c < E; ++c) v[buf][E * tc + c] = d[kk][c];
      }
      __syncthreads();
      const double piv = v[buf][k];
      bad = bad || !(piv > 0.0) || !isfinite(piv);
      // 1 / piv from the hardware estimate r and its correction
      // r (1 + e + e^2), e = 1 - piv r (rounding-level; shorter than a division)
      const double r0 = __builtin_amdgcn_rcp(piv), e0 = fma(-piv, r0, 1.0);
      const double inv = fma(r0, fma(e0, e0, e0), r0);
      if (own) {
        double vc[E];
#pragma unroll
        for (int c = 0; c < E; ++c) vc[c] = v[buf][E * tc + c];
#pragma unroll
        for (int r = 0; r < E; ++r) {
          const double vr = v[buf][E * tr + r] * inv;
#pragma unroll
          for (int c = 0; c < E; ++c) d[r][c] = fma(-vr, vc[c], d[r][c]);
          if (tc == kq) d[r][kk] = vr;                  // a_ik / p
        }
        if (tr == kq) {
#pragma unroll
          for (int c = 0; c < E; ++c) d[kk][c] = vc[c] * inv;   // a_kj / p
          if (tc == kq) d[kk][kk] = -inv;
        }
      }
    }
  }
  // every thread sees the same pivots, so `bad` is uniform
  if (bad && u == 0) atomicCAS(flags, 0, a.flag_base + j + 1);
  if (own) {
    double* out = a.Dw + (int64_t)j * bw * bw;
#pragma unroll
    for (int r = 0; r < E; ++r)
#pragma unroll
      for (int c = 0; c < E; ++c) {
        const int gr = E * tr + r, gc = E * tc + c;
        if (gr < bw && gc < bw && gr >= gc) {
          const double w = bad ? 0.0 : d[r][c];
          out[(int64_t)gr * bw + gc] = w;
          out[(int64_t)gc * bw + gr] = w;
        }
      }
  }
}

// Inner level: P[j][r][c] = sum_c' C[j][r][c'] Dinv[j][c'][c] for every row r; this
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

__global__ __launch_bounds__(256) void panel_batched_kernel(Batch bt) {
  const int d = find_problem(bt.off, bt.n, blockIdx.x);
  const SwArgs a = static_cast<const SwArgs*>(bt.descs)[d];
  const int u = (int)(blockIdx.x - bt.off[d]);
  panel_unit(a, u / a.panel_blocks, u % a.panel_blocks, a.panel_blocks);
}


// One 64-wide k chunk of a 64 x 64 tile product on FP64 MFMA (16x16x4):
// acc[a][b] += Xs[rows of wave][k] Ys[cols of wave][k].  4 waves of 32 x 32.
__device__ __forceinline__ void mfma_chunk(const double (*Xs)[LDP], const double (*Ys)[LDP],
                                           f64x4 (&acc)[2][2], int wy, int wx, int lane) {
#pragma unroll 4
  for (int k = 0; k < B; k += 4) {
    const int kr = k + (lane >> 4);
    double af[2], bf[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      af[a] = Xs[wy * 32 + a * 16 + (lane & 15)][kr];
      bf[a] = Ys[wx * 32 + a * 16 + (lane & 15)][kr];
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
  }
}

// Tile coordinates (I >= J) of lower tile t.
__device__ __forceinline__ void lower_tile(int t, int& I, int& J) {
  I = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  J = t - I * (I + 1) / 2;
}

// Outer level: P[j][r][c] = -sum_k C[j][r][k] Dsym[j][k][c] (Dw holds -D^-1
// in its lower triangle, so P = C D^-1), 64 x 64 output tiles, k in chunks
// of 64 over the bw pivot columns; columns c >= bw are zero.
__global__ __launch_bounds__(256) void panel_gemm_batched_kernel(Batch bt) {
  __shared__ __attribute__((aligned(16))) double Xs[B][LDP];
  __shared__ double Ys[B][LDP];
  SwArgs sa;
  int64_t lid;
  if (!unit_of(SwArgs{}, bt, sa, lid)) return;
  const int N = sa.N, bw = sa.bw, pw = sa.pw;
  const int ct = pw / B, rt = (N + B - 1) / B;
  const int j = (int)(lid / ((int64_t)rt * ct));
  const int rem = (int)(lid % ((int64_t)rt * ct));
  const int I = rem / ct, J = rem % ct;
  const double* Cj = sa.C + (int64_t)j * N * pw;
  const double* Dj = sa.Dw + (int64_t)j * bw * bw;
  double* Pj = sa.P + (int64_t)j * N * pw;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wy = wave >> 1, wx = wave & 1;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  // loads: thread t covers row (or column) t >> 2, 16 consecutive entries
  // from 16 (t & 3), all issued before the first LDS store
  const int lr = tid >> 2, lc = (tid & 3) * 16;
  for (int k0 = 0; k0 < bw; k0 += B) {
    // C rows I B + lr, columns k0 + lc ...: pairs (pw and k0 + lc even, so
    // 16-byte aligned; the pair's second column is < pw), zero past bw
    const int gr = I * B + lr;
    double2 xv[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int gk = k0 + lc + 2 * e;
      xv[e] = make_double2(0.0, 0.0);
      if (gr < N && gk < bw) {
        xv[e] = *reinterpret_cast<const double2*>(Cj + (int64_t)gr * pw + gk);
        if (gk + 1 >= bw) xv[e].y = 0.0;
      }
    }
    // symmetric D (lower triangle stored): entries with column <= row are
    // read along rows of D, the others along columns, so both are
    // contiguous per thread; every entry is written once, zero past bw
    double yl[16], yu[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int gc = J * B + lr, gk = k0 + lc + e;              // Ys[lr][lc + e]
      yl[e] = (gc < bw && gk < bw && gc >= gk) ? Dj[(int64_t)gc * bw + gk] : 0.0;
      const int hc = J * B + lc + e, hk = k0 + lr;              // Ys[lc + e][lr]
      yu[e] = (hc < bw && hk < bw && hc < hk) ? Dj[(int64_t)hk * bw + hc] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e)
      *reinterpret_cast<double2*>(&Xs[lr][lc + 2 * e]) = xv[e];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int gc = J * B + lr, gk = k0 + lc + e;
      if (!(gc < bw && gk < bw && gc < gk)) Ys[lr][lc + e] = yl[e];
      const int hc = J * B + lc + e, hk = k0 + lr;
      if (hc < bw && hk < bw && hc < hk) Ys[lc + e][lr] = yu[e];
    }
    __syncthreads();
    mfma_chunk(Xs, Ys, acc, wy, wx, lane);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = I * B + wy * 32 + a * 16 + (lane >> 4) + 4 * r;
        const int col = J * B + wx * 32 + b * 16 + (lane & 15);
        if (row < N) Pj[(int64_t)row * pw + col] = col < bw ? -acc[a][b][r] : 0.0;
      }
}

// A[I][J] -= sum_k P[I rows][k] C[J rows][k] (k < bw) for lower 64-tiles
// I >= J outside the pivot block's rows and columns.
__global__ __launch_bounds__(256) void update_batched_kernel(Batch bt) {
  __shared__ double Ps[B][LDP];
  __shared__ double Cs[B][LDP];
  SwArgs sa;
  int64_t lid;
  if (!unit_of(SwArgs{}, bt, sa, lid)) return;
  const int N = sa.N, pw = sa.pw, bw = sa.bw;
  const int T = (N + B - 1) / B;
  const int n_tiles = T * (T + 1) / 2;
  const int j = (int)(lid / n_tiles);
  int I, J;
  lower_tile((int)(lid % n_tiles), I, J);
  const int k_lo = sa.kb / B, k_hi = (sa.kb + bw - 1) / B;   // pivot block, in tiles
  if ((I >= k_lo && I <= k_hi) || (J >= k_lo && J <= k_hi)) return;
  const double* Pj = sa.P + (int64_t)j * N * pw;
  const double* Cj = sa.C + (int64_t)j * N * pw;
  double* Aj = sa.A + (int64_t)j * N * N;
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
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < bw; k0 += B) {
    for (int i = tid; i < B * B / 2; i += 256) {
      const int r = i / (B / 2), c2 = (i % (B / 2)) * 2;
      const int gr = I * B + r, gc = J * B + r;
      double2 pv = make_double2(0.0, 0.0), cv = pv;
      // panel columns bw .. pw-1 hold zeros, so whole 64-chunks load as pairs
      if (gr < N) pv = *reinterpret_cast<const double2*>(Pj + (int64_t)gr * pw + k0 + c2);
      if (gc < N) cv = *reinterpret_cast<const double2*>(Cj + (int64_t)gc * pw + k0 + c2);
      *reinterpret_cast<double2*>(&Ps[r][c2]) = pv;
      *reinterpret_cast<double2*>(&Cs[r][c2]) = cv;
    }
    __syncthreads();
    mfma_chunk(Ps, Cs, acc, wy, wx, lane);
    __syncthreads();
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

// Outer level (pivot width 128 or 256, so pivot blocks are unions of whole
// 128-tiles): A[I][J] -= sum_k P[I rows][k] C[J rows][k] for lower 128 x 128
// tiles outside the pivot block's rows and columns.  8 waves of 32 x 64 on
// v_mfma_f64_16x16x4f64; k in double-buffered chunks of 16, stored k-major
// in LDS ([k][row], padded) so that the 16 rows an MFMA operand takes are
// consecutive doubles.  Panel columns bw .. pw-1 hold zeros, so k runs over
// whole chunks.
constexpr int BU = 128;
constexpr int BKU = 16;
constexpr int LDU = BU + 8;

__global__ __launch_bounds__(512, 2) void update128_batched_kernel(Batch bt) {
  __shared__ double Ps[2][BKU][LDU];
  __shared__ double Cs[2][BKU][LDU];
  SwArgs sa;
  int64_t lid;
  if (!unit_of(SwArgs{}, bt, sa, lid)) return;
  const int N = sa.N, pw = sa.pw, bw = sa.bw;
  const int T = (N + BU - 1) / BU;
  const int n_tiles = T * (T + 1) / 2;
  const int j = (int)(lid / n_tiles);
  int I, J;
  lower_tile((int)(lid % n_tiles), I, J);
  const int k_lo = sa.kb / BU, k_hi = (sa.kb + bw - 1) / BU;   // pivot block, in tiles
  if ((I >= k_lo && I <= k_hi) || (J >= k_lo && J <= k_hi)) return;
  const double* Pj = sa.P + (int64_t)j * N * pw;
  const double* Cj = sa.C + (int64_t)j * N * pw;
  double* Aj = sa.A + (int64_t)j * N * N;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wy = wave >> 1, wx = wave & 1;            // rows wy*32, cols wx*64
  // The accumulators start from the tile of A and P enters LDS negated, so
  // the MFMAs leave A - P C^T in them: the tile is read at the start, where
  // its latency overlaps that of the first panel loads, and only stored at
  // the end.
  f64x4 acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = I * BU + wy * 32 + a * 16 + (lane >> 4) + 4 * r;
        const int col = J * BU + wx * 64 + b * 16 + (lane & 15);
        acc[a][b][r] = (row < N && col < N) ? Aj[(int64_t)row * N + col] : 0.0;
      }
  // loader: rows (tid >> 3) + 64 h, k pair (tid & 7) * 2
  const int lr = tid >> 3, lk = (tid & 7) * 2;
  double2 rp[2], rc[2];
  auto gload = [&](int k0) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int pr = I * BU + lr + 64 * h, cr = J * BU + lr + 64 * h;
      rp[h] = pr < N ? *reinterpret_cast<const double2*>(Pj + (int64_t)pr * pw + k0 + lk)
                     : make_double2(0.0, 0.0);
      rc[h] = cr < N ? *reinterpret_cast<const double2*>(Cj + (int64_t)cr * pw + k0 + lk)
                     : make_double2(0.0, 0.0);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      Ps[buf][lk][lr + 64 * h] = -rp[h].x;
      Ps[buf][lk + 1][lr + 64 * h] = -rp[h].y;
      Cs[buf][lk][lr + 64 * h] = rc[h].x;
      Cs[buf][lk + 1][lr + 64 * h] = rc[h].y;
    }
  };
  const int nk = (bw + BKU - 1) / BKU;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int it = 0; it < nk; ++it) {
    const int cur = it & 1;
    if (it + 1 < nk) gload((it + 1) * BKU);
#pragma unroll
    for (int kk = 0; kk < BKU / 4; ++kk) {
      const int kr = 4 * kk + (lane >> 4);
      double af[2], bf[4];
#pragma unroll
      for (int a = 0; a < 2; ++a) af[a] = Ps[cur][kr][wy * 32 + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < 4; ++b) bf[b] = Cs[cur][kr][wx * 64 + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
    if (it + 1 < nk) sstore(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = I * BU + wy * 32 + a * 16 + (lane >> 4) + 4 * r;
        const int col = J * BU + wx * 64 + b * 16 + (lane & 15);
        if (row < N && col < N) Aj[(int64_t)row * N + col] = acc[a][b][r];
      }
}

// Width 128: P = C D^-1 = -C Dw for every 128-row tile of the panel (Dw
// holds -D^-1 in both triangles, so its rows serve as the k-contiguous
// second operand), with the update kernel's tile pipeline: 8 waves of
// 32 x 64, k in double-buffered chunks of 16 stored k-major in LDS.
// Columns c >= bw of P are zero.
__global__ __launch_bounds__(512, 2) void panel128_kernel(Batch bt) {
  __shared__ double Xs[2][BKU][LDU];
  __shared__ double Ds[2][BKU][LDU];
  SwArgs sa;
  int64_t lid;
  if (!unit_of(SwArgs{}, bt, sa, lid)) return;
  const int N = sa.N, pw = sa.pw, bw = sa.bw;
  const int T = (N + BU - 1) / BU;
  const int j = (int)(lid / T), I = (int)(lid % T);
  const double* Cj = sa.C + (int64_t)j * N * pw;
  const double* Dj = sa.Dw + (int64_t)j * bw * bw;
  double* Pj = sa.P + (int64_t)j * N * pw;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wy = wave >> 1, wx = wave & 1;
  f64x4 acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int lr = tid >> 3, lk = (tid & 7) * 2;
  double rx[2][2], rd[2][2];
  auto gload = [&](int k0) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int xr = I * BU + lr + 64 * h, dr = lr + 64 * h;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int k = k0 + lk + e;
        rx[h][e] = (xr < N && k < bw) ? Cj[(int64_t)xr * pw + k] : 0.0;
        rd[h][e] = (dr < bw && k < bw) ? Dj[(int64_t)dr * bw + k] : 0.0;
      }
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        Xs[buf][lk + e][lr + 64 * h] = rx[h][e];
        Ds[buf][lk + e][lr + 64 * h] = rd[h][e];
      }
  };
  const int nk = (bw + BKU - 1) / BKU;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int it = 0; it < nk; ++it) {
    const int cur = it & 1;
    if (it + 1 < nk) gload((it + 1) * BKU);
#pragma unroll
    for (int kk = 0; kk < BKU / 4; ++kk) {
      const int kr = 4 * kk + (lane >> 4);
      double af[2], bf[4];
#pragma unroll
      for (int a = 0; a < 2; ++a) af[a] = Xs[cur][kr][wy * 32 + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < 4; ++b) bf[b] = Ds[cur][kr][wx * 64 + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
    if (it + 1 < nk) sstore(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = I * BU + wy * 32 + a * 16 + (lane >> 4) + 4 * r;
        const int col = wx * 64 + b * 16 + (lane & 15);
        if (row < N) Pj[(int64_t)row * pw + col] = col < bw ? -acc[a][b][r] : 0.0;
      }
}

// Width 128 (one 128-tile per pivot block K), the whole step after the
// panel product in one pass over the lower 128-tiles of A:
//   tiles off row and column K:  A[I][J] -= P[I rows] C[J rows]^T (as above);
//   tiles in column K:           A(r, K) <- P[r]        (the swept column);
//   tiles in row K:              A(K, c) <- P[c]^T      (its mirror in the lower triangle);
//   the pivot tile:              A(K, K) <- -D^-1       (lower triangle, from Dw);
// and every tile in row or column K + 1 also writes its new values into the
// next step's panel Cn (transposed for row K + 1; the diagonal tile fills
// both triangles; zeros past N), which replaces that step's gather.
__global__ __launch_bounds__(512, 2) void update_fused_kernel(Batch bt) {
  __shared__ double Ps[2][BKU][LDU];
  __shared__ double Cs[2][BKU][LDU];
  SwArgs sa;
  int64_t lid;
  if (!unit_of(SwArgs{}, bt, sa, lid)) return;
  const int N = sa.N, pw = sa.pw, bw = sa.bw, kb = sa.kb;
  const int T = (N + BU - 1) / BU;
  const int K = kb / BU, Kn = sa.bwn > 0 ? sa.kbn / BU : -1;
  int I, J, j;
  if (sa.mode == 1) {                 // row Kn (J <= Kn), then column Kn (I > Kn)
    j = (int)(lid / T);
    const int u = (int)(lid % T);
    I = u <= Kn ? Kn : u;
    J = u <= Kn ? u : Kn;
  } else if (sa.mode == 2 && Kn >= 0) {
    // the lower tiles of order T - 1, indices at or past Kn shifted by one
    const int n2 = (T - 1) * T / 2;
    j = (int)(lid / n2);
    lower_tile((int)(lid % n2), I, J);
    I += I >= Kn;
    J += J >= Kn;
  } else {
    const int n_tiles = T * (T + 1) / 2;
    j = (int)(lid / n_tiles);
    lower_tile((int)(lid % n_tiles), I, J);
  }
  const bool in_row = I == K, in_col = J == K;
  const double* Pj = sa.P + (int64_t)j * N * pw;
  const double* Cj = sa.C + (int64_t)j * N * pw;
  double* Aj = sa.A + (int64_t)j * N * N;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wy = wave >> 1, wx = wave & 1;            // rows wy*32, cols wx*64
  f64x4 acc[2][4];
  if (!in_row && !in_col) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = I * BU + wy * 32 + a * 16 + (lane >> 4) + 4 * r;
          const int col = J * BU + wx * 64 + b * 16 + (lane & 15);
          acc[a][b][r] = (row < N && col < N) ? Aj[(int64_t)row * N + col] : 0.0;
        }
    const int lr = tid >> 3, lk = (tid & 7) * 2;
    double2 rp[2], rc[2];
    auto gload = [&](int k0) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int pr = I * BU + lr + 64 * h, cr = J * BU + lr + 64 * h;
        rp[h] = pr < N ? *reinterpret_cast<const double2*>(Pj + (int64_t)pr * pw + k0 + lk)
                       : make_double2(0.0, 0.0);
        rc[h] = cr < N ? *reinterpret_cast<const double2*>(Cj + (int64_t)cr * pw + k0 + lk)
                       : make_double2(0.0, 0.0);
      }
    };
    auto sstore = [&](int buf) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        Ps[buf][lk][lr + 64 * h] = -rp[h].x;
        Ps[buf][lk + 1][lr + 64 * h] = -rp[h].y;
        Cs[buf][lk][lr + 64 * h] = rc[h].x;
        Cs[buf][lk + 1][lr + 64 * h] = rc[h].y;
      }
    };
    const int nk = (bw + BKU - 1) / BKU;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int it = 0; it < nk; ++it) {
      const int cur = it & 1;
      if (it + 1 < nk) gload((it + 1) * BKU);
#pragma unroll
      for (int kk = 0; kk < BKU / 4; ++kk) {
        const int kr = 4 * kk + (lane >> 4);
        double af[2], bf[4];
#pragma unroll
        for (int a = 0; a < 2; ++a) af[a] = Ps[cur][kr][wy * 32 + a * 16 + (lane & 15)];
#pragma unroll
        for (int b = 0; b < 4; ++b) bf[b] = Cs[cur][kr][wx * 64 + b * 16 + (lane & 15)];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
      }
      if (it + 1 < nk) sstore(cur ^ 1);
      __syncthreads();
    }
  } else {
    const double* Dj = sa.Dw + (int64_t)j * bw * bw;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = I * BU + wy * 32 + a * 16 + (lane >> 4) + 4 * r;
          const int col = J * BU + wx * 64 + b * 16 + (lane & 15);
          double v = 0.0;
          if (row < N && col < N) {
            if (in_row && in_col)
              v = row >= col ? Dj[(int64_t)(row - kb) * bw + (col - kb)] : 0.0;
            else if (in_col)
              v = Pj[(int64_t)row * pw + (col - kb)];
            else
              v = Pj[(int64_t)col * pw + (row - kb)];
          }
          acc[a][b][r] = v;
        }
  }
  const bool next_col = J == Kn, next_row = I == Kn;
  double* Cn = sa.Cn + (int64_t)j * N * pw;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = I * BU + wy * 32 + a * 16 + (lane >> 4) + 4 * r;
        const int col = J * BU + wx * 64 + b * 16 + (lane & 15);
        const double v = acc[a][b][r];
        // the pivot tile's upper triangle is not part of the lower storage
        if (row < N && col < N && !(in_row && in_col && row < col))
          Aj[(int64_t)row * N + col] = v;
        if (next_col && next_row) {                    // diagonal tile of the next block
          if (row < N) {
            if (col >= N) {
              Cn[(int64_t)row * pw + (col - sa.kbn)] = 0.0;
            } else if (row >= col) {
              Cn[(int64_t)row * pw + (col - sa.kbn)] = v;
              Cn[(int64_t)col * pw + (row - sa.kbn)] = v;
            }
          }
        } else if (next_col) {
          if (row < N) Cn[(int64_t)row * pw + (col - sa.kbn)] = col < N ? v : 0.0;
        } else if (next_row) {
          if (col < N) Cn[(int64_t)col * pw + (row - sa.kbn)] = row < N ? v : 0.0;
        }
      }
}

// Pivot rows / columns after the update: A(r, K) <- P[r] for r outside K;
// A(K, K) <- -D^-1 (inner: from Dinv; outer: Dw already holds it), lower
// triangle storage.
__device__ __forceinline__ void writeback_elem(const SwArgs& a, int64_t idx) {
  const int64_t NN = (int64_t)a.N * a.N;
  if (idx >= (int64_t)a.F * a.N * a.pw) return;
  const int c = (int)(idx % a.pw);
  const int r = (int)((idx / a.pw) % a.N);
  const int j = (int)(idx / ((int64_t)a.pw * a.N));
  if (c >= a.bw) return;
  const int col = a.kb + c;
  double* Aj = a.A + j * NN;
  if (r >= a.kb && r < a.kb + a.bw) {
    const int rr = r - a.kb;
    if (rr >= c)
      Aj[(int64_t)r * a.N + col] = a.Dw ? a.Dw[((int64_t)j * a.bw + rr) * a.bw + c]
                                        : -a.Dinv[((int64_t)j * B + rr) * B + c];
  } else {
    const double v = a.P[idx];
    if (r > col) Aj[(int64_t)r * a.N + col] = v;
    else Aj[(int64_t)col * a.N + r] = v;
  }
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

// W_j = -(S_j + 1) with the lower triangle of S_j mirrored, in 32 x 32
// tiles: block b of a job is lower tile (P, Q), P >= Q, of matrix j; both
// W(P, Q) and its transpose W(Q, P) are written row-contiguously through an
// LDS copy of the tile.
constexpr int FT = 32;
__device__ __forceinline__ int64_t finish_tiles(int N) {
  const int64_t T = (N + FT - 1) / FT;
  return T * (T + 1) / 2;
}

template <typename T>
__device__ __forceinline__ void finish_tile(const FinArgs& a, int64_t tile, double (*sh)[FT + 1]) {
  const int64_t NN = (int64_t)a.N * a.N, per = finish_tiles(a.N);
  const int64_t j = tile / per;
  int t = (int)(tile % per), P = 0;
  while (t > P) { t -= P + 1; ++P; }                  // t-th tile of block row P
  const int Q = t;
  const double* S = a.S + j * NN;
  T* W = static_cast<T*>(a.W) + j * NN;
  const int c = threadIdx.x % FT, r0 = threadIdx.x / FT;
#pragma unroll
  for (int k = 0; k < FT; k += 256 / FT) {
    const int r = r0 + k, gr = P * FT + r, gc = Q * FT + c;
    sh[r][c] = (gr < a.N && gc < a.N && gr >= gc) ? S[(int64_t)gr * a.N + gc] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < FT; k += 256 / FT) {
    const int r = r0 + k, gr = P * FT + r, gc = Q * FT + c;
    // element (r, c) of tile (P, Q) of the symmetric matrix
    const double sv = (P > Q || r >= c) ? sh[r][c] : sh[c][r];
    if (gr < a.N && gc < a.N) W[(int64_t)gr * a.N + gc] = (T)(-sv - (gr == gc ? 1.0 : 0.0));
    if (P > Q) {
      const int tr = Q * FT + r, tc = P * FT + c;     // element (r, c) of tile (Q, P)
      if (tr < a.N && tc < a.N) W[(int64_t)tr * a.N + tc] = (T)(-sh[c][r]);
    }
  }
  __syncthreads();
}

template <typename T>
__global__ void finish_batched_kernel(Batch bt) {
  __shared__ double sh[FT][FT + 1];
  FinArgs a;
  int64_t first;
  if (!block_of(bt, a, first)) return;
  finish_tile<T>(a, first / kBatchElems, sh);
}

// ------------------------------------------------------------------ host

// One set of F matrices of order N being swept, and its scratch.
struct SweepSet {
  double* A;
  int N, F, flag_base;
};

constexpr int BO = 256;   // widest pivot block
constexpr int BI = 128;   // pivot blocks swept whole in one workgroup
static_assert(BI == BU, "the fused update takes one 128-tile per pivot block");
constexpr int kPivE = 4;  // register block edge of the whole-block pivot sweep

// Scratch (doubles) of a two-level sweep of the given sets.
size_t sweep_scratch(const std::vector<SweepSet>& sets) {
  size_t t = 0;
  for (const SweepSet& s : sets) {
    // panels C and P (two of each, by step parity, at width BI; one P
    // at width BO) and the pivot blocks Dw (two at width BI)
    t += 3 * (size_t)s.F * s.N * BO;
    t += (size_t)s.F * BO * BO;
    t += 4 * (size_t)s.F * BO * BI;                // width BO: C, C, P, P of the Dw sweep
    t += 2 * (size_t)s.F * BI * BI;                //   and its pivot blocks
  }
  return t;
}

// The sweep's launches are planned on the host first: every launch's
// argument structs and work-unit offsets go into one blob, uploaded with a
// single staging copy, and the launches then read their slices of it (one
// copy per sweep instead of one or two per launch).
struct SweepLaunch {
  void (*kern)(Batch);    // nullptr: a pivot kernel or a stream operation (kind)
  int kind;               // 0 pivot_batched_kernel, 1 pivot_dense_kernel<BI, kPivE>,
                          // 2 wait for event `ev`, 3 record event `ev`
  size_t args_at, off_at; // byte offsets of the SwArgs and offsets arrays in the blob
  int n, chunk, threads;
  int64_t units, grid;
  const char* what;
  int side = 0;           // 1: on the context's second stream
  int ev = 0;
};

struct SweepPlan {
  std::vector<unsigned char> blob;
  std::vector<SweepLaunch> launches;
  template <typename T>
  size_t put(const T* p, size_t count) {
    const size_t at = (blob.size() + 15) & ~size_t(15);
    blob.resize(at + count * sizeof(T));
    std::memcpy(blob.data() + at, p, count * sizeof(T));
    return at;
  }
};

// A stream operation of the lookahead: wait for (kind 2) or record (kind 3)
// event ev on the main (side 0) or second (side 1) stream.
void plan_stream_op(SweepPlan& plan, int kind, int side, int ev) {
  SweepLaunch l{nullptr, kind, 0, 0, 0, 0, 0, 0, 0, "stream op"};
  l.side = side;
  l.ev = ev;
  plan.launches.push_back(l);
}

template <typename F>
bool plan_units(SweepPlan& plan, size_t args_at, const std::vector<SwArgs>& st, F units,
                int chunk, bool elems, void (*kern)(Batch), int threads, const char* what,
                int kind = 0, int side = 0) {
  std::vector<int64_t> off(1, 0);
  for (const SwArgs& a : st) {
    const int64_t u = units(a);
    off.push_back(off.back() + (elems ? (u + kBatchElems - 1) / kBatchElems : u));
  }
  if (off.back() == 0) return false;
  const int64_t grid = chunk > 1 ? (off.back() + 8 * chunk - 1) / (8 * chunk) * (8 * chunk)
                                 : off.back();
  SweepLaunch l{kern, kind, args_at, plan.put(off.data(), off.size()), (int)st.size(), chunk,
                threads, off.back(), grid, what};
  l.side = side;
  plan.launches.push_back(l);
  return true;
}

// Plan the sweep of every set to -A^-1 with pivot blocks of width pw: B
// (each 64 x 64 pivot inverted in registers, tiles of 64), BI (each pivot
// block swept whole in the registers of one workgroup, the trailing update
// on 128-tiles) or BO (each pivot block copied and swept at width BI).
// `scr` holds sweep_scratch(sets) doubles.
void plan_sweep(SweepPlan& plan, const std::vector<SweepSet>& sets, int pw, double* scr) {
  const int n = (int)sets.size();
  // X: Dw (outer) or Dinv (inner); at width BI P and X by step parity too
  std::vector<double*> C(n), C2(n), P(n), P2(n), X(n), X2(n);
  size_t o = 0;
  for (int d = 0; d < n; ++d) {
    const SweepSet& s = sets[d];
    C[d] = scr + o;
    o += (size_t)s.F * s.N * pw;
    C2[d] = scr + o;
    o += (size_t)s.F * s.N * pw;
    P[d] = scr + o;
    o += (size_t)s.F * s.N * pw;
    X[d] = scr + o;
    o += pw > B ? (size_t)s.F * pw * pw : (size_t)s.F * B * B;
    P2[d] = P[d];
    X2[d] = X[d];
    if (pw == BI) {
      P2[d] = scr + o;
      o += (size_t)s.F * s.N * pw;
      X2[d] = scr + o;
      o += (size_t)s.F * pw * pw;
    }
  }
  double* inner_scr = scr + o;              // width BO: scratch of the pivot-block sweeps
  int T_max = 0;
  for (const SweepSet& s : sets) T_max = std::max(T_max, (s.N + pw - 1) / pw);
  for (int kt = 0; kt < T_max; ++kt) {
    std::vector<SwArgs> st;
    std::vector<SweepSet> dsets;
    for (int d = 0; d < n; ++d) {
      const SweepSet& s = sets[d];
      const int kb = kt * pw;
      if (kb >= s.N) continue;
      const int bw = std::min(pw, s.N - kb);
      // width BI: the fused update writes the next panel into the other buffer
      double* cur = (pw == BI && (kt & 1)) ? C2[d] : C[d];
      double* nxt = (pw == BI && (kt & 1)) ? C[d] : C2[d];
      const int kbn = kb + pw, bwn = std::max(0, std::min(pw, s.N - kbn));
      double* Pk = (kt & 1) ? P2[d] : P[d];
      double* Xk = (kt & 1) ? X2[d] : X[d];
      SwArgs a{s.A, cur, Pk, pw == B ? Xk : nullptr, pw > B ? Xk : nullptr, s.N, s.F,
               kb, bw, (s.N + B - 1) / B, kt, pw, s.flag_base, std::min(1024, (s.N + 15) / 16),
               nxt, kbn, bwn, 0};
      st.push_back(a);
      if (pw > BI) dsets.push_back(SweepSet{Xk, bw, s.F, s.flag_base});
    }
    const size_t at = plan.put(st.data(), st.size());
    if (pw != BI || kt == 0)
      plan_units(plan, at, st, [](const SwArgs& a) { return (int64_t)a.F * a.N * a.pw; }, 1, true,
                 gather_panel_batched_kernel, 256, "gather_panel");
    if (pw == B) {
      plan_units(plan, at, st, [](const SwArgs& a) { return (int64_t)a.F; }, 1, false, nullptr,
                 PIV_THREADS, "pivot_batched_kernel");
      plan_units(plan, at, st, [](const SwArgs& a) { return (int64_t)a.F * a.panel_blocks; }, 1,
                 false, panel_batched_kernel, 256, "panel_batched_kernel");
    } else if (pw > BI) {
      // copies of the pivot blocks, swept at width BI
      plan_units(plan, at, st, [](const SwArgs& a) { return (int64_t)a.F * a.bw * a.bw; }, 1,
                 true, extract_pivot_batched_kernel, 256, "extract_pivot");
      plan_sweep(plan, dsets, BI, inner_scr);
      plan_units(plan, at, st,
                 [](const SwArgs& a) { return (int64_t)a.F * ((a.N + B - 1) / B) * (a.pw / B); },
                 8, false, panel_gemm_batched_kernel, 256, "panel_gemm");
    } else {
      // the pivot block of every matrix swept whole by one workgroup
      plan_units(plan, at, st, [](const SwArgs& a) { return (int64_t)a.F; }, 1, false, nullptr,
                 PivDense<BI, kPivE>::THREADS, "pivot_dense_kernel", 1);
      plan_units(plan, at, st,
                 [](const SwArgs& a) { return (int64_t)a.F * ((a.N + BU - 1) / BU); }, 8, false,
                 panel128_kernel, 512, "panel128_kernel");
    }
    if (pw == BI) {
      // Update, write-back and the next panel in one pass, split in two
      // launches: the tiles of the next panel's row and column (mode 1, main
      // stream) and the others (mode 2, second stream).  The next step's
      // pivot and panel need only the first, so they run on the main stream
      // while the second stream finishes this step's update (P and Dw are
      // double-buffered by step parity for that).  Mode 1 of step kt + 1
      // rewrites the panel buffer that mode 2 of step kt reads, and the
      // tiles it updates are updated by mode 2 of step kt: it waits for it.
      // The two modes of one step start together (mode 1 alone fills a
      // fraction of the GPU: run first on its own it made the step slower).
      std::vector<SwArgs> s1 = st, s2 = st;
      for (SwArgs& a : s1) a.mode = 1;
      for (SwArgs& a : s2) a.mode = 2;
      const size_t at1 = plan.put(s1.data(), s1.size());
      const size_t at2 = plan.put(s2.data(), s2.size());
      plan_stream_op(plan, 3, 0, 0);              // this step's pivot and panel are done
      if (kt > 0) plan_stream_op(plan, 2, 0, 1);  // the previous step's mode 2 is done
      plan_units(plan, at1, s1,
                 [](const SwArgs& a) {
                   return a.bwn > 0 ? (int64_t)a.F * ((a.N + BU - 1) / BU) : 0;
                 },
                 8, false, update_fused_kernel, 512, "update_fused_kernel");
      plan_stream_op(plan, 2, 1, 0);
      plan_units(plan, at2, s2,
                 [](const SwArgs& a) {
                   const int64_t t = (a.N + BU - 1) / BU;
                   return (int64_t)a.F * (a.bwn > 0 ? (t - 1) * t / 2 : t * (t + 1) / 2);
                 },
                 8, false, update_fused_kernel, 512, "update_fused_kernel", 0, 1);
      plan_stream_op(plan, 3, 1, 1);
      continue;
    }
    if (pw > B) {
      plan_units(plan, at, st,
                 [](const SwArgs& a) {
                   const int64_t t = (a.N + BU - 1) / BU;
                   return (int64_t)a.F * t * (t + 1) / 2;
                 },
                 8, false, update128_batched_kernel, 512, "update128_kernel");
    } else {
      plan_units(plan, at, st, [](const SwArgs& a) { return (int64_t)a.F * a.T * (a.T + 1) / 2; },
                 8, false, update_batched_kernel, 256, "update_kernel");
    }
    plan_units(plan, at, st, [](const SwArgs& a) { return (int64_t)a.F * a.N * a.pw; }, 1, true,
               writeback_batched_kernel, 256, "writeback");
  }
  if (pw == BI && T_max > 0) plan_stream_op(plan, 2, 0, 1);   // join the second stream
}

gw_status sweep(gw_ctx ctx, const std::vector<SweepSet>& sets, int pw, double* scr) {
  SweepPlan plan;
  plan_sweep(plan, sets, pw, scr);
  if (plan.launches.empty()) return GW_OK;
  const unsigned char* dev =
      static_cast<const unsigned char*>(gw::stage(ctx, plan.blob.data(), plan.blob.size()));
  if (!dev) return GW_EINVAL;
  bool two = false;
  for (const SweepLaunch& l : plan.launches) two = two || l.side != 0;
  if (two && !ctx->side_stream) {
    // default priority, like every stream of the library
    GW_HIP(ctx, hipStreamCreateWithFlags(&ctx->side_stream, hipStreamNonBlocking));
    for (hipEvent_t& e : ctx->side_ev)
      GW_HIP(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  for (const SweepLaunch& l : plan.launches) {
    hipStream_t st = l.side ? ctx->side_stream : ctx->stream;
    if (l.kind == 2 && !l.kern) {
      if (two) GW_HIP(ctx, hipStreamWaitEvent(st, ctx->side_ev[l.ev], 0));
      continue;
    }
    if (l.kind == 3 && !l.kern) {
      if (two) GW_HIP(ctx, hipEventRecord(ctx->side_ev[l.ev], st));
      continue;
    }
    const Batch bt{reinterpret_cast<const SwArgs*>(dev + l.args_at),
                   reinterpret_cast<const int64_t*>(dev + l.off_at), l.n, l.chunk, l.units};
    if (l.kern)
      hipLaunchKernelGGL(l.kern, dim3((unsigned)l.grid), dim3(l.threads), 0, st, bt);
    else if (l.kind == 1)
      hipLaunchKernelGGL((pivot_dense_kernel<BI, kPivE>), dim3((unsigned)l.grid), dim3(l.threads), 0,
                         st, bt, ctx->d_flags);
    else
      hipLaunchKernelGGL(pivot_batched_kernel, dim3((unsigned)l.grid), dim3(l.threads), 0, st, bt,
                         ctx->d_flags);
    GW_TRY(gw::launch_check(ctx, l.what));
  }
  return GW_OK;
}

// Assemble, sweep and finish the given screening jobs (device pointers,
// staged x and omega).
struct ScreenJob {
  const double* M;      // device [L][N][N] (sum-over-states: [F][N][N] sums P_j)
  const double* x;      // device [L]
  const double* omega;  // device [F]
  int N, F;
  void* W_hat;
};

gw_status screen_jobs(gw_ctx ctx, gw_precision prec, int L, const std::vector<ScreenJob>& jobs,
                      int sos = 0) {
  size_t a_tot = 0;
  std::vector<SweepSet> sets;
  int flag_base = 0, smem = 0;
  double flops = 0, bytes = 0;
  for (const ScreenJob& j : jobs) {
    if (prec != GW_FP64) a_tot += (size_t)j.F * j.N * j.N;
    if (!sos) smem = std::max(smem, j.F * L);
  }
  double* Aws = nullptr;
  if (a_tot) {
    Aws = static_cast<double*>(gw::ws_get(ctx, WS_SCREEN_A, a_tot * sizeof(double)));
    if (!Aws) return GW_ENOMEM;
  }
  std::vector<AsmArgs> asm_d;
  std::vector<FinArgs> fin_d;
  std::vector<int64_t> n_asm, n_fin;
  size_t ao = 0;
  for (const ScreenJob& j : jobs) {
    double* A = prec == GW_FP64 ? static_cast<double*>(j.W_hat) : Aws + ao;
    if (prec != GW_FP64) ao += (size_t)j.F * j.N * j.N;
    sets.push_back(SweepSet{A, j.N, j.F, flag_base});
    flag_base += j.F;
    asm_d.push_back(AsmArgs{j.M, L, j.N, j.x, j.omega, j.F, A, sos});
    n_asm.push_back((int64_t)j.N * j.N);
    fin_d.push_back(FinArgs{A, j.N, j.F, j.W_hat});
    const int64_t T = (j.N + FT - 1) / FT;
    n_fin.push_back((int64_t)j.F * (T * (T + 1) / 2) * kBatchElems);   // one block per tile
    flops += (double)j.F * j.N * (double)j.N * j.N;
    bytes += (double)j.F * j.N * (double)j.N * 8.0 * 2.0;
  }
  double* scr = static_cast<double*>(
      gw::ws_get(ctx, WS_SCREEN_PANEL, sweep_scratch(sets) * sizeof(double)));
  if (!scr) return GW_ENOMEM;
  // assemble (the sweep works in place), sweep, finish: rerunnable as a whole
  auto run = [&](int pw, bool timed) -> gw_status {
    const int pi = timed ? gw::prof_begin(ctx) : -1;
    std::vector<int64_t> off(1, 0);
    for (int64_t nn : n_asm) off.push_back(off.back() + (nn + kBatchElems - 1) / kBatchElems);
    Batch bt;
    GW_TRY(gw::stage_batch(ctx, asm_d, off, 1, bt));
    hipLaunchKernelGGL(assemble_batched_kernel, dim3((unsigned)off.back()), dim3(256),
                       (size_t)smem * sizeof(double), ctx->stream, bt);
    GW_TRY(gw::launch_check(ctx, "assemble_batched_kernel"));
    GW_TRY(sweep(ctx, sets, pw, scr));
    if (timed) gw::prof_end(ctx, pi, "screen_sweep", flops, bytes);
    return gw::elementwise_batched(ctx, fin_d, n_fin,
                                   prec == GW_FP64 ? finish_batched_kernel<double>
                                                   : finish_batched_kernel<float>,
                                   "finish_batched_kernel");
  };
  // outer pivot width: the rank of the trailing update (autotuned per shape)
  std::string key = sos ? "screen_sos" : "screen";
  for (const ScreenJob& j : jobs) key += ":" + std::to_string(j.N) + "x" + std::to_string(j.F);
  const int pw = gw::tune(ctx, key, {BO, 128, B}, [&](int c) { return run(c, false); });
  return run(pw, true);
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
  const double* dx = gw::stage_t(ctx, x_lt, n_lt);
  const double* dw = gw::stage_t(ctx, omega, n_w);
  if (!dx || !dw) return GW_EINVAL;
  return screen_jobs(ctx, prec, n_lt, {ScreenJob{M, dx, dw, n_naf, n_w, W_hat}});
}

extern "C" gw_status gw_screen_sos(gw_ctx ctx, gw_precision prec, int n_naf, int n_w,
                                   const double* P, void* W_hat) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_screen_sos: ctx is NULL");
  gw::clear_error(ctx);
  GW_REQUIRE(ctx, prec == GW_FP64 || prec == GW_FP32 || prec == GW_BF16X3,
             "gw_screen_sos: unknown precision %d", (int)prec);
  GW_REQUIRE(ctx, n_naf >= 1 && n_w >= 1, "gw_screen_sos: bad sizes (n_naf=%d n_w=%d)", n_naf,
             n_w);
  GW_REQUIRE(ctx, P && W_hat, "gw_screen_sos: NULL argument");
  GW_HIP(ctx, hipSetDevice(ctx->device));
  return screen_jobs(ctx, prec, 1, {ScreenJob{P, nullptr, nullptr, n_naf, n_w, W_hat}}, 1);
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
  std::vector<ScreenJob> sj;
  for (int d = 0; d < n_jobs; ++d) {
    const gw_screen_job& j = jobs[d];
    const double* dx = gw::stage_t(ctx, j.x_lt, n_lt);
    const double* dw = gw::stage_t(ctx, j.omega, j.n_w);
    if (!dx || !dw) return GW_EINVAL;
    sj.push_back(ScreenJob{j.M, dx, dw, j.n_naf, j.n_w, j.W_hat});
  }
  return screen_jobs(ctx, prec, n_lt, sj);
}

namespace gw {

void screen_ws_bytes(gw_precision prec, int N, int F, size_t* a_bytes, size_t* panel_bytes) {
  *a_bytes = prec == GW_FP64 ? 0 : (size_t)F * N * N * sizeof(double);
  *panel_bytes = sweep_scratch({SweepSet{nullptr, N, F, 0}}) * sizeof(double);
}

}  // namespace gw
