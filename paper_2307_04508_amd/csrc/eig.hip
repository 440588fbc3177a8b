// Eigenpairs of the NAF metric (Eq. 12) after its on-chip reduction to
// tridiagonal form (tridiag.hip), with no library calls:
//
//  * eigenvalues by multisection on Sturm counts, per unreduced block of the
//    tridiagonal matrix T: 8 to 32 lanes per eigenvalue evaluate as many
//    points of its bracket per round;
//  * the kept eigenvectors of isolated eigenvalues from the twisted
//    factorisation of T - lambda I, one wave per vector; clusters (gaps
//    below 1e-10 ||T|| inside one block) by inverse iteration, one thread
//    per cluster: an LU factorisation with partial pivoting (tiny pivots
//    replaced by eps ||T||), two solves from a pseudo-random start, the
//    cluster's vectors Gram-Schmidt-orthogonalised against each other;
//  * one Newton-Schulz step Z <- (3 I - Z Z^T) Z / 2 on the kept vectors
//    (rows of Z): the solves leave inner products of order eps ||T|| / gap
//    between neighbours, the step squares them away;
//  * the back-transformation with the Householder reflectors in blocks of
//    256 in compact WY form, Z <- Z (I - V T V^T)^T block by block.
//
// The dense products run on an FP64 MFMA GEMM (v_mfma_f64_16x16x4f64, 128 x
// 128 tiles, register double-buffered) in the two layouts the method needs:
// "NT" C[m][n] = sum_k A[m][k] B[n][k] and "TN" C[m][n] = sum_k A[k][m]
// B[k][n], all row-major, split-K with a fixed-order reduction.
#include <algorithm>
#include <limits>
#include <cmath>
#include <vector>

#include "common.hpp"

namespace {

constexpr int GBM = 128;
constexpr int GBK = 16;
constexpr int GLD = GBM + 1;        // padded LDS row (k-major tiles)

struct G64 {
  const double* A;
  const double* B;
  double* C;
  int M, N, K;
  int64_t lda, ldb, ldc;
  double alpha, beta;       // C = alpha (A B) + beta C; beta == 0: C is not read
  int tm, tn;               // tiles along M and N
  // split K in the kernel (a descriptor passed by value): unit u takes
  // split u / (tm tn), k in [s kper, (s + 1) kper), C + s cstride
  int splits, kper;
  int64_t cstride;
};

// Register stage of one operand: 8 consecutive elements of one row.  A
// k-major operand ([k][rows]) is read 16 k x 128 rows as row k = tid >> 4,
// elements (tid & 15) * 8 ..; a row-major one ([rows][k]) as row tid >> 1,
// k = (tid & 1) * 8 ..  Both land k-major in LDS ([k][row]).
template <bool KMAJ>
__device__ __forceinline__ void dg_load(const double* __restrict__ P, int64_t ld, int lim, int r0,
                                        int k0, int K, int tid, double (&reg)[8]) {
  if (KMAJ) {
    const int k = k0 + (tid >> 4), c = r0 + (tid & 15) * 8;
#pragma unroll
    for (int e = 0; e < 8; ++e)
      reg[e] = (k < K && c + e < lim) ? P[(int64_t)k * ld + c + e] : 0.0;
  } else {
    const int r = r0 + (tid >> 1), k = k0 + (tid & 1) * 8;
#pragma unroll
    for (int e = 0; e < 8; ++e)
      reg[e] = (r < lim && k + e < K) ? P[(int64_t)r * ld + k + e] : 0.0;
  }
}

template <bool KMAJ>
__device__ __forceinline__ void dg_store(double (*S)[GLD], int tid, const double (&reg)[8]) {
  if (KMAJ) {
    const int k = tid >> 4, c = (tid & 15) * 8;
#pragma unroll
    for (int e = 0; e < 8; ++e) S[k][c + e] = reg[e];
  } else {
    const int r = tid >> 1, k = (tid & 1) * 8;
#pragma unroll
    for (int e = 0; e < 8; ++e) S[k + e][r] = reg[e];
  }
}

// One 128 x 128 tile of C = alpha op(A) op(B) (+ beta C) per workgroup, 4
// waves of 64 x 64.  AK: A stored [k][m] (else [m][k]); BK: B stored [k][n]
// (else [n][k]).  Operand tiles of 16 k are staged k-major in LDS from
// registers loaded one stage ahead.
template <bool AK, bool BK>
__global__ __launch_bounds__(256, 2) void dgemm_kernel(Batch bt, G64 a0) {
  __shared__ double As[2][GBK][GLD];
  __shared__ double Bs[2][GBK][GLD];
  G64 g;
  int64_t lid;
  if (!unit_of(a0, bt, g, lid)) return;
  if (g.splits > 1) {
    const int64_t per = (int64_t)g.tm * g.tn;
    const int sp = (int)(lid / per);
    lid -= sp * per;
    const int k0 = min(g.K, sp * g.kper);
    g.K = min(g.K - k0, g.kper);
    g.A += AK ? (int64_t)k0 * g.lda : k0;
    g.B += BK ? (int64_t)k0 * g.ldb : k0;
    g.C += sp * g.cstride;
  }
  const int tn_ = (int)(lid % g.tn), tm_ = (int)(lid / g.tn);
  const int m0 = tm_ * GBM, n0 = tn_ * GBM;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wy = wave >> 1, wx = wave & 1;

  f64x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};

  double ra[8], rb[8];
  const int nk = (g.K + GBK - 1) / GBK;
  if (nk > 0) {
    dg_load<AK>(g.A, g.lda, g.M, m0, 0, g.K, tid, ra);
    dg_load<BK>(g.B, g.ldb, g.N, n0, 0, g.K, tid, rb);
    dg_store<AK>(As[0], tid, ra);
    dg_store<BK>(Bs[0], tid, rb);
  }
  __syncthreads();
  for (int it = 0; it < nk; ++it) {
    const int cur = it & 1;
    if (it + 1 < nk) {
      dg_load<AK>(g.A, g.lda, g.M, m0, (it + 1) * GBK, g.K, tid, ra);
      dg_load<BK>(g.B, g.ldb, g.N, n0, (it + 1) * GBK, g.K, tid, rb);
    }
#pragma unroll
    for (int kk = 0; kk < GBK / 4; ++kk) {
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
    if (it + 1 < nk) {
      dg_store<AK>(As[cur ^ 1], tid, ra);
      dg_store<BK>(Bs[cur ^ 1], tid, rb);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wy * 64 + i * 16 + (lane >> 4) + 4 * r;
        const int col = n0 + wx * 64 + j * 16 + (lane & 15);
        if (row < g.M && col < g.N) {
          double* c = g.C + (int64_t)row * g.ldc + col;
          const double v = g.alpha * acc[i][j][r];
          *c = g.beta != 0.0 ? v + g.beta * *c : v;
        }
      }
}

// dst[m][n] = sum_s part[s][m][n] + beta dst[m][n] (fixed order over s).
struct SumArgs {
  const double* part;       // [S][M][N] contiguous
  int S, M, N;
  double* dst;
  int64_t ldd;
  double beta;
};

__global__ void sum_partials_kernel(SumArgs a) {
  const int64_t total = (int64_t)a.M * a.N;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int s = 0; s < a.S; ++s) v += a.part[(int64_t)s * total + idx];
    double* d = a.dst + (idx / a.N) * a.ldd + idx % a.N;
    *d = a.beta != 0.0 ? v + a.beta * *d : v;
  }
}

inline int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  return (int)std::min<int64_t>(std::max<int64_t>(g, 1), 65536);
}

// ------------------------------------------------------------ tridiagonal

// Sturm step q <- dx - e2 / q with the hardware reciprocal estimate r of q
// (relative error below 2^-22): 1 / q = r (1 + t), t = e + e^2, e = 1 - q r,
// exact to O(e^3), leaves three dependent operations after the estimate.
__device__ __forceinline__ double sturm_step(double q, double dx, double e2) {
  const double r = __builtin_amdgcn_rcp(q);
  const double e = fma(-q, r, 1.0);
  const double er = e2 * r;
  const double t = fma(e, e, e);
  return fma(-er, t, dx - er);
}

// 1 / p to about one rounding (same expansion).
__device__ __forceinline__ double rcp64(double p) {
  const double r = __builtin_amdgcn_rcp(p);
  const double e = fma(-p, r, 1.0);
  return fma(r, fma(e, e, e), r);
}


// Number of eigenvalues of the block (d[0..nb), e2[0..nb-1) squared
// couplings) below x: the signs of the LDL^T pivots of T - x I, a pivot
// smaller than pivmin taken as -pivmin.
__device__ __forceinline__ int sturm_count(const double* __restrict__ d,
                                           const double* __restrict__ e2, int nb, double x,
                                           double pivmin) {
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int c = q < 0.0;
  int i0 = 1;
  for (; i0 + 8 <= nb; i0 += 8) {
    double dd[8], ee[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      dd[j] = d[i0 + j];
      ee[j] = e2[i0 + j - 1];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      q = sturm_step(q, dd[j] - x, ee[j]);
      if (fabs(q) < pivmin) q = -pivmin;
      c += q < 0.0;
    }
  }
  for (; i0 < nb; ++i0) {
    q = sturm_step(q, d[i0] - x, e2[i0 - 1]);
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
  }
  return c;
}

struct BisBlock {
  int s, nb;                // rows s .. s + nb - 1 of T
  double gl, gu;            // a bracket of its eigenvalues
  int out;                  // index in lam of its first computed eigenvalue
  int j0;                   // its first computed eigenvalue (ascending index)
};

struct BisArgs {
  const double* d;
  const double* e2;         // squared couplings, zero at the splits
  const BisBlock* blocks;
  int n_blocks, n;          // n: eigenvalues computed
  double pivmin, abstol;
  double* lam;              // [n]: each block's computed eigenvalues ascending from its out
  int rows;                 // order of T (d and e2 have rows entries)
};

// kBisLanes lanes per eigenvalue count at as many points of its bracket,
// which shrinks (kBisLanes + 1)-fold per round.  The Sturm sequences are
// bound by FP64 issue, not latency, so fewer points per round (more rounds,
// less work) pay while the lanes fill the chip: 32 -> 16 lanes took all
// 3000 eigenvalues from 2.23 to 1.65 ms, 8 lanes all 7000 from 10.4 to 5.6
// ms; the launch picks the count from the number of eigenvalues it computes.
// SH: the workgroup first copies
// d and e2 into LDS (dynamic, 2 n doubles), so the operand loads are LDS
// reads instead of L2 round trips.
constexpr int kBisShMax = 4096;     // orders whose d and e2 fit 64 KB of LDS
template <bool SH, int kBisLanes>
__global__ __launch_bounds__(256) void bisect_kernel(BisArgs a) {
  extern __shared__ double bsh[];
  const double* dd = a.d;
  const double* ee = a.e2;
  if (SH) {
    for (int x = threadIdx.x; x < a.rows; x += blockDim.x) {
      bsh[x] = a.d[x];
      bsh[a.rows + x] = a.e2[x];
    }
    __syncthreads();
    dd = bsh;
    ee = bsh + a.rows;
  }
  const int64_t gt = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int u = (int)(gt / kBisLanes), q = (int)(gt % kBisLanes);
  const int group = (threadIdx.x & 63) / kBisLanes;
  const bool live = u < a.n;
  int lo_b = 0, hi_b = a.n_blocks - 1;      // block of eigenvalue u: last out <= u
  while (live && lo_b < hi_b) {
    const int mid = (lo_b + hi_b + 1) >> 1;
    if (a.blocks[mid].out <= u) lo_b = mid; else hi_b = mid - 1;
  }
  const BisBlock b = a.blocks[live ? lo_b : 0];
  const int j = b.j0 + (u - b.out);
  double lo = b.gl, hi = b.gu;
  const double eps = 1.1102230246251565e-16;
  for (int round = 0; round < 64; ++round) {
    const bool done = !live || hi - lo <= 2.0 * eps * fmax(fabs(lo), fabs(hi)) + a.abstol;
    // every lane of the wave takes part in the ballots; finished groups vote 0
    if (!__ballot(!done)) break;
    const double h = (hi - lo) * (1.0 / (kBisLanes + 1));
    const double x = lo + (q + 1) * h;
    const int c = done ? 0 : sturm_count(dd + b.s, ee + b.s, b.nb, x, a.pivmin);
    const uint64_t bal = __ballot(!done && c > j);
    if (!done) {
      const uint64_t gb = (bal >> (kBisLanes * group)) &
                          (kBisLanes == 64 ? ~0ull : ((1ull << kBisLanes) - 1));
      const int qs = gb ? __ffsll((unsigned long long)gb) - 1 : kBisLanes;  // first point above
      const double nlo = qs == 0 ? lo : lo + qs * h;
      const double nhi = qs == kBisLanes ? hi : lo + (qs + 1) * h;
      lo = nlo;
      hi = nhi;
    }
  }
  if (live && q == 0) a.lam[u] = 0.5 * (lo + hi);
}

// Inverse iteration for what twisted_kernel leaves: clusters (each led by one
// thread) and isolated eigenvalues it marked (every vector when lu_all is
// set and twisted_kernel does not run).  One vector per thread, only
// kInvLanes lanes of each 64-thread workgroup active, so that the serial
// passes' loads (one cache line per lane) spread over more compute units
// (A = 3000: 3.19 ms with 64 lanes, 2.51 ms with 8).  Per-thread arrays live in
// scratch, each thread's contiguous ([thread][array][i]): 0 reciprocal
// pivot, 1 and 2 the two superdiagonals of U, 3 the multiplier, 4 the
// vector, 5 the interchange flag of row pair (k, k + 1).  (Interleaved over
// the threads, [array][i][thread], the loads coalesce, but every element's
// address took its own 64-bit arithmetic: 523 spilled SGPRs, 3.7 ms at
// A = 3000 against 3.2 ms.)  The serial passes read their operands in
// chunks of kInvCh elements, the next chunk's loads issued before the current
// chunk is computed, so memory latency overlaps the dependent arithmetic.
constexpr int kInvArrays = 6;

constexpr int kInvCh = 8;           // prefetch chunk of the inverse-iteration passes
constexpr int kInvStatus = 5;       // array whose element 0 holds twisted_kernel's status
constexpr int kInvLanes = 8;        // active lanes per workgroup of invit_kernel

struct InvJob {
  int s, nb;                // block rows
  double lam;
  int row;                  // output row of Z
  int clen;                 // vectors this thread computes (0: done by a leader)
};

struct InvArgs {
  const double* d;
  const double* e;          // couplings, zero at the splits
  const InvJob* jobs;
  int n_jobs, n;
  double tiny;              // eps ||T||: smallest pivot magnitude
  double* Z;                // [rows][ldz]
  int64_t ldz;
  double* scratch;          // [n_jobs][kInvArrays][n]
  int lanes;                // active lanes per 64-thread workgroup (1..64)
  int lu_all;               // every vector by inverse iteration (twisted_kernel not run)
};

__device__ __forceinline__ double rand_pm1(uint64_t key) {
  uint64_t z = key * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Run body(c0, A, B) over chunks c0 = first, first + step, ... while
// more(c0), alternating the two register sets: body loads the chunk after
// c0 into its third argument and computes c0 from its second.
template <typename R, typename F, typename M>
__device__ __forceinline__ void ping_pong(int first, int step, M more, R& A, R& B, F body) {
  for (int c0 = first; more(c0);) {
    body(c0, A, B);
    c0 += step;
    if (!more(c0)) break;
    body(c0, B, A);
    c0 += step;
  }
}

__global__ __launch_bounds__(64) void invit_kernel(InvArgs a) {
  if ((int)threadIdx.x >= a.lanes) return;
  const int t = blockIdx.x * a.lanes + threadIdx.x;
  if (t >= a.n_jobs) return;
  const InvJob lead = a.jobs[t];
  if (lead.clen == 0) return;
  // an isolated eigenvalue whose vector twisted_kernel has written
  if (lead.clen == 1 && !a.lu_all &&
      a.scratch[(int64_t)t * kInvArrays * a.n + kInvStatus * a.n] == 0.0)
    return;
  // each thread's arrays are contiguous, [thread][array][i]: the addresses
  // of a chunk are one base plus constant offsets (no per-element address
  // arithmetic), at the cost of one cache line per lane per load
  constexpr int64_t st = 1;
  const int64_t plane = a.n;
  double* rp = a.scratch + (int64_t)t * kInvArrays * a.n;
  double* u1 = rp + plane;
  double* u2 = u1 + plane;
  double* mm = u2 + plane;
  double* y = mm + plane;
  double* fl = y + plane;
  const int s = lead.s, nb = lead.nb;
  const double* __restrict__ d = a.d + s;
  const double* __restrict__ e = a.e + s;
  const double tiny = a.tiny;
  for (int c = 0; c < lead.clen; ++c) {
    const InvJob jb = a.jobs[t + c];
    const double lam = jb.lam;
    const uint64_t key = (uint64_t)jb.row << 32;
    // T - lam I = P L U, rows k and k + 1 interchanged when the coupling
    // below the pivot is larger; |multiplier| <= 1
    {
      struct R { double dn[kInvCh], en[kInvCh]; } A, B;
      double ak = d[0] - lam, bk = nb > 1 ? e[0] : 0.0, ck = bk;
      auto load = [&](int k0, R& r) {
#pragma unroll
        for (int j = 0; j < kInvCh; ++j) {
          const int k = k0 + j;
          r.dn[j] = k + 1 < nb ? d[k + 1] : 0.0;
          r.en[j] = k + 2 < nb ? e[k + 1] : 0.0;
        }
      };
      load(0, A);
      ping_pong(0, kInvCh, [&](int k0) { return k0 + 1 < nb; }, A, B, [&](int k0, R& cur, R& nxt) {
        if (k0 + kInvCh + 1 < nb) load(k0 + kInvCh, nxt);
#pragma unroll
        for (int j = 0; j < kInvCh; ++j) {
          const int k = k0 + j;
          if (k + 1 < nb) {
            const double a1 = cur.dn[j] - lam, b1 = cur.en[j];
            const bool sw = fabs(ak) < fabs(ck);
            double p = sw ? ck : ak;
            if (fabs(p) < tiny) p = copysign(tiny, p);
            const double r = rcp64(p);
            const double m = (sw ? ak : ck) * r;
            rp[k * st] = r;
            u1[k * st] = sw ? a1 : bk;
            u2[k * st] = sw ? b1 : 0.0;
            mm[k * st] = m;
            fl[k * st] = sw ? 1.0 : 0.0;
            const double nak = sw ? bk - m * a1 : a1 - m * bk;
            bk = sw ? -m * b1 : b1;
            ak = nak;
            ck = b1;
          }
        }
      });
      if (fabs(ak) < tiny) ak = copysign(tiny, ak);
      rp[(int64_t)(nb - 1) * st] = rcp64(ak);
    }
    // two sweeps from a pseudo-random start; fin scales the sweep's input
    // (the previous sweep's normalisation, applied on load)
    double fin = 1.0;
    for (int sweep = 0; sweep < 2; ++sweep) {
      // y <- L^-1 P y; cur carries the running y[k]
      double run = (sweep == 0 ? rand_pm1(key) : y[0] * fin);
      {
        struct R { double f[kInvCh], m[kInvCh], nx[kInvCh]; } A, B;
        auto load = [&](int k0, R& r) {
#pragma unroll
          for (int j = 0; j < kInvCh; ++j) {
            const int k = k0 + j;
            r.f[j] = k + 1 < nb ? fl[k * st] : 0.0;
            r.m[j] = k + 1 < nb ? mm[k * st] : 0.0;
            r.nx[j] = k + 1 < nb ? (sweep == 0 ? rand_pm1(key + (uint64_t)(k + 1))
                                               : y[(int64_t)(k + 1) * st] * fin)
                                 : 0.0;
          }
        };
        load(0, A);
        ping_pong(0, kInvCh, [&](int k0) { return k0 + 1 < nb; }, A, B,
                  [&](int k0, R& cur, R& nxt) {
          if (k0 + kInvCh + 1 < nb) load(k0 + kInvCh, nxt);
#pragma unroll
          for (int j = 0; j < kInvCh; ++j) {
            if (k0 + j + 1 < nb) {
              const bool sw = cur.f[j] != 0.0;
              const double out = sw ? cur.nx[j] : run;
              run = (sw ? run : cur.nx[j]) - cur.m[j] * out;
              y[(int64_t)(k0 + j) * st] = out;
            }
          }
        });
      }
      // x <- U^-1 y (two superdiagonals), in place from the bottom, with
      // the largest entry and the sum of squares
      double x1 = run * rp[(int64_t)(nb - 1) * st], x2 = 0.0;
      y[(int64_t)(nb - 1) * st] = x1;
      double big = fabs(x1), ss = x1 * x1;
      {
        struct R { double r[kInvCh], v1[kInvCh], v2[kInvCh], yy[kInvCh]; } A, B;
        auto load = [&](int k1, R& r) {
#pragma unroll
          for (int j = 0; j < kInvCh; ++j) {
            const int k = k1 - j;
            r.r[j] = k >= 0 ? rp[k * st] : 0.0;
            r.v1[j] = k >= 0 ? u1[k * st] : 0.0;
            r.v2[j] = k >= 0 ? u2[k * st] : 0.0;
            r.yy[j] = k >= 0 ? y[k * st] : 0.0;
          }
        };
        load(nb - 2, A);
        ping_pong(nb - 2, -kInvCh, [&](int k1) { return k1 >= 0; }, A, B,
                  [&](int k1, R& cur, R& nxt) {
          if (k1 - kInvCh >= 0) load(k1 - kInvCh, nxt);
#pragma unroll
          for (int j = 0; j < kInvCh; ++j) {
            if (k1 - j >= 0) {
              const double x0 = (cur.yy[j] - cur.v1[j] * x1 - cur.v2[j] * x2) * cur.r[j];
              y[(int64_t)(k1 - j) * st] = x0;
              big = fmax(big, fabs(x0));
              ss += x0 * x0;
              x2 = x1;
              x1 = x0;
            }
          }
        });
      }
      if (c > 0 || !(ss > 0.0 && ss < 1e300)) {
        // a cluster, or a sum of squares out of range: scale by the largest
        // entry, Gram-Schmidt against the cluster's earlier vectors
        const double f = big > 0.0 ? 1.0 / big : 0.0;
        for (int i = 0; i < nb; ++i) y[(int64_t)i * st] *= f;
        for (int c2 = 0; c2 < c; ++c2) {
          const double* zp = a.Z + (int64_t)a.jobs[t + c2].row * a.ldz + s;
          double dot = 0.0;
          for (int i = 0; i < nb; ++i) dot += zp[i] * y[(int64_t)i * st];
          for (int i = 0; i < nb; ++i) y[(int64_t)i * st] -= dot * zp[i];
        }
        ss = 0.0;
        for (int i = 0; i < nb; ++i) ss += y[(int64_t)i * st] * y[(int64_t)i * st];
      }
      fin = ss > 0.0 ? 1.0 / sqrt(ss) : 0.0;
    }
    // the normalised vector into its row of Z, zeros outside the block
    double* z = a.Z + (int64_t)jb.row * a.ldz;
    for (int i = 0; i < s; ++i) z[i] = 0.0;
    {
      struct R { double v[kInvCh]; } A, B;
      auto load = [&](int i0, R& r) {
#pragma unroll
        for (int j = 0; j < kInvCh; ++j) r.v[j] = i0 + j < nb ? y[(int64_t)(i0 + j) * st] : 0.0;
      };
      load(0, A);
      ping_pong(0, kInvCh, [&](int i0) { return i0 < nb; }, A, B, [&](int i0, R& cur, R& nxt) {
        if (i0 + kInvCh < nb) load(i0 + kInvCh, nxt);
#pragma unroll
        for (int j = 0; j < kInvCh; ++j)
          if (i0 + j < nb) z[s + i0 + j] = cur.v[j] * fin;
      });
    }
    for (int i = s + nb; i < a.n; ++i) z[i] = 0.0;
  }
}

// Eigenvector of an isolated eigenvalue lam from the twisted factorisation
// of T - lam I (Fernando; Parlett and Dhillon): the top-down pivots
// D+_i = d_i - lam - e_{i-1}^2 / D+_{i-1} and the bottom-up pivots
// D-_i = d_i - lam - e_i^2 / D-_{i+1} give, for every twist index r,
// gamma_r = D+_r + D-_r - (d_r - lam), the reciprocal of the r-th diagonal
// entry of (T - lam I)^-1.  At r = argmin |gamma_r| the solution of
// (T - lam I) z = gamma_r e_r with z_r = 1 is z_i = -(e_i / D+_i) z_{i+1}
// above r and z_i = -(e_{i-1} / D-_i) z_{i-1} below it: one solve from the
// best possible start vector, with residual |gamma_r| / ||z||.
// One wave per job: lanes 0 and 1 run the two pivot recurrences side by
// side (the only serial part), the wave takes the argmin, then builds z in
// chunks of 64 by prefix products across the lanes, and normalises it (the
// sign as below).
// Pivots below eps ||T|| in magnitude are replaced by +-eps ||T||, as in the
// Sturm counts.  A sum of squares out of range marks the job for
// invit_kernel (status 1); status 0 means the row of Z is final.
// Scratch per job: [kInvArrays][n], arrays 0-3 D+, e_i / D+_i, D-,
// e_{i-1} / D-_i; element 0 of array kInvStatus the status.
__global__ __launch_bounds__(64) void twisted_kernel(InvArgs a) {
  const int t = blockIdx.x;
  const InvJob jb = a.jobs[t];
  if (jb.clen != 1) return;                         // clusters: invit_kernel
  const int lane = threadIdx.x;
  const int s = jb.s, nb = jb.nb;
  const double* __restrict__ d = a.d + s;
  const double* __restrict__ e = a.e + s;
  const double lam = jb.lam, tiny = a.tiny;
  const int64_t plane = a.n;
  double* base = a.scratch + (int64_t)t * kInvArrays * plane;
  double* piv_f = base;
  double* mul_f = base + plane;
  double* piv_b = base + 2 * plane;
  double* mul_b = base + 3 * plane;
  double* status = base + kInvStatus * plane;
  if (lane < 2) {
    // step k handles row k (top-down) or row nb - 1 - k (bottom-up); cn is
    // the coupling to the row the next step handles
    const bool fwd = lane == 0;
    double* piv = fwd ? piv_f : piv_b;
    double* mul = fwd ? mul_f : mul_b;
    // coupling of row i to the next row in this direction: e[i] top-down,
    // e[i - 1] bottom-up
    const double* ep = fwd ? e : e - 1;
    double g = 0.0, cprev = 0.0;
    struct R { double dd[kInvCh], cn[kInvCh]; } A, B;
    // Loads without branches or selects (indices clamped into the block;
    // e + s has at least one entry), so that the compiler can leave the
    // prefetched chunk in flight: a load in a branch, or a select on its
    // value, costs a wait for every outstanding access, the prefetch too.
    auto load = [&](int k0, R& r) {
#pragma unroll
      for (int j = 0; j < kInvCh; ++j) {
        const int k = min(k0 + j, nb - 1);
        const int i = fwd ? k : nb - 1 - k;
        r.dd[j] = d[i];
        r.cn[j] = ep[fwd ? i : max(i, 1)];
      }
    };
    auto step = [&](int k, double dd, double craw) {
      const int i = fwd ? k : nb - 1 - k;
      const double cn = k + 1 < nb ? craw : 0.0;
      double x = (dd - lam) - cprev * g;
      if (fabs(x) < tiny) x = copysign(tiny, x);
      g = cn * rcp64(x);
      piv[i] = x;
      mul[i] = g;
      cprev = cn;
    };
    // two whole chunks per trip with no guard, then at most two guarded
    // chunks; the next chunk is always in flight while one is computed
    load(0, A);
    int k0 = 0;
    for (; k0 + 2 * kInvCh <= nb; k0 += 2 * kInvCh) {
      load(k0 + kInvCh, B);
#pragma unroll
      for (int j = 0; j < kInvCh; ++j) step(k0 + j, A.dd[j], A.cn[j]);
      load(k0 + 2 * kInvCh, A);
#pragma unroll
      for (int j = 0; j < kInvCh; ++j) step(k0 + kInvCh + j, B.dd[j], B.cn[j]);
    }
    if (k0 < nb) {
      load(k0 + kInvCh, B);
#pragma unroll
      for (int j = 0; j < kInvCh; ++j)
        if (k0 + j < nb) step(k0 + j, A.dd[j], A.cn[j]);
#pragma unroll
      for (int j = 0; j < kInvCh; ++j)
        if (k0 + kInvCh + j < nb) step(k0 + kInvCh + j, B.dd[j], B.cn[j]);
    }
  }
  __syncthreads();
  // twist index: the first i of least |gamma_i|
  double best = HUGE_VAL;
  int bi = nb;
  for (int i = lane; i < nb; i += 64) {
    const double gm = fabs(piv_f[i] + piv_b[i] - (d[i] - lam));
    if (gm < best) {
      best = gm;
      bi = i;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ob = __shfl_xor(best, off);
    const int oi = __shfl_xor(bi, off);
    if (ob < best || (ob == best && oi < bi)) {
      best = ob;
      bi = oi;
    }
  }
  const int r = bi;                                 // uniform; nb if no finite gamma
  double* z = a.Z + (int64_t)jb.row * a.ldz;
  // the sign makes z's projection on the counter-based random vector
  // rand_pm1(key + i) positive, so that it does not follow the choice of r
  const uint64_t key = (uint64_t)jb.row << 32;
  double ss = 0.0, dot = 0.0;
  if (r < nb) {
    for (int i = lane; i < s; i += 64) z[i] = 0.0;
    for (int i = s + nb + lane; i < a.n; i += 64) z[i] = 0.0;
    if (lane == 0) {
      z[s + r] = 1.0;
      ss = 1.0;
      dot = rand_pm1(key + (uint64_t)r);
    }
    // z_{r-k} = z_{r-k+1} (-e_{r-k} / D+_{r-k}), k = 1..nd (upwards) and
    // z_{r+k} = z_{r+k-1} (-e_{r+k-1} / D-_{r+k}), k = 1..nu (downwards):
    // lane l takes k = k0 + l + 1; inclusive prefix products across the
    // lanes, times the carry (the chunk's last z) of the previous chunk
    const int nd = r, nu = nb - 1 - r;
    const int steps = nd > nu ? nd : nu;
    double cd = 1.0, cu = 1.0;
    // multipliers of the chunk at k0, clamped loads (the next chunk's are in
    // flight while one chunk is scanned; selects at use)
    double fd = mul_f[max(r - lane - 1, 0)], fu = mul_b[min(r + lane + 1, nb - 1)];
    for (int k0 = 0; k0 < steps; k0 += 64) {
      const int k = k0 + lane + 1;
      const double nfd = mul_f[max(r - k - 64, 0)], nfu = mul_b[min(r + k + 64, nb - 1)];
      double md = k <= nd ? -fd : 1.0;
      double mu = k <= nu ? -fu : 1.0;
      fd = nfd;
      fu = nfu;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const double pd = __shfl_up(md, off), pu = __shfl_up(mu, off);
        if (lane >= off) {
          md *= pd;
          mu *= pu;
        }
      }
      const double zd = cd * md, zu = cu * mu;
      if (k <= nd) {
        z[s + r - k] = zd;
        ss += zd * zd;
        dot += zd * rand_pm1(key + (uint64_t)(r - k));
      }
      if (k <= nu) {
        z[s + r + k] = zu;
        ss += zu * zu;
        dot += zu * rand_pm1(key + (uint64_t)(r + k));
      }
      cd = __shfl(zd, 63);
      cu = __shfl(zu, 63);
    }
    for (int off = 32; off > 0; off >>= 1) {
      ss += __shfl_xor(ss, off);
      dot += __shfl_xor(dot, off);
    }
  }
  if (!(ss > 0.0 && ss < 1e300)) {
    if (lane == 0) status[0] = 1.0;
    return;
  }
  __syncthreads();
  const double f = (dot < 0.0 ? -1.0 : 1.0) / sqrt(ss);
  for (int i = lane; i < nb; i += 64) z[s + i] *= f;
  if (lane == 0) status[0] = 0.0;
}

// G (n x n, ld) with its lower triangle computed: the strictly upper part
// <- the transpose of the strictly lower part, and v added on the diagonal.
// One 32 x 32 tile per workgroup of 32 x 8 threads, tiles on or below the
// diagonal only: the lower tile is read through LDS, written transposed.
__global__ void mirror_lower_kernel(double* __restrict__ G, int n, int64_t ld, double v) {
  __shared__ double t[32][33];
  // blockIdx.x enumerates the lower tiles (ti >= tj) row by row
  const int b = blockIdx.x;
  int ti = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= b) ++ti;
  while (ti * (ti + 1) / 2 > b) --ti;
  const int tj = b - ti * (ti + 1) / 2;
  const int r0 = ti * 32, c0 = tj * 32;
  const int tx = threadIdx.x, ty = threadIdx.y;
  for (int y = ty; y < 32; y += 8) {
    const int i = r0 + y, j = c0 + tx;
    t[y][tx] = (i < n && j < n) ? G[(int64_t)i * ld + j] : 0.0;
  }
  __syncthreads();
  // element (c0 + y, r0 + tx) of the upper triangle <- t[tx][y]
  for (int y = ty; y < 32; y += 8) {
    const int i = c0 + y, j = r0 + tx;
    if (i < n && j < n) {
      if (j > i) G[(int64_t)i * ld + j] = t[tx][y];
      else if (j == i) G[(int64_t)i * ld + j] = t[tx][y] + v;
    }
  }
}

// Reflector k of the reduction as an explicit vector in column k of K
// (column-major): zeros above row k + 1, one at row k + 1, the stored part
// below; the whole column zero when tau_k = 0 (the reflector is the identity).
__global__ void explicit_reflectors_kernel(double* __restrict__ V, int n,
                                           const double* __restrict__ tau) {
  const int k = blockIdx.x;
  const bool zero = tau[k] == 0.0;
  double* col = V + (int64_t)k * n;
  const int top = zero ? n : k + 2;
  for (int i = threadIdx.x; i < top; i += blockDim.x)
    col[i] = (i == k + 1 && !zero) ? 1.0 : 0.0;
}

// Block b's T^-1 = diag(1 / tau) + strictly upper part of V_b^T V_b, in
// place over the Gram matrix S_b (row-major nb x nb, w = the block's
// reflector count): zeros below the diagonal, 1 on the diagonal for tau = 0
// (its reflector vector is zero, so the block factor is unaffected), and the
// identity outside the leading w x w part.
__global__ void tinv_kernel(double* __restrict__ S, int nb, int n_refl,
                            const double* __restrict__ tau) {
  const int b = blockIdx.x;
  const int w = min(nb, n_refl - b * nb);
  double* T = S + (int64_t)b * nb * nb;
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
    const int i = e / nb, k = e % nb;
    if (i >= w || k >= w || i > k) {
      T[e] = i == k ? 1.0 : 0.0;
    } else if (i == k) {
      const double t = tau[b * nb + i];
      T[e] = t != 0.0 ? 1.0 / t : 1.0;
    }
  }
}

// The 32 x 32 diagonal blocks of each T^-1 inverted in place (row-major, ld
// nb): one wave per block, lane j computes column j from the bottom row up,
// T[i][j] = -(sum_{i<k<=j} Ti[i][k] T[k][j]) / Ti[i][i].
constexpr int kLeaf = 32;
__global__ __launch_bounds__(64) void inv_leaf_kernel(double* __restrict__ S, int nb) {
  __shared__ double L[kLeaf][kLeaf + 1];
  __shared__ double X[kLeaf][kLeaf + 1];
  const int per = nb / kLeaf;
  const int b = blockIdx.x / per, l = blockIdx.x % per;
  double* base = S + (int64_t)b * nb * nb + (int64_t)l * kLeaf * nb + l * kLeaf;
  const int tid = threadIdx.x;
  for (int e = tid; e < kLeaf * kLeaf; e += 64) L[e / kLeaf][e % kLeaf] = base[(e / kLeaf) * (int64_t)nb + e % kLeaf];
  __syncthreads();
  if (tid < kLeaf) {
    const int j = tid;
    for (int i = kLeaf - 1; i >= 0; --i) {
      double v = 0.0;
      if (i == j) {
        v = 1.0 / L[i][i];
      } else if (i < j) {
        double acc = 0.0;
        for (int k = i + 1; k <= j; ++k) acc += L[i][k] * X[k][j];
        v = -acc / L[i][i];
      }
      X[i][j] = v;
    }
  }
  __syncthreads();
  for (int e = tid; e < kLeaf * kLeaf; e += 64) base[(e / kLeaf) * (int64_t)nb + e % kLeaf] = X[e / kLeaf][e % kLeaf];
}

}  // namespace

namespace gw {

constexpr int kTriBackNb = 256;       // reflectors per compact-WY block
static_assert(kTriBackNb % kLeaf == 0, "block of reflectors: whole leaves");

gw_status dgemm_run(gw_ctx ctx, const std::vector<DGemm>& v, int splits, double* ws) {
  if (v.empty()) return GW_OK;
  const bool ak = v[0].ak, bk = v[0].bk;
  std::vector<G64> descs;
  std::vector<int64_t> off(1, 0);
  std::vector<SumArgs> sums;
  size_t wo = 0;
  const int S = splits > 1 ? splits : 1;
  for (const DGemm& g : v) {
    if (g.ak != ak || g.bk != bk) return fail(ctx, GW_EINVAL, "dgemm_run: mixed layouts in one batch");
    if (g.M <= 0 || g.N <= 0) continue;
    const int tm = (g.M + GBM - 1) / GBM, tnn = (g.N + GBM - 1) / GBM;
    const int kper = ((g.K + S - 1) / S + GBK - 1) / GBK * GBK;
    for (int s = 0; s < S; ++s) {
      const int k0 = std::min(g.K, s * kper), k1 = std::min(g.K, k0 + kper);
      G64 d;
      d.M = g.M;
      d.N = g.N;
      d.K = k1 - k0;
      d.lda = g.lda;
      d.ldb = g.ldb;
      d.A = ak ? g.A + (int64_t)k0 * g.lda : g.A + k0;
      d.B = bk ? g.B + (int64_t)k0 * g.ldb : g.B + k0;
      if (S > 1) {
        d.C = ws + wo + (size_t)s * g.M * g.N;
        d.ldc = g.N;
        d.beta = 0.0;
      } else {
        d.C = g.C;
        d.ldc = g.ldc;
        d.beta = g.beta;
      }
      d.alpha = g.alpha;
      d.tm = tm;
      d.tn = tnn;
      d.splits = 1;
      d.kper = 0;
      d.cstride = 0;
      descs.push_back(d);
      off.push_back(off.back() + (int64_t)tm * tnn);
    }
    if (S > 1) {
      sums.push_back(SumArgs{ws + wo, S, g.M, g.N, g.C, g.ldc, g.beta});
      wo += (size_t)S * g.M * g.N;
    }
  }
  if (descs.empty()) return GW_OK;
  // one product (its K splits included): the descriptor goes by value with
  // the launch, no staging copy; several: a staged descriptor array
  Batch bt{nullptr, nullptr, 0, 1, 0};
  G64 a0 = descs[0];
  const int64_t units = off.back();
  if (descs.size() == (size_t)S) {
    // descs[0] is split 0 of the one product: widen it to the whole K
    const DGemm* one = nullptr;
    for (const DGemm& g : v)
      if (g.M > 0 && g.N > 0) one = &g;
    a0.A = one->A;
    a0.B = one->B;
    a0.K = one->K;
    a0.splits = S;
    a0.kper = ((one->K + S - 1) / S + GBK - 1) / GBK * GBK;
    a0.cstride = (int64_t)one->M * one->N;
  } else {
    GW_TRY(stage_batch(ctx, descs, off, 1, bt));
  }
  const dim3 grid((unsigned)units), block(256);
  if (ak && bk)
    hipLaunchKernelGGL((dgemm_kernel<true, true>), grid, block, 0, ctx->stream, bt, a0);
  else if (!ak && !bk)
    hipLaunchKernelGGL((dgemm_kernel<false, false>), grid, block, 0, ctx->stream, bt, a0);
  else if (!ak && bk)
    hipLaunchKernelGGL((dgemm_kernel<false, true>), grid, block, 0, ctx->stream, bt, a0);
  else
    return fail(ctx, GW_EINVAL, "dgemm_run: layout not built");
  GW_TRY(launch_check(ctx, "dgemm_kernel"));
  for (const SumArgs& sa : sums) {
    hipLaunchKernelGGL(sum_partials_kernel, dim3(grid_for((int64_t)sa.M * sa.N, 256)), dim3(256),
                       0, ctx->stream, sa);
    GW_TRY(launch_check(ctx, "sum_partials_kernel"));
  }
  return GW_OK;
}

constexpr int kBackSplits = 8;        // K splits of the V^T Z products
constexpr int kGramSplits = 8;        // K splits of the Gram matrices V_b^T V_b
constexpr int kOrthSplits = 4;        // K splits of the Newton-Schulz Z Z^T

// Back-transformation workspace at order n for `cols` vectors, in doubles.
static size_t back_ws_elems(int n, int cols) {
  const int nb = kTriBackNb;
  const size_t blocks = n > 1 ? (size_t)(n - 1 + nb - 1) / nb : 0;
  const size_t nb2 = (size_t)nb * nb;
  // T blocks, Gram partials (kGramSplits) or recursion temporaries, T V
  // products, V^T Z partials and their sum
  return blocks * nb2 + (size_t)kGramSplits * blocks * nb2 + blocks * nb * (size_t)n +
         (size_t)(kBackSplits + 1) * nb * cols;
}

// Workspace of naf_tri_solve at order n, in doubles (kept count up to n).
size_t tri_solve_ws_elems(int n) {
  const size_t nn = (size_t)n * n;
  const size_t invit = nn + (size_t)kInvArrays * nn;                 // Z + per-thread arrays
  // Z + G + kOrthSplits partials of G's lower bands (band i: at most GBM rows
  // by GBM (i + 1) columns, so at most (n + GBM)(n + 2 GBM) / 2 per split)
  const size_t orth =
      nn + nn + (size_t)kOrthSplits * (((size_t)n + GBM) * ((size_t)n + 2 * GBM) / 2);
  return (size_t)n + std::max(std::max(invit, orth), back_ws_elems(n, n));
}

// U rows 0 .. cols-1 (eigenvectors of T, ld n) <- Q applied to each:
// Q = H_0 H_1 ... H_{n-2} from the reflectors in K, in blocks of kTriBackNb
// in the compact form H_k0 ... H_k0+w-1 = I - V T V^T, the last block first.
// T is upper triangular with T^-1 = diag(1 / tau) + (strictly upper part of
// V^T V) (appending one reflector at a time to the product gives this
// recurrence); it is inverted by doubling: 32 x 32 diagonal blocks directly,
// then [[A, B], [0, C]]^-1 = [[A', -A' B C'], [0, C']] on FP64 MFMA, the
// products of all blocks batched per level.  With P = T^T V^T (all blocks at
// once, before the sequential part), each block is Z <- Z - (Z V) P.
static gw_status tri_back_own(gw_ctx ctx, double* K, int n, const double* d_tau, double* U,
                              int cols, double* ws) {
  if (n < 2 || cols < 1) return GW_OK;
  const int pt = prof_begin(ctx);
  const int n_refl = n - 1, nb = kTriBackNb;
  const int n_blocks = (n_refl + nb - 1) / nb;
  const size_t nb2 = (size_t)nb * nb;
  double* Tm = ws;                                          // [n_blocks][nb][nb]
  double* tmp = Tm + n_blocks * nb2;                        // [kGramSplits n_blocks][nb][nb]
  double* P = tmp + (size_t)kGramSplits * n_blocks * nb2;   // per block [w][n - r0]
  double* Wp = P + (size_t)n_blocks * nb * n;               // [kBackSplits][nb][cols]
  double* W = Wp + (size_t)kBackSplits * nb * cols;         // [nb][cols]
  hipLaunchKernelGGL(explicit_reflectors_kernel, dim3(n_refl), dim3(256), 0, ctx->stream, K, n,
                     d_tau);
  GW_TRY(launch_check(ctx, "explicit_reflectors_kernel"));
  // Gram matrices V_b^T V_b over the rows below each block's first reflector
  std::vector<DGemm> g;
  for (int b = 0; b < n_blocks; ++b) {
    const int k0 = b * nb, w = std::min(nb, n_refl - k0), r0 = k0 + 1;
    const double* Vb = K + (int64_t)k0 * n + r0;            // row j: reflector k0 + j, ld n
    g.push_back(DGemm{false, false, Vb, Vb, Tm + b * nb2, w, w, n - r0, n, n, nb, 1.0, 0.0});
  }
  GW_TRY(dgemm_run(ctx, g, kGramSplits, tmp));
  hipLaunchKernelGGL(tinv_kernel, dim3(n_blocks), dim3(256), 0, ctx->stream, Tm, nb, n_refl,
                     d_tau);
  GW_TRY(launch_check(ctx, "tinv_kernel"));
  hipLaunchKernelGGL(inv_leaf_kernel, dim3(n_blocks * (nb / kLeaf)), dim3(64), 0, ctx->stream,
                     Tm, nb);
  GW_TRY(launch_check(ctx, "inv_leaf_kernel"));
  for (int h = kLeaf; h < nb; h *= 2) {
    std::vector<DGemm> g1, g2;
    for (int b = 0; b < n_blocks; ++b) {
      double* Tb = Tm + b * nb2;
      for (int p = 0; p < nb / (2 * h); ++p) {
        const int r0 = 2 * h * p;
        double* X = tmp + b * nb2 + (size_t)p * h * h;      // [h][h]
        double* ul = Tb + (int64_t)r0 * nb + r0;
        // X = A' B, then the upper-right block = -X C'
        g1.push_back(DGemm{false, true, ul, ul + h, X, h, h, h, nb, nb, h, 1.0, 0.0});
        g2.push_back(DGemm{false, true, X, ul + (int64_t)h * nb + h, ul + h, h, h, h, h, nb, nb,
                           -1.0, 0.0});
      }
    }
    GW_TRY(dgemm_run(ctx, g1, 1, nullptr));
    GW_TRY(dgemm_run(ctx, g2, 1, nullptr));
  }
  // P_b = T_b^T V_b^T ([w][m], ld m)
  std::vector<double*> Pb(n_blocks);
  g.clear();
  size_t po = 0;
  for (int b = 0; b < n_blocks; ++b) {
    const int k0 = b * nb, w = std::min(nb, n_refl - k0), r0 = k0 + 1, m = n - r0;
    Pb[b] = P + po;
    po += (size_t)w * m;
    g.push_back(DGemm{true, true, Tm + b * nb2, K + (int64_t)k0 * n + r0, Pb[b], w, m, w, nb, n, m,
                      1.0, 0.0});
  }
  GW_TRY(dgemm_run(ctx, g, 1, nullptr));
  for (int b = n_blocks - 1; b >= 0; --b) {
    const int k0 = b * nb, w = std::min(nb, n_refl - k0), r0 = k0 + 1, m = n - r0;
    const double* Vb = K + (int64_t)k0 * n + r0;
    // W = V_b^T Z^T ([w][cols]), then Z <- Z - W^T P_b
    GW_TRY(dgemm_run(ctx, {DGemm{false, false, Vb, U + r0, W, w, cols, m, n, n, cols, 1.0, 0.0}},
                     kBackSplits, Wp));
    GW_TRY(dgemm_run(ctx, {DGemm{true, true, W, Pb[b], U + r0, cols, m, w, cols, m, n, -1.0, 1.0}},
                     1, nullptr));
  }
  // per block 2 w cols m for V^T Z and as much for the update
  double fl = 0.0;
  for (int b = 0; b < n_blocks; ++b) {
    const int k0 = b * nb;
    fl += 4.0 * std::min(nb, n_refl - k0) * (double)cols * (n - k0 - 1);
  }
  prof_end(ctx, pt, "naf_back", fl, 0.0);
  return GW_OK;
}

// The "eigvec" family of gw_autotune_restrict allows code 1 and not code 0:
// every eigenvector by LU inverse iteration.
static bool eigvec_lu_only(gw_ctx ctx) {
  const auto f = ctx->tune_filter.find("eigvec");
  if (f == ctx->tune_filter.end()) return false;
  const int mod = f->second.first, res = f->second.second;
  return 0 % mod != res && 1 % mod == res;
}

// Number of eigenvalues of the block (d, e2 as in sturm_count) below x, on
// the host.
static int sturm_count_host(const double* d, const double* e2, int nb, double x,
                            double pivmin) {
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int c = q < 0.0;
  for (int i = 1; i < nb; ++i) {
    q = (d[i] - x) - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
  }
  return c;
}

// The eigenpairs of T (diagonal d_d, couplings d_e; device, order n) and the
// kept eigenvectors of the original matrix.  K holds the reflectors of the
// reduction (column k below the subdiagonal, tau in d_tau).  On return:
// ev (host [n]) the eigenvalues in descending order, *keep_out the number
// kept (> eps_naf, at most max_keep when > 0), U rows 0 .. keep-1 the kept
// eigenvectors of the original matrix (descending), ld n.  With all_eigs
// false only the eigenvalues above eps_naf (found by a Sturm count at it, one
// below it for margin) are computed, and the rest of ev is -infinity.
// Synchronises.
gw_status naf_tri_solve(gw_ctx ctx, double* K, int n, const double* d_d, const double* d_e,
                        const double* d_tau, double eps_naf, int max_keep, double* U,
                        std::vector<double>& ev, int* keep_out, bool all_eigs) {
  std::vector<double> d(n), e(n > 1 ? n - 1 : 0);
  GW_HIP(ctx, hipMemcpyAsync(d.data(), d_d, n * sizeof(double), hipMemcpyDeviceToHost,
                             ctx->stream));
  if (n > 1)
    GW_HIP(ctx, hipMemcpyAsync(e.data(), d_e, (n - 1) * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream));
  GW_HIP(ctx, hipStreamSynchronize(ctx->stream));
  const double eps = 1.1102230246251565e-16;
  double tnorm = 0.0;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
    tnorm = std::max(tnorm, fabs(d[i]) + r);
  }
  const double tn = std::max(tnorm, 1e-300);
  // unreduced blocks: a coupling negligible next to its diagonal neighbours
  // splits T (it is then taken as zero)
  std::vector<double> e2(std::max(n, 1), 0.0), ez(std::max(n, 1), 0.0);
  std::vector<BisBlock> blocks;
  double emax2 = 0.0;
  int s0 = 0;
  for (int i = 0; i < n; ++i) {
    const bool split = i + 1 == n || fabs(e[i]) <= eps * sqrt(fabs(d[i]) * fabs(d[i + 1])) ||
                       fabs(e[i]) <= eps * eps * tn;
    if (!split) {
      ez[i] = e[i];
      e2[i] = e[i] * e[i];
      emax2 = std::max(emax2, e2[i]);
    } else {
      double gl = d[s0], gu = d[s0];
      for (int k = s0; k <= i; ++k) {
        const double r = (k > s0 ? fabs(ez[k - 1]) : 0.0) + (k < i ? fabs(ez[k]) : 0.0);
        gl = std::min(gl, d[k] - r);
        gu = std::max(gu, d[k] + r);
      }
      const double pad = 4.0 * eps * (i - s0 + 1) * tn;
      blocks.push_back(BisBlock{s0, i - s0 + 1, gl - pad, gu + pad, s0, 0});
      s0 = i + 1;
    }
  }
  const double pivmin = 2.2250738585072014e-308 * std::max(1.0, emax2);
  // the eigenvalues to compute: all, or per block those above eps_naf and
  // one below (a Sturm count in FP64 at eps_naf; the filter below decides)
  int m = n;
  if (!all_eigs) {
    m = 0;
    for (BisBlock& b : blocks) {
      const int c = sturm_count_host(d.data() + b.s, e2.data() + b.s, b.nb, eps_naf, pivmin);
      b.j0 = std::max(0, c - 1);
      b.out = m;
      m += b.nb - b.j0;
    }
  }
  const double* d_e2 = stage_t(ctx, e2.data(), n);
  const double* d_ez = stage_t(ctx, ez.data(), n);
  const BisBlock* d_blocks = stage_t(ctx, blocks.data(), blocks.size());
  if (!d_e2 || !d_ez || !d_blocks) return GW_EINVAL;
  double* ws = static_cast<double*>(ws_get(ctx, WS_EIG_Y, tri_solve_ws_elems(n) * sizeof(double)));
  if (!ws) return GW_ENOMEM;
  double* lam = ws;                                   // [n]
  double* rest = ws + n;
  const int pb = prof_begin(ctx);
  // the number of computed eigenvalues is m, the bisection's "n"
  const BisArgs ba{d_d, d_e2, d_blocks, (int)blocks.size(), m, pivmin, eps * tn, lam, n};
  // points per eigenvalue: about 24k-48k lanes in all (fewer eigenvalues,
  // more points and fewer rounds)
  const int lanes = m <= 2048 ? 32 : (m <= 4096 ? 16 : 8);
  const dim3 bg((unsigned)(((int64_t)lanes * m + 255) / 256));
  const size_t sh = n <= kBisShMax ? 2 * (size_t)n * sizeof(double) : 0;
  if (m > 0) {
    if (sh && lanes == 32)
      hipLaunchKernelGGL((bisect_kernel<true, 32>), bg, dim3(256), sh, ctx->stream, ba);
    else if (sh && lanes == 16)
      hipLaunchKernelGGL((bisect_kernel<true, 16>), bg, dim3(256), sh, ctx->stream, ba);
    else if (sh)
      hipLaunchKernelGGL((bisect_kernel<true, 8>), bg, dim3(256), sh, ctx->stream, ba);
    else if (lanes == 32)
      hipLaunchKernelGGL((bisect_kernel<false, 32>), bg, dim3(256), 0, ctx->stream, ba);
    else if (lanes == 16)
      hipLaunchKernelGGL((bisect_kernel<false, 16>), bg, dim3(256), 0, ctx->stream, ba);
    else
      hipLaunchKernelGGL((bisect_kernel<false, 8>), bg, dim3(256), 0, ctx->stream, ba);
  }
  GW_TRY(launch_check(ctx, "bisect_kernel"));
  prof_end(ctx, pb, "naf_bisect", 0.0, 0.0);
  std::vector<double> lh(std::max(m, 1));
  if (m > 0)
    GW_HIP(ctx, hipMemcpyAsync(lh.data(), lam, m * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream));
  GW_HIP(ctx, hipStreamSynchronize(ctx->stream));
  // descending order over all blocks
  std::vector<int> order(m), blk_of(std::max(m, 1));
  for (size_t b = 0; b < blocks.size(); ++b) {
    const int cnt = all_eigs ? blocks[b].nb : blocks[b].nb - blocks[b].j0;
    for (int j = 0; j < cnt; ++j) blk_of[blocks[b].out + j] = (int)b;
  }
  for (int i = 0; i < m; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return lh[x] > lh[y]; });
  ev.assign(n, -std::numeric_limits<double>::infinity());
  for (int i = 0; i < m; ++i) ev[i] = lh[order[i]];
  int keep = 0;
  while (keep < m && ev[keep] > eps_naf) ++keep;
  if (max_keep > 0) keep = std::min(keep, max_keep);
  *keep_out = keep;
  if (keep == 0) return GW_OK;
  // inverse-iteration jobs: kept eigenvalues by block, ascending; a run of
  // gaps below 1e-10 ||T|| inside a block is one cluster, led by one thread
  std::vector<int> kept(order.begin(), order.begin() + keep);
  std::vector<int> row_of(n, -1);
  for (int p = 0; p < keep; ++p) row_of[kept[p]] = p;
  std::sort(kept.begin(), kept.end());
  std::vector<InvJob> jobs;
  const double cgap = 1e-10 * tn;
  for (size_t i = 0; i < kept.size();) {
    const int b = blk_of[kept[i]];
    size_t j = i + 1;
    while (j < kept.size() && blk_of[kept[j]] == b && lh[kept[j]] - lh[kept[j - 1]] < cgap) ++j;
    for (size_t c = i; c < j; ++c)
      jobs.push_back(InvJob{blocks[b].s, blocks[b].nb, lh[kept[c]], row_of[kept[c]],
                            c == i ? (int)(j - i) : 0});
    i = j;
  }
  const InvJob* d_jobs = stage_t(ctx, jobs.data(), jobs.size());
  if (!d_jobs) return GW_EINVAL;
  double* Z = rest;                                   // [keep][n]
  double* scratch = Z + (size_t)keep * n;             // [keep][kInvArrays][n]
  const int pi = prof_begin(ctx);
  const int nj = (int)jobs.size();
  const bool lu_all = eigvec_lu_only(ctx);
  const InvArgs ia{d_d,  d_ez, d_jobs, nj, n, eps * tn, Z, (int64_t)n, scratch, kInvLanes,
                   lu_all ? 1 : 0};
  if (!lu_all) {
    hipLaunchKernelGGL(twisted_kernel, dim3((unsigned)nj), dim3(64), 0, ctx->stream, ia);
    GW_TRY(launch_check(ctx, "twisted_kernel"));
  }
  hipLaunchKernelGGL(invit_kernel, dim3((unsigned)((nj + kInvLanes - 1) / kInvLanes)), dim3(64),
                     0, ctx->stream, ia);
  GW_TRY(launch_check(ctx, "invit_kernel"));
  prof_end(ctx, pi, "naf_invit", 0.0, 0.0);
  // Newton-Schulz: G = -Z Z^T / 2 + 3 I / 2, U = G Z (G symmetric: TN).
  // Only the tile rows' lower parts of Z Z^T are multiplied (one product per
  // 128-row band, columns up to the band's end), then mirrored.
  double* G = scratch;                                // [keep][keep]
  double* gws = G + (size_t)keep * keep;              // split-K partials of G
  const int pn = prof_begin(ctx);
  std::vector<DGemm> gl;
  for (int i0 = 0; i0 < keep; i0 += GBM)
    gl.push_back(DGemm{false, false, Z + (int64_t)i0 * n, Z, G + (int64_t)i0 * keep,
                       std::min(GBM, keep - i0), std::min(keep, i0 + GBM), n, n, n, keep, -0.5,
                       0.0});
  GW_TRY(dgemm_run(ctx, gl, kOrthSplits, gws));
  {
    const int nt = (keep + 31) / 32;
    hipLaunchKernelGGL(mirror_lower_kernel, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(32, 8), 0,
                       ctx->stream, G, keep, (int64_t)keep, 1.5);
    GW_TRY(launch_check(ctx, "mirror_lower_kernel"));
  }
  GW_TRY(dgemm_run(ctx, {DGemm{true, true, G, Z, U, keep, n, keep, keep, n, n, 1.0, 0.0}}, 1,
                   nullptr));
  // Z Z^T counted once (symmetric) and G Z
  prof_end(ctx, pn, "naf_orth", 3.0 * (double)keep * keep * n, 0.0);
  return tri_back_own(ctx, K, n, d_tau, U, keep, rest);
}

}  // namespace gw
