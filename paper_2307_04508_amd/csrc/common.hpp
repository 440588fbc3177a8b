// Internal declarations shared by the gwlt library sources (not part of the
// public ABI).  Context, workspace, error reporting and small device helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "gwlt.h"

// Workspace slots owned by a context.  Each slot is a device buffer grown on
// demand; growing waits for the stream first.
enum WsSlot {
  WS_STAGE = 0,     // device side of the host->device staging ring
  WS_SYRK_PART,     // split-K partial tiles of the SYRK kernels
  WS_SYRK_SCALE,    // per-row Laplace scale factors
  WS_SCREEN_A,      // FP64 working matrices of the screening sweep
  WS_SCREEN_PANEL,  // pivot column panels, scaled panels, pivot inverses
  WS_SIGMA_PART,    // per-column-block row-dot partials of W_nm
  WS_SIGMA_W,       // W_nm [F][Q*M] FP64
  WS_SIGMA_RT,      // FP32 k-major copy of the QP rows of R~ for the contraction
  WS_EIG,           // eigensolver scratch (eigenvalues, off-diagonal, info)
  WS_QP,            // Pade / QP outputs
  WS_G_RT_OV,       // whole-step driver: NAF-transformed ov tensor
  WS_G_RT_QP,       // whole-step driver: NAF-transformed QP rows
  WS_G_K,           // whole-step driver: NAF metric
  WS_G_U,           // whole-step driver: NAF basis
  WS_G_M,           // whole-step driver: Laplace matrices M^m
  WS_G_WHAT,        // whole-step driver: screened interaction
  WS_G_SIGMA,       // whole-step driver: Sigma(i w) on the Pade nodes
  WS_B_RT_OV,       // batched driver: NAF-transformed ov tensors
  WS_B_RT_QP,       // batched driver: NAF-transformed QP rows
  WS_B_K,           // batched driver: padded NAF metrics
  WS_B_U,           // batched driver: NAF bases
  WS_B_M,           // batched driver: Laplace matrices
  WS_B_WHAT,        // batched driver: screened interactions
  WS_B_SIGMA,       // batched driver: Sigma(i w) and QP outputs
  WS_B_EIG,         // batched driver: eigenvalues, off-diagonals, info
  WS_TRI,           // tridiagonalisation exchange buffers and barrier counters
  WS_EIG_Y,         // eigenvectors of the tridiagonal matrix
  WS_NAF_T,         // k-major FP32 copies of the NAF transform's operands
  WS_B3_CHI,        // BF16x3 polarizability: split scaled rows (hi, lo) of a chunk
  WS_B3_R,          // BF16x3 contraction: split QP rows (hi, lo)
  WS_B3_W,          // BF16x3 contraction: split screened interactions (hi, lo)
  WS_TRI_SUB,       // HBM reduction: exchange buffers of its on-chip trailing part
  WS_TRI_COPY,      // HBM reduction: contiguous copy of the trailing block
  WS_COUNT
};

constexpr size_t kStageBytes = size_t(4) << 20;   // staging ring size
constexpr size_t kArenaBytes = size_t(32) << 20;  // per-graph copy of staged arrays

struct BatchGraph;

// One bracketed launch recorded while kernel timing is enabled.
struct ProfEvent {
  std::string name;
  hipEvent_t a = nullptr, b = nullptr;
  double flops = 0, bytes = 0;
};
struct ProfStat {
  double ms = 0, flops = 0, bytes = 0;
  int64_t launches = 0;
};

struct gw_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  void* ws[WS_COUNT] = {};
  size_t ws_bytes[WS_COUNT] = {};
  // host->device staging ring for small host arrays passed by value
  unsigned char* stage_host = nullptr;   // pinned
  size_t stage_off = 0;
  // device flags for deferred errors: [0] screening non-SPD (freq index + 1)
  int* d_flags = nullptr;
  // kernel timing (gw_profile_enable)
  bool prof = false;
  std::vector<ProfEvent> prof_pending;
  std::map<std::string, ProfStat> prof_stats;
  // graph capture (gw_graph_begin / gw_graph_end): while capturing, host
  // arrays are staged into a per-graph device arena instead of the ring, so
  // replays read what the captured calls were given
  bool capturing = false;
  hipStream_t user_stream = nullptr;     // restored when the capture ends
  hipStream_t capture_stream = nullptr;  // private, created lazily
  // second stream of the screening sweep's lookahead (forked from and
  // joined back into `stream` by events), created lazily
  hipStream_t side_stream = nullptr;
  hipEvent_t side_ev[2] = {nullptr, nullptr};
  unsigned char* arena_dev = nullptr;
  std::vector<unsigned char> arena_host;
  int live_graphs = 0;                   // caller-held graphs (workspace pinned)
  BatchGraph* batch_graph = nullptr;     // gw_g0w0_batched's cached graph
  // launch-shape autotuner (gw_autotune): chosen candidate per shape key
  bool autotune = true;
  std::map<std::string, int> tuned;
  // gw_autotune_restrict: family -> (modulus, residue) filter on candidates
  std::map<std::string, std::pair<int, int>> tune_filter;
};

// A captured, instantiated graph and the arena its kernels read.
struct gw_graph_s {
  gw_ctx ctx = nullptr;
  hipGraphExec_t exec = nullptr;
  void* arena = nullptr;
};

namespace gw {

gw_status fail(gw_ctx ctx, gw_status st, const char* fmt, ...);
void clear_error(gw_ctx ctx);
gw_status hip_check(gw_ctx ctx, hipError_t e, const char* what);
// Device buffer of at least `bytes` for `slot` (nullptr on failure; ctx->err set).
void* ws_get(gw_ctx ctx, WsSlot slot, size_t bytes);
// Copy a small host array into the staging ring; returns its device address.
const void* stage(gw_ctx ctx, const void* host, size_t bytes);
template <typename T>
inline const T* stage_t(gw_ctx ctx, const T* host, size_t n) {
  return static_cast<const T*>(stage(ctx, host, n * sizeof(T)));
}
// Launch-shape autotuner: the first time `key` is seen (tuning on, not
// capturing), time trial(c) for every candidate with HIP events on the
// context's stream and keep the fastest; later calls (and capture, or tuning
// off: the first candidate) return the kept choice without trials.  trial
// must be free of side effects beyond scratch, or idempotent.  The family of
// a key is its text before the first ':'; a restriction set for the family
// keeps only the candidates c with c % modulus == residue (all of them when
// none matches).
int tune(gw_ctx ctx, const std::string& key, const std::vector<int>& cand,
         const std::function<gw_status(int)>& trial);
// Begin / end a capture on the context (used by the public graph calls and
// the batched driver).  end_capture instantiates the graph into *out.
gw_status begin_capture(gw_ctx ctx);
gw_status end_capture(gw_ctx ctx, gw_graph_s* out);
void drop_batch_graph(gw_ctx ctx);
// Read and clear the deferred device error flags (synchronises).
gw_status check_flags(gw_ctx ctx);
gw_status launch_check(gw_ctx ctx, const char* what);

// Kernel timing: prof_begin records a start event on the context's stream
// (returns -1 when timing is off); prof_end records the end event and the
// algorithmic flops / bytes of the bracketed work under `name`.
int prof_begin(gw_ctx ctx);
void prof_end(gw_ctx ctx, int idx, const char* name, double flops, double bytes);

// ---- launchers implemented in the kernel sources ----
// Scaled SYRK: C[m] (+)= X^T diag(s_m) X over rows of X, lower triangle.
// scale: [L][k_rows] per-row factors of the element type, or nullptr for a
// constant factor `cscale`.  out: [L][N][N] FP64.
gw_status syrk_launch(gw_ctx ctx, gw_precision prec, const void* X,
                      int64_t k_rows, int N, int64_t ld, int L,
                      const void* scale, double cscale, double* out,
                      int accumulate, const char* prof_name);
gw_status mirror_lower(gw_ctx ctx, double* M, int L, int N);

// Batched forms: one launch over the work of several problems.
struct SyrkJob {
  const void* X;        // [k_rows][ld]
  int64_t k_rows;
  int N;
  int64_t ld;
  int L;
  const void* scale;    // [L][k_rows] or nullptr
  double cscale;
  double* out;          // [L][N][N] FP64, lower triangle
  int accumulate;
};
struct ScaleJob {
  int L;
  const double* x;      // device [L]
  const double* w;      // device [L]
  int n_i, n_virt;
  const double* eps_i;  // device [n_i]
  const double* eps_a;  // device [n_virt]
  void* out;            // device [L][n_i * n_virt]
};
struct MirrorJob {
  double* M;
  int L, N;
};
gw_status syrk_batched_launch(gw_ctx ctx, gw_precision prec, const std::vector<SyrkJob>& jobs,
                              const char* prof_name);
gw_status lt_scale_batched(gw_ctx ctx, gw_precision prec, const std::vector<ScaleJob>& jobs);
gw_status mirror_lower_batched(gw_ctx ctx, const std::vector<MirrorJob>& jobs);
// Pade + QP for several jobs (device arrays), outputs [3 * state] on the device.
struct QpJob {
  int n_qp, n_pade;
  const double* omega_pade;
  const double* sigma_iw;
  const double* eps_n;
  const double* static_n;
  double eps_F;
};
gw_status qp_batched_launch(gw_ctx ctx, const std::vector<QpJob>& jobs, double eta, double tol,
                            int max_iter, double* out);
// Batched NAF pieces (naf.hip).
struct NafEigJob {
  const double* K;      // device [A][A] metric, lower triangle
  int A;
  double* U;            // device [A][A]: eigenvectors as rows, descending (may alias K)
  double* eig;          // host [A]: eigenvalues, descending
  double eps_naf;       // eigenvectors needed: eigenvalue > eps_naf,
  int max_keep;         // at most max_keep of them when > 0
  bool all_eigs = true; // false: eigenvalues below eps_naf need not be computed
                        // (eig then holds -infinity past the computed ones)
};
gw_status naf_eig_batched(gw_ctx ctx, const std::vector<NafEigJob>& jobs);
// FP32 transposes dst[c][r] = src[r][c] (c < cols, r < rows; rows up to
// ld_dst - 1 are zero-filled), all jobs in one launch.
struct TransposeJob {
  const float* src;     // [rows][ld_src]
  int64_t rows, ld_src;
  int cols;
  float* dst;           // [cols][ld_dst]
  int64_t ld_dst;
};
gw_status transpose_f32(gw_ctx ctx, const std::vector<TransposeJob>& jobs);
// Householder tridiagonalisation (LAPACK dsytrd form, lower) of symmetric
// matrices held whole on chip by a cooperative launch; see tridiag.hip.
struct TriIn {
  double* K;            // device [n][n] symmetric; out: reflectors (column-major)
  int n;
  double* d;            // device [n]
  double* e;            // device [n - 1]
  double* tau;          // device [n - 1]
};
// Largest order the on-chip reduction takes on this context's device.
int tridiag_max_order(gw_ctx ctx);
// Householder reduction to tridiagonal form (same outputs as tridiag_jobs)
// of one matrix of any order, held in HBM: panels of columns, each one
// cooperative launch, and a rank-2·panel trailing update on FP64 MFMA, until
// the trailing block fits the on-chip reduction, which finishes it.
// Asynchronous; a barrier timeout raises ctx->d_flags[1].
gw_status tridiag_blocked(gw_ctx ctx, const TriIn& job);
// C (+)= alpha op(A) op(B) in FP64 on MFMA (eig.hip): ak, A stored [k][m]
// (else [m][k]); bk, B stored [k][n] (else [n][k]); all row-major.  With
// splits > 1 the K range is cut into `splits` pieces whose products go to
// ws ([S][M][N] per product, in order) and are summed in a fixed order into
// C.  The products of one call share the layout and launch together, so
// they must write disjoint C.
struct DGemm {
  bool ak, bk;
  const double* A;
  const double* B;
  double* C;
  int M, N, K;
  int64_t lda, ldb, ldc;
  double alpha, beta;
};
gw_status dgemm_run(gw_ctx ctx, const std::vector<DGemm>& v, int splits, double* ws);
// Workspace (WS_EIG_Y, doubles) of naf_tri_solve at order n.
size_t tri_solve_ws_elems(int n);
gw_status tridiag_jobs(gw_ctx ctx, const std::vector<TriIn>& jobs, WsSlot slot = WS_TRI);
struct NafGemmJob {
  const void* A;        // [rows][K]
  const double* U;      // [>= ncols][K]
  void* C;              // [rows][ldc]
  int64_t rows;
  int K, ncols;
  int64_t ldc;
};
gw_status naf_gemm_batched(gw_ctx ctx, gw_precision prec, const std::vector<NafGemmJob>& jobs);
// Workspace each call needs at given sizes (gw_reserve).
size_t syrk_part_bytes(gw_precision prec, int64_t k_rows, int N, int L);
void screen_ws_bytes(gw_precision prec, int N, int F, size_t* a_bytes, size_t* panel_bytes);
void sigma_ws_bytes(int N, int64_t rows, int F, size_t* part_bytes, size_t* w_bytes,
                    size_t* rt_bytes);
// Zero n doubles with a kernel (capturable, unlike hipMemsetAsync).
gw_status fill_zero(gw_ctx ctx, double* p, int64_t n);
// Device address of the fixed scratch of gw_sigma_diag_noalloc on `device`
// (which must be current); called once per device at context creation.
gw_status sigma_scratch_init(gw_ctx ctx, int device);
gw_status lt_scale_launch(gw_ctx ctx, gw_precision prec, int L,
                          const double* d_x, const double* d_w, int n_i,
                          int n_virt, const double* d_eps_i,
                          const double* d_eps_a, void* scale,
                          int sos);

}  // namespace gw

#define GW_REQUIRE(ctx, cond, ...)                                  \
  do {                                                              \
    if (!(cond)) return gw::fail((ctx), GW_EINVAL, __VA_ARGS__);    \
  } while (0)

#define GW_HIP(ctx, call)                                           \
  do {                                                              \
    gw_status _s = gw::hip_check((ctx), (call), #call);             \
    if (_s != GW_OK) return _s;                                     \
  } while (0)

#define GW_TRY(expr)                                                \
  do {                                                              \
    gw_status _s = (expr);                                          \
    if (_s != GW_OK) return _s;                                     \
  } while (0)

// ---------------------------------------------------------------- device side
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// DPP move of a double (both 32-bit halves) inside the wave's rows of 16
// lanes, or a row broadcast; lanes of rows outside ROW_MASK receive 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xF, false);
  return __hiloint2double(hi, lo);
}
// Sums over each half wave, complete in lane 31 (lanes 0-31) and lane 63
// (lanes 32-63): quad sums, half-row and row mirrors, then the last lane of
// rows 0 and 2 broadcast into rows 1 and 3.  VALU only (a shuffle tree
// would take an LDS permute per step).
// Sums over each row of 16 lanes, in every lane of the row.
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_move<0xB1, 0xF>(v);     // quad_perm [1,0,3,2]
  v += dpp_move<0x4E, 0xF>(v);     // quad_perm [2,3,0,1]
  v += dpp_move<0x141, 0xF>(v);    // row_half_mirror
  v += dpp_move<0x140, 0xF>(v);    // row_mirror
  return v;
}
__device__ __forceinline__ double half_wave_sum(double v) {
  v = row16_sum(v);
  v += dpp_move<0x142, 0xA>(v);    // row_bcast:15 into rows 1 and 3
  return v;
}

// Map a hardware workgroup index to a logical one so that workgroups placed
// on the same XCD (dispatched round-robin over the 8 XCDs) receive
// consecutive logical indices and share data through that XCD's L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t G) {
  const int64_t x = b & 7, slot = b >> 3;
  const int64_t g8 = G >> 3, rem = G & 7;
  return x * g8 + (x < rem ? x : rem) + slot;
}

// Batched launches put the work units of several problems in one grid:
// problem d owns the logical units [off[d], off[d+1]) and its arguments are
// descs[d].  Workgroups map to units in chunks of `chunk` consecutive units
// per XCD, the chunks dealt round-robin over the 8 XCDs, so every XCD gets a
// share of every problem while units that share data stay on one XCD.  The
// grid is padded to a multiple of 8 * chunk; surplus workgroups exit.
struct Batch {
  const void* descs;      // device array of per-problem argument structs
  const int64_t* off;     // device [n + 1] unit offsets
  int n;
  int chunk;
  int64_t units;          // off[n]
};

__device__ __forceinline__ int64_t xcd_chunk_remap(int64_t b, int chunk) {
  const int64_t x = b & 7, s = b >> 3;
  return ((s / chunk) * 8 + x) * chunk + s % chunk;
}

__device__ __forceinline__ int find_problem(const int64_t* __restrict__ off, int n, int64_t u) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= u) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// The logical unit of this workgroup and its problem's arguments: a single
// problem (bt.descs == nullptr) uses a0 and the XCD remap of the whole grid.
template <typename Args>
__device__ __forceinline__ bool unit_of(const Args& a0, const Batch& bt, Args& a, int64_t& lid) {
  if (!bt.descs) {
    a = a0;
    lid = xcd_remap(blockIdx.x, gridDim.x);
    return true;
  }
  const int64_t u = xcd_chunk_remap(blockIdx.x, bt.chunk);
  if (u >= bt.units) return false;
  const int d = find_problem(bt.off, bt.n, u);
  a = static_cast<const Args*>(bt.descs)[d];
  lid = u - bt.off[d];
  return true;
}

// Same for element-wise kernels: a batched problem owns whole blocks of
// kBatchElems elements, one 256-thread workgroup each (4 elements per
// thread, strided by 256); returns the first element index of the block.
constexpr int kBatchElems = 1024;
template <typename Args>
__device__ __forceinline__ bool block_of(const Batch& bt, Args& a, int64_t& first) {
  const int64_t u = blockIdx.x;
  if (u >= bt.units) return false;
  const int d = find_problem(bt.off, bt.n, u);
  a = static_cast<const Args*>(bt.descs)[d];
  first = (u - bt.off[d]) * kBatchElems;
  return true;
}

// ---------------------------------------------------------- batched launches
namespace gw {

// Stage a descriptor table and its unit offsets; returns the Batch.
template <typename Args>
inline gw_status stage_batch(gw_ctx ctx, const std::vector<Args>& d,
                             const std::vector<int64_t>& off, int chunk, Batch& bt) {
  const Args* dd = static_cast<const Args*>(stage(ctx, d.data(), d.size() * sizeof(Args)));
  const int64_t* doff = static_cast<const int64_t*>(stage(ctx, off.data(), off.size() * sizeof(int64_t)));
  if (!dd || !doff) return GW_EINVAL;
  bt = Batch{dd, doff, (int)d.size(), chunk, off.back()};
  return GW_OK;
}

template <typename Args>
inline gw_status elementwise_batched(gw_ctx ctx, const std::vector<Args>& d,
                                     const std::vector<int64_t>& n_elems, void (*kern)(Batch),
                                     const char* what) {
  std::vector<int64_t> off(1, 0);
  for (int64_t n : n_elems) off.push_back(off.back() + (n + kBatchElems - 1) / kBatchElems);
  if (off.back() == 0) return GW_OK;
  Batch bt;
  GW_TRY(stage_batch(ctx, d, off, 1, bt));
  hipLaunchKernelGGL(kern, dim3((unsigned)off.back()), dim3(256), 0, ctx->stream, bt);
  return launch_check(ctx, what);
}

}  // namespace gw
