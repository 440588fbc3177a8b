// Internal declarations shared by the gwlt library sources (not part of the
// public ABI).  Context, workspace, error reporting and small device helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
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
  WS_EIG,           // eigensolver scratch (eigenvalues, off-diagonal, info)
  WS_QP,            // Pade / QP outputs
  WS_G_RT_OV,       // whole-step driver: NAF-transformed ov tensor
  WS_G_RT_QP,       // whole-step driver: NAF-transformed QP rows
  WS_G_K,           // whole-step driver: NAF metric
  WS_G_U,           // whole-step driver: NAF basis
  WS_G_M,           // whole-step driver: Laplace matrices M^m
  WS_G_WHAT,        // whole-step driver: screened interaction
  WS_G_SIGMA,       // whole-step driver: Sigma(i w) on the Pade nodes
  WS_COUNT
};

constexpr size_t kStageBytes = size_t(4) << 20;   // staging ring size

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
  void* rocblas = nullptr;               // rocblas_handle, created lazily
  // kernel timing (gw_profile_enable)
  bool prof = false;
  std::vector<ProfEvent> prof_pending;
  std::map<std::string, ProfStat> prof_stats;
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
gw_status lt_scale_launch(gw_ctx ctx, gw_precision prec, int L,
                          const double* d_x, const double* d_w, int n_i,
                          int n_virt, const double* d_eps_i,
                          const double* d_eps_a, void* scale);

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

// Map a hardware workgroup index to a logical one so that workgroups placed
// on the same XCD (dispatched round-robin over the 8 XCDs) receive
// consecutive logical indices and share data through that XCD's L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t G) {
  const int64_t x = b & 7, slot = b >> 3;
  const int64_t g8 = G >> 3, rem = G & 7;
  return x * g8 + (x < rem ? x : rem) + slot;
}
