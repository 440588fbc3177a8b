// Context lifetime, workspace, staging and error reporting.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <fstream>
#include <sstream>

#include "common.hpp"

static thread_local std::string g_free_err;   // errors of context-free calls

namespace gw {

gw_status fail(gw_ctx ctx, gw_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf; else g_free_err = buf;
  return st;
}

void clear_error(gw_ctx ctx) {
  if (ctx) ctx->err.clear(); else g_free_err.clear();
}

gw_status hip_check(gw_ctx ctx, hipError_t e, const char* what) {
  if (e == hipSuccess) return GW_OK;
  return fail(ctx, e == hipErrorOutOfMemory ? GW_ENOMEM : GW_EDEVICE,
              "%s: %s", what, hipGetErrorString(e));
}

gw_status launch_check(gw_ctx ctx, const char* what) {
  return hip_check(ctx, hipGetLastError(), what);
}

void* ws_get(gw_ctx ctx, WsSlot slot, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (ctx->ws_bytes[slot] >= bytes) return ctx->ws[slot];
  if (ctx->capturing) {
    fail(ctx, GW_EUNSUPPORTED,
         "workspace would grow during graph capture; run the calls once eagerly "
         "(or gw_reserve) before capturing them");
    return nullptr;
  }
  if (ctx->live_graphs > 0) {
    fail(ctx, GW_EUNSUPPORTED,
         "workspace would grow while a captured graph references it; destroy the graph first");
    return nullptr;
  }
  drop_batch_graph(ctx);   // the cached batched graph references the old buffers
  if (ctx->ws[slot]) {
    if (hipStreamSynchronize(ctx->stream) != hipSuccess ||
        hipFree(ctx->ws[slot]) != hipSuccess) {
      fail(ctx, GW_EDEVICE, "workspace release failed");
      ctx->ws[slot] = nullptr;
      ctx->ws_bytes[slot] = 0;
      return nullptr;
    }
    ctx->ws[slot] = nullptr;
    ctx->ws_bytes[slot] = 0;
  }
  size_t want = (bytes + 4095) & ~size_t(4095);
  void* p = nullptr;
  if (hipMalloc(&p, want) != hipSuccess) {
    (void)hipGetLastError();
    fail(ctx, GW_ENOMEM, "workspace allocation of %zu bytes failed", want);
    return nullptr;
  }
  ctx->ws[slot] = p;
  ctx->ws_bytes[slot] = want;
  return p;
}

const void* stage(gw_ctx ctx, const void* host, size_t bytes) {
  size_t need = (bytes + 255) & ~size_t(255);
  if (ctx->capturing) {
    const size_t off = ctx->arena_host.size();
    if (off + need > kArenaBytes) {
      fail(ctx, GW_ENOMEM, "graph capture arena exhausted (%zu bytes)", kArenaBytes);
      return nullptr;
    }
    ctx->arena_host.resize(off + need);
    std::memcpy(ctx->arena_host.data() + off, host, bytes);
    return ctx->arena_dev + off;
  }
  if (need > kStageBytes) {
    fail(ctx, GW_EINVAL, "host array of %zu bytes exceeds the staging ring", bytes);
    return nullptr;
  }
  if (ctx->stage_off + need > kStageBytes) {
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
      fail(ctx, GW_EDEVICE, "stream synchronisation failed");
      return nullptr;
    }
    ctx->stage_off = 0;
  }
  unsigned char* dev = static_cast<unsigned char*>(ctx->ws[WS_STAGE]);
  std::memcpy(ctx->stage_host + ctx->stage_off, host, bytes);
  if (hipMemcpyAsync(dev + ctx->stage_off, ctx->stage_host + ctx->stage_off,
                     bytes, hipMemcpyHostToDevice, ctx->stream) != hipSuccess) {
    fail(ctx, GW_EDEVICE, "staging copy failed");
    return nullptr;
  }
  const void* out = dev + ctx->stage_off;
  ctx->stage_off += need;
  return out;
}

gw_status check_flags(gw_ctx ctx) {
  int h[4] = {0, 0, 0, 0};
  GW_HIP(ctx, hipMemcpyAsync(h, ctx->d_flags, sizeof h, hipMemcpyDeviceToHost, ctx->stream));
  GW_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (h[0] != 0) {
    GW_HIP(ctx, hipMemsetAsync(ctx->d_flags, 0, sizeof h, ctx->stream));
    GW_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return fail(ctx, GW_ENOTSPD,
                "1 - Pi is not positive definite at frequency index %d", h[0] - 1);
  }
  return GW_OK;
}

int prof_begin(gw_ctx ctx) {
  if (!ctx->prof || ctx->capturing) return -1;
  ProfEvent e;
  if (hipEventCreate(&e.a) != hipSuccess || hipEventCreate(&e.b) != hipSuccess) return -1;
  hipEventRecord(e.a, ctx->stream);
  ctx->prof_pending.push_back(e);
  return (int)ctx->prof_pending.size() - 1;
}

void prof_end(gw_ctx ctx, int idx, const char* name, double flops, double bytes) {
  if (idx < 0 || idx >= (int)ctx->prof_pending.size()) return;
  ProfEvent& e = ctx->prof_pending[idx];
  e.name = name;
  e.flops = flops;
  e.bytes = bytes;
  hipEventRecord(e.b, ctx->stream);
}

static void prof_resolve(gw_ctx ctx) {
  for (ProfEvent& e : ctx->prof_pending) {
    float ms = 0.f;
    if (!e.name.empty() && hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
      ProfStat& s = ctx->prof_stats[e.name];
      s.ms += ms;
      s.flops += e.flops;
      s.bytes += e.bytes;
      s.launches += 1;
    }
    hipEventDestroy(e.a);
    hipEventDestroy(e.b);
  }
  ctx->prof_pending.clear();
}

int tune(gw_ctx ctx, const std::string& key, const std::vector<int>& all,
         const std::function<gw_status(int)>& trial) {
  std::vector<int> cand = all;
  auto f = ctx->tune_filter.find(key.substr(0, key.find(':')));
  if (f != ctx->tune_filter.end()) {
    std::vector<int> kept;
    for (int c : all)
      if (c % f->second.first == f->second.second) kept.push_back(c);
    if (!kept.empty()) cand = kept;
  }
  auto it = ctx->tuned.find(key);
  if (it != ctx->tuned.end() && std::find(cand.begin(), cand.end(), it->second) != cand.end())
    return it->second;
  if (!ctx->autotune || ctx->capturing || cand.size() < 2) return cand.empty() ? 0 : cand[0];
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    if (a) hipEventDestroy(a);
    return cand[0];
  }
  int best = cand[0];
  float best_ms = 1e30f;
  for (int c : cand) {
    for (int rep = 0; rep < 2; ++rep) {   // the first run warms caches and workspace
      hipEventRecord(a, ctx->stream);
      const gw_status st = trial(c);
      hipEventRecord(b, ctx->stream);
      float ms = 0.f;
      if (st != GW_OK || hipEventSynchronize(b) != hipSuccess ||
          hipEventElapsedTime(&ms, a, b) != hipSuccess)
        break;
      if (rep == 1 && ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  (void)hipGetLastError();
  clear_error(ctx);
  ctx->tuned[key] = best;
  return best;
}

gw_status begin_capture(gw_ctx ctx) {
  if (ctx->capturing) return fail(ctx, GW_EINVAL, "a graph capture is already in progress");
  GW_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (!ctx->capture_stream)
    GW_HIP(ctx, hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
  void* arena = nullptr;
  if (hipMalloc(&arena, kArenaBytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, GW_ENOMEM, "graph arena allocation failed");
  }
  ctx->arena_dev = static_cast<unsigned char*>(arena);
  ctx->arena_host.clear();
  ctx->user_stream = ctx->stream;
  ctx->stream = ctx->capture_stream;
  if (hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
    ctx->stream = ctx->user_stream;
    hipFree(arena);
    ctx->arena_dev = nullptr;
    return fail(ctx, GW_EDEVICE, "hipStreamBeginCapture failed");
  }
  ctx->capturing = true;
  return GW_OK;
}

gw_status end_capture(gw_ctx ctx, gw_graph_s* out) {
  if (!ctx->capturing) return fail(ctx, GW_EINVAL, "no graph capture in progress");
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(ctx->stream, &graph);
  ctx->stream = ctx->user_stream;
  ctx->capturing = false;
  hipGraphExec_t exec = nullptr;
  hipError_t ei = hipErrorUnknown;
  if (e == hipSuccess && graph) {
    ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
  }
  hipError_t ec = hipSuccess;
  if (ei == hipSuccess && !ctx->arena_host.empty())
    ec = hipMemcpy(ctx->arena_dev, ctx->arena_host.data(), ctx->arena_host.size(),
                   hipMemcpyHostToDevice);
  if (e != hipSuccess || ei != hipSuccess || ec != hipSuccess) {
    if (exec) hipGraphExecDestroy(exec);
    hipFree(ctx->arena_dev);
    ctx->arena_dev = nullptr;
    (void)hipGetLastError();
    return fail(ctx, GW_EDEVICE, "graph capture failed (%s)",
                hipGetErrorString(e != hipSuccess ? e : (ei != hipSuccess ? ei : ec)));
  }
  out->ctx = ctx;
  out->exec = exec;
  out->arena = ctx->arena_dev;
  ctx->arena_dev = nullptr;
  ctx->arena_host.clear();
  return GW_OK;
}

}  // namespace gw

extern "C" {

gw_status gw_reserve(gw_ctx ctx, gw_precision prec, const gw_dims* d) {
  if (!ctx || !d) return gw::fail(ctx, GW_EINVAL, "gw_reserve: NULL argument");
  gw::clear_error(ctx);
  if (ctx->capturing) return gw::fail(ctx, GW_EUNSUPPORTED, "gw_reserve inside a graph capture");
  GW_REQUIRE(ctx, prec == GW_FP64 || prec == GW_FP32 || prec == GW_BF16X3,
             "gw_reserve: unknown precision %d", (int)prec);
  GW_REQUIRE(ctx, d->n_aux >= 0 && d->n_naf >= 0 && d->n_occ_act >= 0 && d->n_virt >= 0 &&
                      d->n_mo >= 0 && d->n_qp >= 0 && d->n_lt >= 0 && d->n_w >= 0 &&
                      d->n_pade >= 0 && d->chunk_i >= 0,
             "gw_reserve: negative size");
  GW_HIP(ctx, hipSetDevice(ctx->device));
  const int ci = d->chunk_i > 0 ? std::min(d->chunk_i, d->n_occ_act) : d->n_occ_act;
  const int64_t k_chi = (int64_t)ci * d->n_virt;
  const int64_t k_oo = (int64_t)ci * d->n_occ_act;
  const gw_precision mp = prec == GW_FP64 ? GW_FP64 : GW_FP32;
  const size_t esz = prec == GW_FP64 ? 8 : 4;
  size_t part = 0;
  if (d->n_naf > 0 && d->n_lt > 0) part = gw::syrk_part_bytes(prec, k_chi, d->n_naf, d->n_lt);
  if (d->n_aux > 0) {
    part = std::max(part, gw::syrk_part_bytes(mp, k_chi, d->n_aux, 1));
    part = std::max(part, gw::syrk_part_bytes(mp, k_oo, d->n_aux, 1));
  }
  size_t sa = 0, sp = 0, gp = 0, gwb = 0, grt = 0;
  if (d->n_naf > 0 && d->n_w > 0) {
    gw::screen_ws_bytes(prec, d->n_naf, d->n_w, &sa, &sp);
    gw::sigma_ws_bytes(d->n_naf, (int64_t)d->n_qp * d->n_mo, d->n_w, &gp, &gwb, &grt);
    if (prec != GW_FP32) grt = 0;
  }
  const struct { WsSlot slot; size_t bytes; } want[] = {
      {WS_SYRK_PART, part},
      {WS_SYRK_SCALE, (size_t)d->n_lt * k_chi * esz},
      {WS_SCREEN_A, sa},
      {WS_SCREEN_PANEL, sp},
      {WS_SIGMA_PART, gp},
      {WS_SIGMA_W, gwb},
      {WS_SIGMA_RT, grt},
      {WS_EIG, (3 * (size_t)d->n_aux + 8) * sizeof(double)},
      {WS_EIG_Y, d->n_aux <= gw::tridiag_max_order(ctx)
                     ? gw::tri_solve_ws_elems(d->n_aux) * sizeof(double) : 0},
      {WS_QP, 3 * (size_t)d->n_qp * sizeof(double)},
  };
  for (const auto& w : want)
    if (w.bytes > 0 && !gw::ws_get(ctx, w.slot, w.bytes)) return GW_ENOMEM;
  return GW_OK;
}

gw_status gw_autotune(gw_ctx ctx, int enable, int* n_tuned) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_autotune: ctx is NULL");
  gw::clear_error(ctx);
  if (enable >= 0) ctx->autotune = enable != 0;
  if (enable == 2) ctx->tuned.clear();
  if (n_tuned) *n_tuned = (int)ctx->tuned.size();
  return GW_OK;
}

// First line of a saved choice file: the format and the device the choices
// were timed on (architecture and compute-unit count).
static gw_status tune_file_header(gw_ctx ctx, std::string& out) {
  hipDeviceProp_t prop;
  GW_HIP(ctx, hipGetDeviceProperties(&prop, ctx->device));
  char buf[512];
  std::snprintf(buf, sizeof buf, "# gwlt autotune 1 arch=%s cus=%d", prop.gcnArchName,
                prop.multiProcessorCount);
  out = buf;
  return GW_OK;
}

gw_status gw_autotune_save(gw_ctx ctx, const char* path) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_autotune_save: ctx is NULL");
  gw::clear_error(ctx);
  if (!path) return gw::fail(ctx, GW_EINVAL, "gw_autotune_save: path is NULL");
  std::string hdr;
  GW_TRY(tune_file_header(ctx, hdr));
  std::ofstream f(path, std::ios::out | std::ios::trunc);
  if (!f) return gw::fail(ctx, GW_EINVAL, "gw_autotune_save: cannot open %s", path);
  f << hdr << "\n";
  for (const auto& kv : ctx->tuned) f << kv.second << " " << kv.first << "\n";
  f.close();
  if (!f) return gw::fail(ctx, GW_EINVAL, "gw_autotune_save: writing %s failed", path);
  return GW_OK;
}

gw_status gw_autotune_load(gw_ctx ctx, const char* path, int* n_loaded) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_autotune_load: ctx is NULL");
  gw::clear_error(ctx);
  if (n_loaded) *n_loaded = 0;
  if (!path) return gw::fail(ctx, GW_EINVAL, "gw_autotune_load: path is NULL");
  std::string hdr;
  GW_TRY(tune_file_header(ctx, hdr));
  std::ifstream f(path);
  if (!f) return gw::fail(ctx, GW_EINVAL, "gw_autotune_load: cannot open %s", path);
  std::string line;
  if (!std::getline(f, line) || line != hdr)
    return gw::fail(ctx, GW_EINVAL, "gw_autotune_load: %s was not saved on this device (%s)",
                    path, hdr.c_str());
  // parse everything first: a malformed file changes nothing
  std::map<std::string, int> got;
  int lineno = 1;
  while (std::getline(f, line)) {
    ++lineno;
    if (line.empty()) continue;
    std::istringstream ls(line);
    int choice = 0;
    std::string key;
    if (!(ls >> choice) || ls.get() != ' ' || !std::getline(ls, key) || key.empty() ||
        key.find(' ') != std::string::npos)
      return gw::fail(ctx, GW_EINVAL, "gw_autotune_load: %s line %d is malformed", path, lineno);
    got[key] = choice;
  }
  for (const auto& kv : got) ctx->tuned[kv.first] = kv.second;
  if (n_loaded) *n_loaded = (int)got.size();
  return GW_OK;
}

gw_status gw_autotune_restrict(gw_ctx ctx, const char* family, int modulus, int residue) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_autotune_restrict: ctx is NULL");
  gw::clear_error(ctx);
  if (!family || modulus < 0 || (modulus > 0 && (residue < 0 || residue >= modulus)))
    return gw::fail(ctx, GW_EINVAL, "gw_autotune_restrict: bad family, modulus or residue");
  if (modulus == 0)
    ctx->tune_filter.erase(family);
  else
    ctx->tune_filter[family] = {modulus, residue};
  return GW_OK;
}

gw_status gw_graph_begin(gw_ctx ctx) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_graph_begin: ctx is NULL");
  gw::clear_error(ctx);
  GW_HIP(ctx, hipSetDevice(ctx->device));
  return gw::begin_capture(ctx);
}

gw_status gw_graph_end(gw_ctx ctx, gw_graph* out) {
  if (!ctx || !out) return gw::fail(ctx, GW_EINVAL, "gw_graph_end: NULL argument");
  *out = nullptr;
  gw_graph_s g;
  GW_TRY(gw::end_capture(ctx, &g));
  *out = new gw_graph_s(g);
  ctx->live_graphs += 1;
  return GW_OK;
}

gw_status gw_graph_launch(gw_ctx ctx, gw_graph g) {
  if (!ctx || !g || g->ctx != ctx)
    return gw::fail(ctx, GW_EINVAL, "gw_graph_launch: bad graph or context");
  if (ctx->capturing) return gw::fail(ctx, GW_EUNSUPPORTED, "gw_graph_launch inside a capture");
  GW_HIP(ctx, hipSetDevice(ctx->device));
  GW_HIP(ctx, hipGraphLaunch(g->exec, ctx->stream));
  return GW_OK;
}

gw_status gw_graph_destroy(gw_graph g) {
  if (!g) return GW_OK;
  gw_ctx ctx = g->ctx;
  hipSetDevice(ctx->device);
  hipStreamSynchronize(ctx->stream);
  if (g->exec) hipGraphExecDestroy(g->exec);
  if (g->arena) hipFree(g->arena);
  ctx->live_graphs -= 1;
  delete g;
  return GW_OK;
}


gw_status gw_profile_enable(gw_ctx ctx, int enable) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_profile_enable: ctx is NULL");
  if (ctx->capturing) return gw::fail(ctx, GW_EUNSUPPORTED, "gw_profile_enable inside a graph capture");
  GW_HIP(ctx, hipStreamSynchronize(ctx->stream));
  gw::prof_resolve(ctx);
  ctx->prof_stats.clear();
  ctx->prof = enable != 0;
  return GW_OK;
}

gw_status gw_profile_get(gw_ctx ctx, const char* kernel, double* total_ms, int64_t* launches,
                         double* flops, double* bytes) {
  if (!ctx || !kernel) return gw::fail(ctx, GW_EINVAL, "gw_profile_get: NULL argument");
  if (ctx->capturing) return gw::fail(ctx, GW_EUNSUPPORTED, "gw_profile_get inside a graph capture");
  GW_HIP(ctx, hipStreamSynchronize(ctx->stream));
  gw::prof_resolve(ctx);
  auto it = ctx->prof_stats.find(kernel);
  const ProfStat z{};
  const ProfStat& s = it == ctx->prof_stats.end() ? z : it->second;
  if (total_ms) *total_ms = s.ms;
  if (launches) *launches = s.launches;
  if (flops) *flops = s.flops;
  if (bytes) *bytes = s.bytes;
  return GW_OK;
}

gw_status gw_create(gw_ctx* out, int device, void* hip_stream) {
  if (!out) return gw::fail(nullptr, GW_EINVAL, "gw_create: out is NULL");
  *out = nullptr;
  int n = 0;
  const hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess)
    return gw::fail(nullptr, GW_EDEVICE, "gw_create: hipGetDeviceCount failed: %s",
                    hipGetErrorString(e));
  if (device < 0 || device >= n)
    return gw::fail(nullptr, GW_EINVAL, "gw_create: no HIP device %d (%d visible)", device, n);
  if (hipSetDevice(device) != hipSuccess)
    return gw::fail(nullptr, GW_EDEVICE, "gw_create: hipSetDevice failed");
  gw_ctx c = new gw_ctx_s();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (hipHostMalloc(reinterpret_cast<void**>(&c->stage_host), kStageBytes) != hipSuccess ||
      !gw::ws_get(c, WS_STAGE, kStageBytes) ||
      hipMalloc(reinterpret_cast<void**>(&c->d_flags), 4 * sizeof(int)) != hipSuccess ||
      hipMemset(c->d_flags, 0, 4 * sizeof(int)) != hipSuccess) {
    gw_destroy(c);
    return gw::fail(nullptr, GW_ENOMEM, "gw_create: allocation failed");
  }
  // the no-allocation entry point's scratch address on this device; a
  // failure here is reported by that entry point, which retries the lookup
  (void)gw::sigma_scratch_init(c, device);
  gw::clear_error(c);
  *out = c;
  return GW_OK;
}

gw_status gw_destroy(gw_ctx ctx) {
  if (!ctx) return GW_OK;
  hipSetDevice(ctx->device);
  if (ctx->stream) hipStreamSynchronize(ctx->stream); else hipDeviceSynchronize();
  gw::drop_batch_graph(ctx);
  if (ctx->capture_stream) hipStreamDestroy(ctx->capture_stream);
  if (ctx->side_stream) {
    hipStreamSynchronize(ctx->side_stream);
    hipStreamDestroy(ctx->side_stream);
  }
  for (hipEvent_t e : ctx->side_ev)
    if (e) hipEventDestroy(e);
  for (int i = 0; i < WS_COUNT; ++i)
    if (ctx->ws[i]) hipFree(ctx->ws[i]);
  if (ctx->d_flags) hipFree(ctx->d_flags);
  if (ctx->stage_host) hipHostFree(ctx->stage_host);
  for (auto& e : ctx->prof_pending) {
    hipEventDestroy(e.a);
    hipEventDestroy(e.b);
  }
  delete ctx;
  return GW_OK;
}

gw_status gw_set_stream(gw_ctx ctx, void* hip_stream) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_set_stream: ctx is NULL");
  if (ctx->capturing) return gw::fail(ctx, GW_EUNSUPPORTED, "gw_set_stream inside a graph capture");
  GW_HIP(ctx, hipStreamSynchronize(ctx->stream));
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return GW_OK;
}

gw_status gw_sync(gw_ctx ctx) {
  if (!ctx) return gw::fail(nullptr, GW_EINVAL, "gw_sync: ctx is NULL");
  if (ctx->capturing) return gw::fail(ctx, GW_EUNSUPPORTED, "gw_sync inside a graph capture");
  GW_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return gw::check_flags(ctx);
}

const char* gw_last_error(gw_ctx ctx) {
  return ctx ? ctx->err.c_str() : g_free_err.c_str();
}

const char* gw_status_string(gw_status s) {
  switch (s) {
    case GW_OK: return "GW_OK";
    case GW_EINVAL: return "GW_EINVAL";
    case GW_ENOMEM: return "GW_ENOMEM";
    case GW_EDEVICE: return "GW_EDEVICE";
    case GW_ENOTSPD: return "GW_ENOTSPD";
    case GW_EPADE: return "GW_EPADE";
    case GW_ENOCONV: return "GW_ENOCONV";
    case GW_EUNSUPPORTED: return "GW_EUNSUPPORTED";
  }
  return "GW_UNKNOWN";
}

}  // extern "C"
