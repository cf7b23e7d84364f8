// C ABI entry points of libgsplat: argument validation (before any HIP call),
// camera set-up and dispatch to the kernel launchers.
#include <math.h>

#include <cmath>
#include <cstdio>
#include <cstring>

#include <map>
#include <string>
#include <vector>

#include "gs_internal.h"

#include <atomic>
#include <mutex>

namespace gs {

static thread_local std::string t_error;

void set_error(const std::string& msg) { t_error = msg; }

gs_status fail(gs_status code, const std::string& msg) {
  set_error(msg);
  return code;
}

gs_status check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return GS_OK;
  return fail(GS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

gs_status check_launch(const char* what) { return check_hip(hipGetLastError(), what); }

gs_status validate_camera(const gs_camera* c) {
  if (!c) return fail(GS_ERR_INVALID_ARG, "camera is NULL");
  if (c->width <= 0 || c->height <= 0) return fail(GS_ERR_INVALID_ARG, "camera width/height must be positive");
  if (c->width > 32768 || c->height > 32768) return fail(GS_ERR_INVALID_ARG, "camera larger than 32768 px");
  const float vals[] = {c->fx, c->fy, c->cx, c->cy, c->near_z, c->tan_half_fov_x, c->tan_half_fov_y};
  for (float v : vals)
    if (!isfinite(v)) return fail(GS_ERR_INVALID_ARG, "camera has a non-finite intrinsic");
  if (!(c->fx > 0.f) || !(c->fy > 0.f) || !(c->near_z > 0.f) || !(c->tan_half_fov_x > 0.f) ||
      !(c->tan_half_fov_y > 0.f))
    return fail(GS_ERR_INVALID_ARG, "camera fx, fy, near_z and tan_half_fov must be positive");
  for (int i = 0; i < 9; ++i)
    if (!isfinite(c->R_cw[i])) return fail(GS_ERR_INVALID_ARG, "camera R_cw is not finite");
  for (int i = 0; i < 3; ++i)
    if (!isfinite(c->t_cw[i]) || !isfinite(c->bg[i])) return fail(GS_ERR_INVALID_ARG, "camera t_cw/bg not finite");
  return GS_OK;
}

DevCam make_devcam(const gs_camera& c) {
  DevCam d;
  d.width = c.width;
  d.height = c.height;
  d.tiles_x = (c.width + kTile - 1) / kTile;
  d.tiles_y = (c.height + kTile - 1) / kTile;
  d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
  d.near_z = c.near_z;
  d.lim_x = kSlopeLimit * c.tan_half_fov_x;
  d.lim_y = kSlopeLimit * c.tan_half_fov_y;
  for (int i = 0; i < 9; ++i) d.R[i] = c.R_cw[i];
  for (int i = 0; i < 3; ++i) { d.t[i] = c.t_cw[i]; d.bg[i] = c.bg[i]; }
  // camera centre -R^T t, formed in double and rounded once
  for (int i = 0; i < 3; ++i) {
    const double v = -(static_cast<double>(c.R_cw[i]) * c.t_cw[0] + static_cast<double>(c.R_cw[3 + i]) * c.t_cw[1] +
                       static_cast<double>(c.R_cw[6 + i]) * c.t_cw[2]);
    d.centre[i] = static_cast<float>(v);
  }
  return d;
}

static gs_status validate_gaussians(const gs_gaussians* g, const char* fn) {
  const std::string f(fn);
  if (!g) return fail(GS_ERR_INVALID_ARG, f + ": gaussians is NULL");
  if (g->n < 0) return fail(GS_ERR_INVALID_ARG, f + ": n < 0");
  if (g->n > (int64_t(1) << 30)) return fail(GS_ERR_INVALID_ARG, f + ": n above 2^30");
  if (g->colour_mode != 0 && g->colour_mode != 1) return fail(GS_ERR_INVALID_ARG, f + ": unknown colour_mode");
  if (g->colour_mode == 0 && (g->sh_degree < 0 || g->sh_degree > 3))
    return fail(GS_ERR_INVALID_ARG, f + ": sh_degree must be in 0..3");
  if (g->n > 0) {
    if (!g->means || !g->log_scales || !g->quats || !g->logits)
      return fail(GS_ERR_INVALID_ARG, f + ": NULL parameter array");
    if (g->colour_mode == 0 && !g->sh) return fail(GS_ERR_INVALID_ARG, f + ": sh is NULL");
    if (g->colour_mode == 1 && (!g->latents || !g->mlp))
      return fail(GS_ERR_INVALID_ARG, f + ": colour_mode 1 needs latents and the packed decoder");
    if (g->colour_mode == 1 && reinterpret_cast<uintptr_t>(g->latents) % 16 != 0)
      return fail(GS_ERR_INVALID_ARG, f + ": latents must be 16-byte aligned");
  }
  return GS_OK;
}

static gs_status validate_projected(const gs_projected* p, int64_t n, const char* fn) {
  const std::string f(fn);
  if (!p) return fail(GS_ERR_INVALID_ARG, f + ": projected is NULL");
  if (n > 0 && (!p->records || !p->depth || !p->radius || !p->tiles_touched))
    return fail(GS_ERR_INVALID_ARG, f + ": NULL projected array");
  if (reinterpret_cast<uintptr_t>(p->records) % 16 != 0)
    return fail(GS_ERR_INVALID_ARG, f + ": records must be 16-byte aligned");
  return GS_OK;
}

// ------------------------------------------------------------ kernel timer
// One timer per process: the backward of an autograd step runs on another
// host thread than its forward, and both must be seen.
namespace {
struct TimerRec {
  const char* name;
  hipEvent_t a, b;
};
std::atomic<bool> g_timing{false};
std::mutex g_timer_mu;
std::vector<TimerRec> g_recs;
std::vector<hipEvent_t> g_pool;
hipError_t g_timer_err = hipSuccess;

// caller holds g_timer_mu
hipEvent_t pool_get() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  const hipError_t r = hipEventCreate(&e);
  if (r != hipSuccess) {
    g_timer_err = r;
    return nullptr;
  }
  return e;
}
}  // namespace

TimedLaunch::TimedLaunch(const char* name, hipStream_t s) : slot_(-1), s_(s) {
  if (!g_timing.load(std::memory_order_acquire)) return;
  std::lock_guard<std::mutex> lock(g_timer_mu);
  hipEvent_t a = pool_get();
  hipEvent_t b = a ? pool_get() : nullptr;
  if (!b) {
    if (a) g_pool.push_back(a);
    return;
  }
  const hipError_t r = hipEventRecord(a, s);
  if (r != hipSuccess) {
    g_timer_err = r;
    g_pool.push_back(a);
    g_pool.push_back(b);
    return;
  }
  g_recs.push_back({name, a, b});
  slot_ = static_cast<int>(g_recs.size()) - 1;
}

TimedLaunch::~TimedLaunch() {
  if (slot_ < 0) return;
  std::lock_guard<std::mutex> lock(g_timer_mu);
  if (slot_ >= static_cast<int>(g_recs.size())) return;  // the timer was stopped meanwhile
  const hipError_t r = hipEventRecord(g_recs[slot_].b, s_);
  if (r != hipSuccess) g_timer_err = r;
}

}  // namespace gs

using namespace gs;

extern "C" {

const char* gs_last_error(void) { return t_error.c_str(); }

const char* gs_version(void) { return "gsplat-mi355 0.1 (gfx950)"; }

gs_status gs_project(const gs_gaussians* g, const gs_camera* cam, gs_projected* out, gs_stream stream) {
  set_error("");
  gs_status st;
  if ((st = validate_gaussians(g, "gs_project")) != GS_OK) return st;
  if ((st = validate_camera(cam)) != GS_OK) return st;
  if ((st = validate_projected(out, g->n, "gs_project")) != GS_OK) return st;
  return launch_project(*g, make_devcam(*cam), *out, static_cast<hipStream_t>(stream));
}

gs_status gs_bin_sort_workspace(int64_t n, int64_t capacity, const gs_camera* cam, size_t* bytes) {
  set_error("");
  gs_status st;
  if ((st = validate_camera(cam)) != GS_OK) return st;
  if (n < 0 || capacity < 0 || !bytes) return fail(GS_ERR_INVALID_ARG, "gs_bin_sort_workspace: bad n/capacity/bytes");
  const DevCam d = make_devcam(*cam);
  *bytes = binsort_workspace(n, capacity, d.tiles_x, d.tiles_y);
  return GS_OK;
}

gs_status gs_bin_sort(int64_t n, const gs_projected* proj, const gs_camera* cam, void* ws, size_t ws_bytes,
                      uint32_t* point_list, int64_t capacity, uint32_t* ranges, int64_t* k_out, gs_stream stream) {
  set_error("");
  gs_status st;
  if (n < 0 || n > (int64_t(1) << 30)) return fail(GS_ERR_INVALID_ARG, "gs_bin_sort: bad n");
  if ((st = validate_camera(cam)) != GS_OK) return st;
  if ((st = validate_projected(proj, n, "gs_bin_sort")) != GS_OK) return st;
  if (!k_out || !ranges || capacity < 0 || (capacity > 0 && !point_list) || (!ws && ws_bytes > 0))
    return fail(GS_ERR_INVALID_ARG, "gs_bin_sort: NULL output or negative capacity");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(GS_ERR_INVALID_ARG, "gs_bin_sort: ws not 256-aligned");
  const DevCam d = make_devcam(*cam);
  if (ws_bytes < binsort_workspace(n, capacity, d.tiles_x, d.tiles_y))
    return fail(GS_ERR_INVALID_ARG, "gs_bin_sort: workspace too small");
  return run_bin_sort(n, *proj, d, ws, ws_bytes, point_list, capacity, ranges, k_out, nullptr,
                      static_cast<hipStream_t>(stream));
}

gs_status gs_bin_sort_async(int64_t n, const gs_projected* proj, const gs_camera* cam, void* ws, size_t ws_bytes,
                            uint32_t* point_list, int64_t capacity, uint32_t* ranges, uint64_t* k_dev,
                            gs_stream stream) {
  set_error("");
  gs_status st;
  if (n < 0 || n > (int64_t(1) << 30)) return fail(GS_ERR_INVALID_ARG, "gs_bin_sort_async: bad n");
  if ((st = validate_camera(cam)) != GS_OK) return st;
  if ((st = validate_projected(proj, n, "gs_bin_sort_async")) != GS_OK) return st;
  if (!k_dev || !ranges || capacity < 0 || (capacity > 0 && !point_list) || (!ws && ws_bytes > 0))
    return fail(GS_ERR_INVALID_ARG, "gs_bin_sort_async: NULL output or negative capacity");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
    return fail(GS_ERR_INVALID_ARG, "gs_bin_sort_async: ws not 256-aligned");
  const DevCam d = make_devcam(*cam);
  if (!binsort_direct(d.tiles_x, d.tiles_y))
    return fail(GS_ERR_UNSUPPORTED, "gs_bin_sort_async: frame too large for the direct emission; use gs_bin_sort");
  if (ws_bytes < binsort_workspace(n, capacity, d.tiles_x, d.tiles_y))
    return fail(GS_ERR_INVALID_ARG, "gs_bin_sort_async: workspace too small");
  return run_bin_sort(n, *proj, d, ws, ws_bytes, point_list, capacity, ranges, nullptr,
                      reinterpret_cast<unsigned long long*>(k_dev), static_cast<hipStream_t>(stream));
}

namespace {
// The schedule argument of the compositing calls: a work split in the low
// byte, optionally or-ed with GS_RENDER_COLOUR_HASH.
gs_status validate_schedule(int32_t schedule, int32_t deterministic, bool backward, const char* fn) {
  const int32_t split = schedule & 0xFF, flags = schedule & ~0xFF;
  if (split < GS_SCHEDULE_PLAIN || split > GS_SCHEDULE_MERGED || (flags & ~GS_RENDER_COLOUR_HASH) != 0)
    return fail(GS_ERR_INVALID_ARG, std::string(fn) + ": unknown schedule");
  if (flags && split == GS_SCHEDULE_MERGED)
    return fail(GS_ERR_UNSUPPORTED, std::string(fn) + ": colour-hash sampling needs schedule PLAIN or BALANCED");
  if (flags && backward && deterministic)
    return fail(GS_ERR_UNSUPPORTED, std::string(fn) + ": colour-hash sampling has no deterministic backward");
  return GS_OK;
}
}  // namespace

gs_status gs_render_fwd(int64_t n, const gs_projected* proj, const uint32_t* point_list, const uint32_t* ranges,
                        int64_t k, const gs_camera* cam, float* image, float* final_T, uint32_t* n_contrib,
                        float* t_ckpt, int32_t schedule, gs_stream stream) {
  set_error("");
  gs_status st;
  if (n < 0 || k < 0) return fail(GS_ERR_INVALID_ARG, "gs_render_fwd: negative n or k");
  if ((st = validate_camera(cam)) != GS_OK) return st;
  if ((st = validate_projected(proj, n, "gs_render_fwd")) != GS_OK) return st;
  if (!ranges || !image || !final_T || !n_contrib || (k > 0 && !point_list))
    return fail(GS_ERR_INVALID_ARG, "gs_render_fwd: NULL array");
  if ((st = validate_schedule(schedule, 0, false, "gs_render_fwd")) != GS_OK) return st;
  if ((schedule & 0xFF) != GS_SCHEDULE_PLAIN && !t_ckpt)
    return fail(GS_ERR_INVALID_ARG, "gs_render_fwd: the balanced schedules keep their plan in t_ckpt");
  return launch_render_fwd(*proj, point_list, ranges, k, make_devcam(*cam), image, final_T, n_contrib, t_ckpt,
                           schedule, static_cast<hipStream_t>(stream));
}

gs_status gs_render_count(int64_t n, const gs_projected* proj, const uint32_t* point_list, const uint32_t* ranges,
                          int64_t k, const gs_camera* cam, uint64_t* counts, gs_stream stream) {
  set_error("");
  gs_status st;
  if (n < 0 || k < 0) return fail(GS_ERR_INVALID_ARG, "gs_render_count: negative n or k");
  if ((st = validate_camera(cam)) != GS_OK) return st;
  if ((st = validate_projected(proj, n, "gs_render_count")) != GS_OK) return st;
  if (!ranges || !counts || (k > 0 && !point_list)) return fail(GS_ERR_INVALID_ARG, "gs_render_count: NULL array");
  return launch_render_count(*proj, point_list, ranges, make_devcam(*cam),
                             reinterpret_cast<unsigned long long*>(counts), static_cast<hipStream_t>(stream));
}

gs_status gs_colour_hash_table(int64_t n, const gs_projected* proj, const uint32_t* point_list,
                               const uint32_t* ranges, int64_t k, const gs_camera* cam, uint32_t* count,
                               float* sums, uint16_t* bucket, uint32_t* rep, gs_stream stream) {
  set_error("");
  gs_status st;
  if (n < 0 || k < 0) return fail(GS_ERR_INVALID_ARG, "gs_colour_hash_table: negative n or k");
  if ((st = validate_camera(cam)) != GS_OK) return st;
  if ((st = validate_projected(proj, n, "gs_colour_hash_table")) != GS_OK) return st;
  if (!ranges || (k > 0 && !point_list)) return fail(GS_ERR_INVALID_ARG, "gs_colour_hash_table: NULL array");
  return launch_chs_table(*proj, point_list, ranges, make_devcam(*cam), count, sums, bucket, rep,
                          static_cast<hipStream_t>(stream));
}

gs_status gs_render_ckpt_floats(int64_t k, const gs_camera* cam, size_t* floats) {
  set_error("");
  gs_status st;
  if ((st = validate_camera(cam)) != GS_OK) return st;
  if (k < 0 || !floats) return fail(GS_ERR_INVALID_ARG, "gs_render_ckpt_floats: bad arguments");
  const DevCam d = make_devcam(*cam);
  *floats = ckpt_floats(k, static_cast<int64_t>(d.tiles_x) * d.tiles_y);
  return GS_OK;
}

gs_status gs_render_bwd_2d_workspace(int64_t n, int64_t k, const gs_camera* cam, int32_t deterministic,
                                     size_t* bytes) {
  set_error("");
  gs_status st;
  if ((st = validate_camera(cam)) != GS_OK) return st;
  if (n < 0 || k < 0 || !bytes) return fail(GS_ERR_INVALID_ARG, "gs_render_bwd_2d_workspace: bad arguments");
  const DevCam d = make_devcam(*cam);
  *bytes = render_bwd_workspace(n, k, d.tiles_x * d.tiles_y, deterministic);
  return GS_OK;
}

gs_status gs_render_bwd_2d(int64_t n, const gs_projected* proj, const uint32_t* point_list, const uint32_t* ranges,
                           int64_t k, const gs_camera* cam, const float* final_T, const uint32_t* n_contrib,
                           const float* t_ckpt, const float* dL_dimage, float* g2d, void* ws, size_t ws_bytes,
                           int32_t deterministic, int32_t schedule, gs_stream stream) {
  set_error("");
  gs_status st;
  if (n < 0 || k < 0) return fail(GS_ERR_INVALID_ARG, "gs_render_bwd_2d: negative n or k");
  if ((st = validate_camera(cam)) != GS_OK) return st;
  if ((st = validate_projected(proj, n, "gs_render_bwd_2d")) != GS_OK) return st;
  if (!ranges || !final_T || !n_contrib || !t_ckpt || !dL_dimage || (n > 0 && !g2d) || (k > 0 && !point_list))
    return fail(GS_ERR_INVALID_ARG, "gs_render_bwd_2d: NULL array");
  const DevCam d = make_devcam(*cam);
  if ((st = validate_schedule(schedule, deterministic, true, "gs_render_bwd_2d")) != GS_OK) return st;
  if (ws_bytes < render_bwd_workspace(n, k, d.tiles_x * d.tiles_y, deterministic) || !ws)
    return fail(GS_ERR_INVALID_ARG, "gs_render_bwd_2d: workspace too small");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(GS_ERR_INVALID_ARG, "gs_render_bwd_2d: ws not 256-aligned");
  if (n == 0) return GS_OK;
  return launch_render_bwd(n, *proj, point_list, ranges, k, d, final_T, n_contrib, t_ckpt, dL_dimage, g2d, ws,
                           ws_bytes, deterministic, schedule, nullptr, static_cast<hipStream_t>(stream));
}

// Workspace of the full backward: the record gradients g2d[9][n] (unless the
// projection reads the compositing's accumulator rows directly: atomic mode,
// SH colour), the compositing backward's workspace, the decoder backward's.
namespace {
struct FullBwdWs {
  float* g2d;
  void* ws2d;
  void* wspb;
  size_t bytes;
  bool rows;
};
FullBwdWs carve_full_bwd(void* base, const gs_gaussians& g, int64_t k, int ntiles, int deterministic) {
  FullBwdWs f;
  f.rows = !deterministic;
  Carver c(base);
  f.g2d = c.take<float>(f.rows ? 0 : static_cast<size_t>(GS_G2D) * static_cast<size_t>(g.n));
  f.ws2d = c.take<char>(render_bwd_workspace(g.n, k, ntiles, deterministic));
  f.wspb = c.take<char>(g.colour_mode == 1 ? mlp_bwd_workspace(g.n, 1) : 0);
  f.bytes = c.off;
  return f;
}
}  // namespace

gs_status gs_render_bwd_workspace(const gs_gaussians* g, int64_t k, const gs_camera* cam, int32_t deterministic,
                                  size_t* bytes) {
  set_error("");
  gs_status st;
  if ((st = validate_gaussians(g, "gs_render_bwd_workspace")) != GS_OK) return st;
  if ((st = validate_camera(cam)) != GS_OK) return st;
  if (k < 0 || !bytes) return fail(GS_ERR_INVALID_ARG, "gs_render_bwd_workspace: bad arguments");
  const DevCam d = make_devcam(*cam);
  *bytes = carve_full_bwd(nullptr, *g, k, d.tiles_x * d.tiles_y, deterministic).bytes;
  return GS_OK;
}

gs_status gs_render_bwd(const gs_gaussians* g, const gs_camera* cam, const gs_projected* proj,
                        const uint32_t* point_list, const uint32_t* ranges, int64_t k, const float* final_T,
                        const uint32_t* n_contrib, const float* t_ckpt, const float* dL_dimage,
                        gs_gaussians_grad* grad, gs_densify_stats* stats, void* ws, size_t ws_bytes,
                        int32_t deterministic, int32_t schedule, gs_stream stream) {
  set_error("");
  gs_status st;
  if ((st = validate_gaussians(g, "gs_render_bwd")) != GS_OK) return st;
  if ((st = validate_camera(cam)) != GS_OK) return st;
  const int64_t n = g->n;
  if (k < 0) return fail(GS_ERR_INVALID_ARG, "gs_render_bwd: negative k");
  if ((st = validate_projected(proj, n, "gs_render_bwd")) != GS_OK) return st;
  if (!ranges || !final_T || !n_contrib || !t_ckpt || !dL_dimage || (k > 0 && !point_list))
    return fail(GS_ERR_INVALID_ARG, "gs_render_bwd: NULL array");
  if (!grad) return fail(GS_ERR_INVALID_ARG, "gs_render_bwd: grad is NULL");
  const bool mlp = g->colour_mode == 1;
  if (n > 0 && (!grad->means || !grad->log_scales || !grad->quats || !grad->logits || (!mlp && !grad->sh) ||
                (mlp && (!grad->latents || !grad->mlp))))
    return fail(GS_ERR_INVALID_ARG, "gs_render_bwd: NULL gradient array");
  if (stats && n > 0 && (!stats->grad_norm_sum || !stats->visible_count))
    return fail(GS_ERR_INVALID_ARG, "gs_render_bwd: NULL densification statistics array");
  if ((st = validate_schedule(schedule, deterministic, true, "gs_render_bwd")) != GS_OK) return st;
  const DevCam d = make_devcam(*cam);
  const FullBwdWs layout = carve_full_bwd(nullptr, *g, k, d.tiles_x * d.tiles_y, deterministic);
  if (!ws || ws_bytes < layout.bytes) return fail(GS_ERR_INVALID_ARG, "gs_render_bwd: workspace too small");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(GS_ERR_INVALID_ARG, "gs_render_bwd: ws not 256-aligned");
  if (n == 0) return GS_OK;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const FullBwdWs f = carve_full_bwd(ws, *g, k, d.tiles_x * d.tiles_y, deterministic);
  const float* rows = nullptr;
  st = launch_render_bwd(n, *proj, point_list, ranges, k, d, final_T, n_contrib, t_ckpt, dL_dimage,
                         f.rows ? nullptr : f.g2d, f.ws2d, ws_bytes - (static_cast<char*>(f.ws2d) - static_cast<char*>(ws)),
                         deterministic, schedule, &rows, s);
  if (st != GS_OK) return st;
  return launch_project_bwd(*g, d, proj->radius, f.rows ? rows : f.g2d, f.rows, proj->tiles_touched, stats, *grad,
                            f.wspb, g->colour_mode == 1 ? nullptr : proj->colour_grad, s);
}

gs_status gs_project_bwd_workspace(const gs_gaussians* g, size_t* bytes) {
  set_error("");
  if (!g || !bytes) return fail(GS_ERR_INVALID_ARG, "gs_project_bwd_workspace: NULL pointer");
  if (g->n < 0 || g->n > (int64_t(1) << 30)) return fail(GS_ERR_INVALID_ARG, "gs_project_bwd_workspace: bad n");
  *bytes = g->colour_mode == 1 ? mlp_bwd_workspace(g->n, 1) : 0;
  return GS_OK;
}

gs_status gs_project_bwd(const gs_gaussians* g, const gs_camera* cam, const gs_projected* proj, const float* g2d,
                         gs_gaussians_grad* grad, void* ws, size_t ws_bytes, gs_stream stream) {
  set_error("");
  gs_status st;
  if ((st = validate_gaussians(g, "gs_project_bwd")) != GS_OK) return st;
  if ((st = validate_camera(cam)) != GS_OK) return st;
  if (!grad) return fail(GS_ERR_INVALID_ARG, "gs_project_bwd: grad is NULL");
  const bool mlp = g->colour_mode == 1;
  if (g->n > 0 && (!g2d || !grad->means || !grad->log_scales || !grad->quats || !grad->logits ||
                   (!mlp && !grad->sh) || (mlp && (!grad->latents || !grad->mlp))))
    return fail(GS_ERR_INVALID_ARG, "gs_project_bwd: NULL gradient array");
  if (mlp && g->n > 0) {
    if (!proj || !proj->radius) return fail(GS_ERR_INVALID_ARG, "gs_project_bwd: colour_mode 1 needs proj->radius");
    if (!ws || ws_bytes < mlp_bwd_workspace(g->n, 1))
      return fail(GS_ERR_INVALID_ARG, "gs_project_bwd: workspace too small");
  }
  if (g->n == 0) return GS_OK;
  return launch_project_bwd(*g, make_devcam(*cam), mlp ? proj->radius : nullptr, g2d, false, nullptr, nullptr, *grad,
                            ws, (!mlp && proj) ? proj->colour_grad : nullptr, static_cast<hipStream_t>(stream));
}

gs_status gs_mlp_pack(const uint16_t* params, void* packed, gs_stream stream) {
  set_error("");
  if (!params || !packed) return fail(GS_ERR_INVALID_ARG, "gs_mlp_pack: NULL pointer");
  if (reinterpret_cast<uintptr_t>(packed) % 16 != 0) return fail(GS_ERR_INVALID_ARG, "gs_mlp_pack: packed not aligned");
  return launch_mlp_pack(params, packed, static_cast<hipStream_t>(stream));
}

gs_status gs_mlp_fwd(int64_t S, int32_t per, const uint16_t* latents, const float* dirs, const void* packed,
                     float* rgb, gs_stream stream) {
  set_error("");
  if (S < 0 || S > (int64_t(1) << 31) - 64 || per <= 0) return fail(GS_ERR_INVALID_ARG, "gs_mlp_fwd: bad S or per");
  if (S > 0 && (!latents || !dirs || !packed || !rgb)) return fail(GS_ERR_INVALID_ARG, "gs_mlp_fwd: NULL pointer");
  if (reinterpret_cast<uintptr_t>(latents) % 16 != 0 || reinterpret_cast<uintptr_t>(packed) % 16 != 0)
    return fail(GS_ERR_INVALID_ARG, "gs_mlp_fwd: latents and packed must be 16-byte aligned");
  return launch_mlp_fwd(S, per, latents, dirs, packed, rgb, static_cast<hipStream_t>(stream));
}

static bool pow2_per(int32_t per) { return per > 0 && per <= 4096 && (per & (per - 1)) == 0; }

gs_status gs_mlp_bwd_workspace(int64_t S, int32_t per, size_t* bytes) {
  set_error("");
  if (!bytes || S < 0 || S > (int64_t(1) << 31) - 64 || !pow2_per(per))
    return fail(GS_ERR_INVALID_ARG, "gs_mlp_bwd_workspace: bad arguments");
  *bytes = mlp_bwd_workspace(S, per);
  return GS_OK;
}

gs_status gs_mlp_bwd(int64_t S, int32_t per, const uint16_t* latents, const float* dirs, const void* packed,
                     const float* dL_drgb, const float* target, float scale, float* dlatents, float* dparams,
                     float* loss, void* ws, size_t ws_bytes, gs_stream stream) {
  set_error("");
  if (S < 0 || S > (int64_t(1) << 31) - 64 || !pow2_per(per) || S % per != 0)
    return fail(GS_ERR_INVALID_ARG, "gs_mlp_bwd: S must be a multiple of per, per a power of two <= 4096");
  if (!packed || !dparams || (S > 0 && (!latents || !dirs || !dlatents || (!dL_drgb && !target))))
    return fail(GS_ERR_INVALID_ARG, "gs_mlp_bwd: NULL pointer");
  if (reinterpret_cast<uintptr_t>(latents) % 16 != 0 || reinterpret_cast<uintptr_t>(packed) % 16 != 0)
    return fail(GS_ERR_INVALID_ARG, "gs_mlp_bwd: latents and packed must be 16-byte aligned");
  if (!std::isfinite(scale)) return fail(GS_ERR_INVALID_ARG, "gs_mlp_bwd: scale not finite");
  if (!ws || ws_bytes < mlp_bwd_workspace(S, per)) return fail(GS_ERR_INVALID_ARG, "gs_mlp_bwd: workspace too small");
  return launch_mlp_bwd(S, per, latents, dirs, packed, dL_drgb, dL_drgb ? nullptr : target, scale, dlatents, dparams,
                        loss, ws, static_cast<hipStream_t>(stream));
}

gs_status gs_sh_colour(int64_t S, int32_t per, int64_t n, int32_t sh_degree, const float* sh, const float* dirs,
                       int32_t clamp01, float* rgb, gs_stream stream) {
  set_error("");
  if (S < 0 || S > (int64_t(1) << 31) - 256 || per <= 0 || n < 0 || sh_degree < 0 || sh_degree > 3 ||
      (S + per - 1) / per > n)
    return fail(GS_ERR_INVALID_ARG, "gs_sh_colour: bad sizes");
  if (S > 0 && (!sh || !dirs || !rgb)) return fail(GS_ERR_INVALID_ARG, "gs_sh_colour: NULL pointer");
  return launch_sh_colour(S, per, n, sh_degree, sh, dirs, clamp01, rgb, static_cast<hipStream_t>(stream));
}

gs_status gs_adam_step(int64_t n, float* param, const float* grad, float* m, float* v, uint16_t* param_bf16,
                       float lr, float beta1, float beta2, float eps, int32_t step, gs_stream stream) {
  set_error("");
  if (n < 0 || step < 1 || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
      !std::isfinite(lr) || !(eps > 0.0f))
    return fail(GS_ERR_INVALID_ARG, "gs_adam_step: bad arguments");
  if (n > 0 && (!param || !grad || !m || !v)) return fail(GS_ERR_INVALID_ARG, "gs_adam_step: NULL pointer");
  const double bc1 = 1.0 - std::pow(static_cast<double>(beta1), step);
  const double bc2 = 1.0 - std::pow(static_cast<double>(beta2), step);
  return launch_adam(n, param, grad, m, v, param_bf16, lr, beta1, beta2, eps, static_cast<float>(bc1),
                     static_cast<float>(bc2), static_cast<hipStream_t>(stream));
}

gs_status gs_adam_gaussians(int64_t n, int32_t sh_degree, const gs_param_arrays* params, const gs_gaussians_grad* grad,
                            const gs_param_arrays* m, const gs_param_arrays* v, const gs_adam_config* cfg,
                            gs_stream stream) {
  set_error("");
  if (n < 0 || n > (int64_t(1) << 30) || sh_degree < 0 || sh_degree > 3 || !params || !grad || !m || !v || !cfg)
    return fail(GS_ERR_INVALID_ARG, "gs_adam_gaussians: bad arguments");
  const float lrs[] = {cfg->lr_means, cfg->lr_log_scales, cfg->lr_quats, cfg->lr_logits, cfg->lr_sh_dc,
                       cfg->lr_sh_rest};
  for (float lr : lrs)
    if (!std::isfinite(lr)) return fail(GS_ERR_INVALID_ARG, "gs_adam_gaussians: non-finite learning rate");
  if (cfg->step < 1 || !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) || !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) ||
      !(cfg->eps > 0.0f))
    return fail(GS_ERR_INVALID_ARG, "gs_adam_gaussians: bad step, betas or eps");
  if (n > 0) {
    const gs_param_arrays* sets[] = {params, m, v};
    for (const gs_param_arrays* a : sets)
      if (!a->means || !a->log_scales || !a->quats || !a->logits || !a->sh)
        return fail(GS_ERR_INVALID_ARG, "gs_adam_gaussians: NULL parameter or moment array");
    if (!grad->means || !grad->log_scales || !grad->quats || !grad->logits || !grad->sh)
      return fail(GS_ERR_INVALID_ARG, "gs_adam_gaussians: NULL gradient array");
  }
  if (n == 0) return GS_OK;
  return launch_adam_gaussians(n, sh_degree, *params, *grad, *m, *v, *cfg, static_cast<hipStream_t>(stream));
}

gs_status gs_density_control_workspace(int64_t n, size_t* bytes) {
  set_error("");
  if (n < 0 || n > (int64_t(1) << 30) || !bytes) return fail(GS_ERR_INVALID_ARG, "gs_density_control_workspace: bad arguments");
  *bytes = density_workspace(n);
  return GS_OK;
}

gs_status gs_density_control(const gs_gaussians* g, const gs_density_params* prm, const float* noise,
                             gs_param_arrays* out, int64_t capacity, void* ws, size_t ws_bytes,
                             gs_density_report* report, gs_density_points* points, gs_stream stream) {
  set_error("");
  gs_status st;
  if ((st = validate_gaussians(g, "gs_density_control")) != GS_OK) return st;
  if (g->colour_mode != 0) return fail(GS_ERR_INVALID_ARG, "gs_density_control: SH colour (colour_mode 0) only");
  if (!prm || !out || capacity < 0) return fail(GS_ERR_INVALID_ARG, "gs_density_control: bad arguments");
  const gs_density_params& p = *prm;
  if (!(p.radius > 0.0f) || !std::isfinite(p.radius) || !(p.alpha >= 0.0f) || !std::isfinite(p.alpha) ||
      !(p.beta >= 0.0f) || !std::isfinite(p.beta) || p.knn < 1 || p.knn > 8 || !std::isfinite(p.spread) ||
      !(p.jitter >= 0.0f) || !std::isfinite(p.jitter) || !std::isfinite(p.gamma))
    return fail(GS_ERR_INVALID_ARG, "gs_density_control: parameter out of range");
  if (g->n > 0 && (!noise || !out->means || !out->log_scales || !out->quats || !out->logits || !out->sh))
    return fail(GS_ERR_INVALID_ARG, "gs_density_control: NULL array");
  if (!ws || ws_bytes < density_workspace(g->n)) return fail(GS_ERR_INVALID_ARG, "gs_density_control: workspace too small");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(GS_ERR_INVALID_ARG, "gs_density_control: ws not 256-aligned");
  return launch_density_control(*g, p, noise, *out, capacity, ws, report, points, static_cast<hipStream_t>(stream));
}

gs_status gs_kernel_timer_start(void) {
  set_error("");
  std::lock_guard<std::mutex> lock(g_timer_mu);
  if (g_timing.load()) return fail(GS_ERR_INVALID_ARG, "gs_kernel_timer_start: the timer is already running");
  g_recs.clear();
  g_timer_err = hipSuccess;
  g_timing.store(true, std::memory_order_release);
  return GS_OK;
}

gs_status gs_kernel_timer_stop(char* buf, size_t size, size_t* needed) {
  set_error("");
  std::vector<TimerRec> recs;
  hipError_t terr;
  {
    std::lock_guard<std::mutex> lock(g_timer_mu);
    if (!g_timing.load()) return fail(GS_ERR_INVALID_ARG, "gs_kernel_timer_stop: the timer is not running");
    g_timing.store(false, std::memory_order_release);
    recs.swap(g_recs);
    terr = g_timer_err;
  }
  std::vector<std::string> order;
  std::map<std::string, std::pair<long long, double>> acc;
  gs_status st = GS_OK;
  for (const TimerRec& r : recs) {
    float ms = 0.0f;
    if (st == GS_OK) st = check_hip(hipEventSynchronize(r.b), "hipEventSynchronize");
    if (st == GS_OK) st = check_hip(hipEventElapsedTime(&ms, r.a, r.b), "hipEventElapsedTime");
    auto it = acc.find(r.name);
    if (it == acc.end()) {
      order.push_back(r.name);
      it = acc.emplace(r.name, std::make_pair(0LL, 0.0)).first;
    }
    it->second.first += 1;
    it->second.second += ms;
  }
  {
    std::lock_guard<std::mutex> lock(g_timer_mu);
    for (const TimerRec& r : recs) {
      g_pool.push_back(r.a);
      g_pool.push_back(r.b);
    }
  }
  if (st == GS_OK && terr != hipSuccess) st = check_hip(terr, "kernel timer event");
  std::string out;
  for (const std::string& name : order) {
    char line[256];
    snprintf(line, sizeof line, "%s %lld %.6f\n", name.c_str(), acc[name].first, acc[name].second);
    out += line;
  }
  if (needed) *needed = out.size() + 1;
  if (buf && size > 0) {
    const size_t m = std::min(size - 1, out.size());
    memcpy(buf, out.data(), m);
    buf[m] = '\0';
  }
  return st;
}

gs_status gs_l1_loss(const float* img, const float* target, int64_t count, float* loss, float* grad,
                     float* partials, gs_stream stream) {
  set_error("");
  if (count <= 0 || !img || !target || !loss || !partials)
    return fail(GS_ERR_INVALID_ARG, "gs_l1_loss: bad arguments");
  return launch_l1(img, target, count, loss, grad, partials, static_cast<hipStream_t>(stream));
}

gs_status gs_l1_loss_static(const float* img, const float* target, int64_t count, float* loss, float* grad,
                            gs_stream stream) {
  set_error("");
  if (count <= 0 || !img || !target || !loss)
    return fail(GS_ERR_INVALID_ARG, "gs_l1_loss_static: bad arguments");
  // one partial sum per partial-sum workgroup, at most GS_L1_PARTIALS of them
  if (std::min<int64_t>(GS_L1_PARTIALS, ceil_div(count, 256)) > GS_L1_STATIC_PARTIALS)
    return fail(GS_ERR_CAPACITY, "gs_l1_loss_static: more partial sums than the static scratch holds");
  float* partials = nullptr;
  gs_status st = static_scratch(&partials);
  if (st != GS_OK) return st;
  return launch_l1(img, target, count, loss, grad, partials, static_cast<hipStream_t>(stream));
}

}  // extern "C"
