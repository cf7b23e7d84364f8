// Internal declarations shared by the HIP translation units of libgsplat.
// Nothing here is part of the public ABI (include/gsplat.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>

#include "gsplat.h"

namespace gs {

constexpr int kTile = GS_TILE;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;
constexpr float kDilation = 0.3f;
constexpr float kSlopeLimit = 1.3f;
constexpr float kRadiusMax = 4194304.0f;  // 2^22 px

// Camera as the kernels see it (passed by value).
struct DevCam {
  int width, height, tiles_x, tiles_y;
  float fx, fy, cx, cy, near_z, lim_x, lim_y;
  float R[9];
  float t[3];
  float centre[3];  // camera centre in world space, -R^T t
  float bg[3];
};

DevCam make_devcam(const gs_camera& c);

// thread-local error message
void set_error(const std::string& msg);
gs_status fail(gs_status code, const std::string& msg);
gs_status check_hip(hipError_t e, const char* what);
gs_status check_launch(const char* what);
gs_status validate_camera(const gs_camera* cam);

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Transmittance checkpoint buffer for K entries over `ntiles` tiles: the
// checkpoints, then the forward's tile plan, then each tile's work count
// (largest n_contrib of its pixels), which the backward plans from, then the
// forward's per-batch colour sums (three planes laid out like the checkpoints).
inline size_t ckpt_core_floats(int64_t k, int64_t ntiles) { return static_cast<size_t>(k / 256 + ntiles + 1) * 256; }
inline size_t ckpt_floats(int64_t k, int64_t ntiles) {
  // plan: 16-value header + one entry per tile; work counts: one per tile;
  // then the per-batch colour sums, three planes of the checkpoint layout
  return 4 * ckpt_core_floats(k, ntiles) + 16 + 2 * static_cast<size_t>(ntiles);
}

// Aligned carve-out of a caller-supplied workspace.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
    off += count * sizeof(T);
    return p;
  }
};

// ------------------------------------------------------------------ device

// floor division toward -inf by a positive constant
__device__ __forceinline__ int floordiv_tile(int a) {
  return (a >= 0) ? (a / kTile) : -((-a + kTile - 1) / kTile);
}

// Tile rectangle of the closed square [u - r, u + r] x [v - r, v + r]
// intersected with the tile grid, in integers after one floor of u and v.
// Returns the tile count (0 if none) and the inclusive bounds.
__device__ __forceinline__ int tile_rect(float u, float v, int r, int tx, int ty, int& x0, int& x1, int& y0,
                                         int& y1) {
  x0 = 0; x1 = -1; y0 = 0; y1 = -1;
  if (r <= 0 || !isfinite(u) || !isfinite(v)) return 0;
  const float fr = static_cast<float>(r);
  if (u < -fr || u >= static_cast<float>(kTile * tx + r)) return 0;
  if (v < -fr || v >= static_cast<float>(kTile * ty + r)) return 0;
  const int fu = static_cast<int>(floorf(u)), fv = static_cast<int>(floorf(v));
  x0 = max(0, floordiv_tile(fu - r));
  x1 = min(tx - 1, floordiv_tile(fu + r));
  y0 = max(0, floordiv_tile(fv - r));
  y1 = min(ty - 1, floordiv_tile(fv + r));
  if (x0 > x1 || y0 > y1) return 0;
  return (x1 - x0 + 1) * (y1 - y0 + 1);
}

// Map a linear block index to a work index so that consecutive work items land
// on the same XCD (blocks are dispatched round-robin over the 8 XCDs).
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  constexpr int kXcd = 8;
  const int per = nblocks / kXcd;
  const int rem = nblocks % kXcd;
  const int xcd = bid % kXcd;
  const int local = bid / kXcd;
  // XCDs [0, rem) own per+1 items, the rest own per items
  const int start = xcd * per + min(xcd, rem);
  return start + local;
}

// Row k of a [rows][n] structure-of-arrays field, advanced to the first of
// the THREADS consecutive elements of this workgroup.  The pointer is uniform
// across the workgroup and is pinned to scalar registers (readfirstlane keeps
// the compiler from folding the lane offset into it), so each load or store
// takes the scalar base plus the lane's 32-bit threadIdx.x offset: no per-lane
// 64-bit address arithmetic, and k * n is formed in 64 bits.
// The result points into the global address space, as the fields do.
template <typename T>
using global_ptr = __attribute__((address_space(1))) T*;
template <int THREADS, typename T>
__device__ __forceinline__ global_ptr<T> soa_row(T* base, int k, int64_t n) {
  const uint64_t a = reinterpret_cast<uint64_t>(base + static_cast<int64_t>(blockIdx.x) * THREADS +
                                                static_cast<int64_t>(k) * n);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(a));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(a >> 32));
  return reinterpret_cast<global_ptr<T>>((static_cast<uint64_t>(hi) << 32) | lo);
}

// Per-Gaussian gradient accumulator rows of the compositing backward (atomic
// mode): nine sums padded to 48 bytes (three float4s; a row lies within one
// 128-byte L2 line for six Gaussians in eight and straddles two for the
// rest; 64-byte rows, one line each, cost a third more HBM traffic to clear
// and re-read and measured slower).  The sums hold the record
// gradients up to constant factors (powers of 2 ln 2) that grad_scale applies
// once per Gaussian: u, v, Sigma'_xx, Sigma'_xy (both entries), Sigma'_yy,
// opacity, r, g, b.
constexpr int kAccStride = 12;
constexpr float kLn2 = 0.6931471805599453f;
__device__ __forceinline__ float grad_scale(int c) {
  constexpr float l1 = 2.0f * kLn2, l2 = 2.0f * kLn2 * kLn2;
  return c < 2 ? l1 : (c == 3 ? l2 + l2 : (c < 5 ? l2 : 1.0f));
}

}  // namespace gs

// Launchers implemented in the kernel translation units.
namespace gs {
// Measurement: while gs_kernel_timer_start is in effect on the calling
// thread, a TimedLaunch in scope around a kernel launch records a HIP event on
// the launch stream before and after it (a no-op otherwise).
struct TimedLaunch {
  TimedLaunch(const char* name, hipStream_t s);
  ~TimedLaunch();
  TimedLaunch(const TimedLaunch&) = delete;
  TimedLaunch& operator=(const TimedLaunch&) = delete;

 private:
  int slot_;
  hipStream_t s_;
};

gs_status launch_project(const gs_gaussians& g, const DevCam& cam, gs_projected& out, hipStream_t s);
constexpr int kPlanHeader = 16;
size_t plan_ints(int ntiles);
gs_status launch_tile_plan(int ntiles, const uint32_t* ranges, const uint32_t* counts, float heavy_factor,
                           int light_max, int32_t* plan, hipStream_t s);
// Also clears zero[0, zero_n4) (float4s) in the same launch when zero_n4 > 0.
gs_status launch_batch_plan(int ntiles, const uint32_t* ranges, const uint32_t* work, int light_max, int32_t* items,
                            int32_t* light, float4* zero, int64_t zero_n4, hipStream_t s);
// Backward work items (pairs) for K entries over ntiles tiles, with header.
inline size_t batch_item_ints(int64_t k, int64_t ntiles) {
  return 16 + 2 * static_cast<size_t>(k / 256 + ntiles + 1);
}
// Record gradients handed to the projection backward: g2d[9][n] (rows ==
// false) or the compositing backward's accumulator rows acc[n][kAccStride]
// before grad_scale (rows == true; with the learned colour the decoder's
// backward reads its colour gradient from them too).  stats (optional) gets
// |dL/d(u, v)| added per Gaussian and count += 1 where tiles_touched > 0.
// cgrad (optional, SH colour): the projection's colour_grad, read instead of
// the SH coefficients.
gs_status launch_project_bwd(const gs_gaussians& g, const DevCam& cam, const int* radius, const float* g2d, bool rows,
                             const uint32_t* tiles_touched, gs_densify_stats* stats, gs_gaussians_grad& grad,
                             void* ws, const float* cgrad, hipStream_t s);
size_t binsort_workspace(int64_t n, int64_t capacity, int tiles_x, int tiles_y);
// Exclusive prefix sum of n uint32 values (out may alias in); sums holds
// scan_sums_words(n) words, total (optional) receives the 64-bit sum.
size_t scan_sums_words(int64_t n);
gs_status launch_exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* sums,
                                unsigned long long* total, hipStream_t s);
// k_dev == NULL: waits for K (*k_out); else no wait, K and the look-back
// flag go to k_dev[0], k_dev[1] (direct emission only, see binsort_direct).
gs_status run_bin_sort(int64_t n, const gs_projected& proj, const DevCam& cam, void* ws, size_t ws_bytes,
                       uint32_t* point_list, int64_t capacity, uint32_t* ranges, int64_t* k_out,
                       unsigned long long* k_dev, hipStream_t s);
bool binsort_direct(int tiles_x, int tiles_y);
size_t density_workspace(int64_t n);
gs_status launch_density_control(const gs_gaussians& g, const gs_density_params& prm, const float* noise,
                                 gs_param_arrays& out, int64_t cap, void* ws, gs_density_report* rep,
                                 gs_density_points* pts_out, hipStream_t s);
gs_status launch_chs_table(const gs_projected& proj, const uint32_t* point_list, const uint32_t* ranges,
                           const DevCam& cam, uint32_t* tab_count, float* tab_sum, uint16_t* bucket_out,
                           uint32_t* rep_out, hipStream_t s);
gs_status launch_render_fwd(const gs_projected& proj, const uint32_t* point_list, const uint32_t* ranges, int64_t k,
                            const DevCam& cam, float* image, float* final_T, uint32_t* n_contrib, float* t_ckpt,
                            int schedule, hipStream_t s);
gs_status launch_render_count(const gs_projected& proj, const uint32_t* point_list, const uint32_t* ranges,
                              const DevCam& cam, unsigned long long* counts, hipStream_t s);
size_t render_bwd_workspace(int64_t n, int64_t k, int ntiles, int deterministic);
// g2d == NULL (atomic mode only): the sums stay in the accumulator rows,
// returned in *rows_out (acc[n][kAccStride], before grad_scale).
gs_status launch_render_bwd(int64_t n, const gs_projected& proj, const uint32_t* point_list, const uint32_t* ranges,
                            int64_t k, const DevCam& cam, const float* final_T,
                            const uint32_t* n_contrib, const float* t_ckpt, const float* dL_dimage, float* g2d, void* ws,
                            size_t ws_bytes, int deterministic, int schedule, const float** rows_out, hipStream_t s);
gs_status launch_mlp_pack(const uint16_t* params, void* packed, hipStream_t s);
gs_status launch_mlp_fwd(int64_t S, int per, const uint16_t* latents, const float* dirs, const void* packed,
                         float* rgb, hipStream_t s);
gs_status launch_mlp_render(int64_t n, const uint16_t* latents, const float* means, const int* radius,
                            const DevCam& cam, const void* packed, float* records, hipStream_t s);
size_t mlp_packed_bytes();
size_t mlp_bwd_workspace(int64_t S, int per);
gs_status launch_mlp_bwd(int64_t S, int per, const uint16_t* latents, const float* dirs, const void* packed,
                         const float* dL_drgb, const float* target, float scale, float* dlat, float* dparams,
                         float* loss, void* ws, hipStream_t s);
// dL/dc from g2d rows 6..8 (g2d[9][n], rows == false) or from entries 6..8
// of the accumulator rows acc[n][kAccStride] (rows == true; grad_scale is 1
// for the colour channels).
gs_status launch_mlp_render_bwd(int64_t n, const uint16_t* latents, const float* means, const int* radius,
                                const DevCam& cam, const void* packed, const float* g2d, bool rows, float* dlat,
                                float* dmeans, float* dparams, void* ws, hipStream_t s);
gs_status launch_sh_colour(int64_t S, int per, int64_t n, int deg, const float* sh, const float* dirs, int clamp01,
                           float* out, hipStream_t s);
gs_status launch_adam(int64_t n, float* p, const float* g, float* m, float* v, uint16_t* pb, float lr, float b1,
                      float b2, float eps, float bc1, float bc2, hipStream_t s);
gs_status launch_l1(const float* img, const float* target, int64_t count, float* loss, float* grad, float* partials,
                    hipStream_t s);
// Device address of the current GPU's copy of the no-allocation L1 scratch
// array (GS_L1_STATIC_PARTIALS floats), looked up once per device.
gs_status static_scratch(float** out);
gs_status launch_adam_gaussians(int64_t n, int sh_degree, const gs_param_arrays& p, const gs_gaussians_grad& g,
                                const gs_param_arrays& m, const gs_param_arrays& v, const gs_adam_config& cfg,
                                hipStream_t s);
}  // namespace gs
