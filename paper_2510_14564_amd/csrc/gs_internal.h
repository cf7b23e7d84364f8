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

}  // namespace gs

// Launchers implemented in the kernel translation units.
namespace gs {
gs_status launch_project(const gs_gaussians& g, const DevCam& cam, gs_projected& out, hipStream_t s);
constexpr int kPlanHeader = 16;
size_t plan_ints(int ntiles);
gs_status launch_tile_plan(int ntiles, const uint32_t* ranges, const uint32_t* counts, float heavy_factor,
                           int light_max, int32_t* plan, hipStream_t s);
gs_status launch_batch_plan(int ntiles, const uint32_t* ranges, const uint32_t* work, int light_max, int32_t* items,
                            int32_t* light, hipStream_t s);
// Backward work items (pairs) for K entries over ntiles tiles, with header.
inline size_t batch_item_ints(int64_t k, int64_t ntiles) {
  return 16 + 2 * static_cast<size_t>(k / 256 + ntiles + 1);
}
gs_status launch_project_bwd(const gs_gaussians& g, const DevCam& cam, const int* radius, const float* g2d,
                             gs_gaussians_grad& grad, void* ws, hipStream_t s);
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
gs_status launch_render_fwd(const gs_projected& proj, const uint32_t* point_list, const uint32_t* ranges, int64_t k,
                            const DevCam& cam, float* image, float* final_T, uint32_t* n_contrib, float* t_ckpt,
                            int schedule, hipStream_t s);
gs_status launch_render_count(const gs_projected& proj, const uint32_t* point_list, const uint32_t* ranges,
                              const DevCam& cam, unsigned long long* counts, hipStream_t s);
size_t render_bwd_workspace(int64_t n, int64_t k, int ntiles, int deterministic);
gs_status launch_render_bwd(int64_t n, const gs_projected& proj, const uint32_t* point_list, const uint32_t* ranges,
                            int64_t k, const DevCam& cam, const float* final_T,
                            const uint32_t* n_contrib, const float* t_ckpt, const float* dL_dimage, float* g2d, void* ws,
                            size_t ws_bytes, int deterministic, int schedule, hipStream_t s);
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
gs_status launch_mlp_render_bwd(int64_t n, const uint16_t* latents, const float* means, const int* radius,
                                const DevCam& cam, const void* packed, const float* g2d, float* dlat,
                                float* dmeans, float* dparams, void* ws, hipStream_t s);
gs_status launch_sh_colour(int64_t S, int per, int64_t n, int deg, const float* sh, const float* dirs, int clamp01,
                           float* out, hipStream_t s);
gs_status launch_adam(int64_t n, float* p, const float* g, float* m, float* v, uint16_t* pb, float lr, float b1,
                      float b2, float eps, float bc1, float bc2, hipStream_t s);
gs_status launch_l1(const float* img, const float* target, int64_t count, float* loss, float* grad, float* partials,
                    hipStream_t s);
}  // namespace gs
