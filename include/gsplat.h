/*
 * gsplat.h -- C ABI of the MI355X (gfx950) differentiable tile-splatting library
 * (libgsplat.so).  It implements the per-iteration hot path of 3D Gaussian
 * Splatting training that BalanceGS (arXiv 2510.14564) accelerates: projection
 * of 3D Gaussians to 2D conics with SH colour, binning into 16x16 tiles with a
 * depth sort, front-to-back compositing, and the matching backward pass.
 *
 * Conventions shared by every call:
 *  - Every array pointer is a DEVICE pointer owned by the caller; the library
 *    never frees or retains it.  Descriptor structs (gs_camera, gs_gaussians,
 *    ...) live in HOST memory and are read during the call only.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the default stream)
 *    and is asynchronous, except gs_bin_sort, which synchronises `stream` once
 *    to read the number of (tile, Gaussian) pairs.
 *  - Arrays are structure-of-arrays with the Gaussian index fastest, so that
 *    consecutive threads read consecutive addresses.
 *  - Gradient outputs are overwritten, never accumulated.
 *  - Every call returns a gs_status.  Argument checks run before any HIP call,
 *    so a GS_ERR_INVALID_ARG return never touches the device.  The message of
 *    the last failure on the calling thread is available from gs_last_error().
 *  - Scalars are FP32; index and count arrays are uint32/int32.
 */
#ifndef GSPLAT_MI355_H
#define GSPLAT_MI355_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* gs_stream; /* hipStream_t */

typedef enum {
  GS_OK = 0,
  GS_ERR_INVALID_ARG = -1, /* bad pointer, size, degree, camera or workspace */
  GS_ERR_CAPACITY = -2,    /* output capacity too small; required size reported */
  GS_ERR_HIP = -3,         /* a HIP runtime call or kernel launch failed */
  GS_ERR_UNSUPPORTED = -4  /* a valid but unimplemented combination */
} gs_status;

#define GS_TILE 16        /* tile edge in pixels: 16x16 pixel blocks share one list (Sec. IV-C.1) */
#define GS_REC_FLOATS 12  /* floats per projected record (48 bytes, 16-byte aligned) */
#define GS_G2D 9          /* per-Gaussian 2D gradients: u v Sxx Sxy Syy o r g b (see gs_render_bwd_2d) */
#define GS_MLP_LATENT 16  /* learned-colour latent width */
#define GS_MLP_HIDDEN 64
#define GS_MLP_PARAMS 6467 /* 64*32 + 64 + 64*64 + 64 + 3*64 + 3 */

/* Pinhole camera.  Pixel (x, y) is sampled at (x + 0.5, y + 0.5); the
 * principal point is (cx, cy).  R_cw (row-major) and t_cw map world points
 * into the camera frame (x right, y down, z forward): t = R_cw mu + t_cw; this
 * is the viewing transform W of Sec. II-A.  Gaussians with camera depth
 * t_z <= near_z are culled.  tan_half_fov_* bound the image-plane slopes used
 * in the projective Jacobian J (clamped to 1.3x the half field of view).  bg is
 * the background colour added with the remaining transmittance. */
typedef struct {
  int32_t width, height;
  float fx, fy, cx, cy;
  float near_z;
  float tan_half_fov_x, tan_half_fov_y;
  float R_cw[9];
  float t_cw[3];
  float bg[3];
} gs_camera;

/* Gaussian set (Sec. II-A: centre mu, covariance Sigma from scale and
 * rotation, opacity, SH colour).  Device arrays, index fastest:
 *   means[3][n], log_scales[3][n]  (Sigma = R(q) diag(exp(s))^2 R(q)^T),
 *   quats[4][n] (w, x, y, z; normalised inside), logits[n] (o = sigmoid),
 *   sh[(D+1)^2][3][n] real SH coefficients, coefficient j / channel c at
 *   sh[(3j + c) n + i], D = sh_degree in 0..3 (colour_mode 0).
 * colour_mode 1 (learned colour decoder) replaces sh by latents (bf16 bit
 * patterns, [n][16], 16-byte aligned) and mlp (the decoder's packed operand
 * image written by gs_mlp_pack); sh_degree is ignored. */
typedef struct {
  int64_t n;
  int32_t sh_degree;
  int32_t colour_mode;
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* logits;
  const float* sh;
  const uint16_t* latents;
  const uint16_t* mlp;
} gs_gaussians;

/* Output of gs_project, input of the later stages.
 *   records[n][12]: u, v, A, B | C, opacity, r, g | b, depth, ex, ey
 *     (u, v) = projected centre in pixels, (A, B, C) = conic = inverse of the
 *     2D covariance Sigma' = J W Sigma W^T J^T + 0.3 I (Sec. II-A), opacity,
 *     colour (r, g, b).  One interleaved 48-byte record per Gaussian so that the
 *     per-tile gathers read whole records (the interleaved colour layout of
 *     Sec. V).  (ex, ey) are the half-extents of a box around (u, v) outside
 *     which alpha < 1/255 everywhere (with a small safety margin); the
 *     compositing kernels use it to skip whole waves of pixels.
 *   depth[n]: camera-space t_z (the sort key: Sec. II-A blends in depth order).
 *   radius[n]: ceil(3 sqrt(lambda_max(Sigma'))) pixels, 0 when culled.
 *   tiles_touched[n]: number of 16x16 tiles met by the square of half-width
 *     radius around (u, v), 0 when culled or off-screen.
 *   colour_grad[10][n] (optional, may be NULL; SH colour only): for the
 *     backward, the derivative of the colour with respect to the unit view
 *     direction (rows k = 3 ch + axis, 0..8) and in row 9 a bit mask stored
 *     in the float's bits: bit ch set when channel ch was not clamped at 0,
 *     bit 3 when the unclamped colour is finite.  When present gs_project
 *     writes it and the projection backward reads it instead of the 48 SH
 *     coefficients; when NULL the backward re-reads them. */
typedef struct {
  float* records;
  float* depth;
  int32_t* radius;
  uint32_t* tiles_touched;
  float* colour_grad;
} gs_projected;

/* Gradients with respect to the raw parameters, same layouts as gs_gaussians,
 * FP32.  For colour_mode 1, latents is float[n][16] and mlp float[GS_MLP_PARAMS];
 * pointers of the other mode must be NULL. */
typedef struct {
  float* means;
  float* log_scales;
  float* quats;
  float* logits;
  float* sh;
  float* latents;
  float* mlp;
} gs_gaussians_grad;

/* Message of the last failed call on this thread ("" if none). */
const char* gs_last_error(void);

/* Library version string. */
const char* gs_version(void);

/* Projection (Sec. II-A): per Gaussian, opacity, covariance from scale and
 * rotation, EWA projection Sigma' = J W Sigma W^T J^T with the first-order
 * pinhole Jacobian J plus a 0.3 px^2 low-pass dilation, conic with a
 * determinant guard, 3-sigma radius, tile count, and colour: real SH of degree
 * sh_degree evaluated at the unit camera-to-Gaussian direction, plus 0.5,
 * clamped at 0 (colour_mode 0), or the learned decoder (colour_mode 1).
 * Culled Gaussians (t_z <= near_z, non-finite values, det <= 0, radius above
 * 2^22) get a zero record, radius 0 and tiles_touched 0.
 * Errors: INVALID_ARG for n < 0, NULL arrays (when n > 0), sh_degree outside
 * 0..3, an unknown colour_mode, a non-positive or non-finite camera. */
gs_status gs_project(const gs_gaussians* g, const gs_camera* cam, gs_projected* out, gs_stream stream);

/* Workspace bytes for gs_bin_sort with n Gaussians and up to `capacity`
 * (tile, Gaussian) pairs.  Host-only; never touches the device. */
gs_status gs_bin_sort_workspace(int64_t n, int64_t capacity, const gs_camera* cam, size_t* bytes);

/* Tile binning and depth sort (Sec. II-A, front-to-back blending order;
 * Sec. IV-C.1, 16x16 tiles).  Every Gaussian emits one entry per tile its square meets; entries
 * are ordered by (tile, FP32 bit pattern of depth, Gaussian index), a total
 * order, so the result is unique and bit-reproducible.
 *   point_list[capacity]: Gaussian index of each entry, in that order.
 *   ranges[T][2]: [start, end) of tile t's entries (empty tiles get
 *     (S_t, S_t)), T = ceil(W/16) * ceil(H/16), tiles row-major.
 *   *k_out: number of entries K.
 * Synchronises `stream` once (to read K).  If K > capacity it returns
 * GS_ERR_CAPACITY with *k_out = K and point_list/ranges undefined; the caller
 * grows the buffers (and the workspace) and calls again.
 * ws must hold gs_bin_sort_workspace(n, capacity) bytes, 256-byte aligned. */
gs_status gs_bin_sort(int64_t n, const gs_projected* proj, const gs_camera* cam, void* ws, size_t ws_bytes,
                      uint32_t* point_list, int64_t capacity, uint32_t* ranges, int64_t* k_out,
                      gs_stream stream);

/* gs_bin_sort without the wait: the same lists, with K written to k_dev[0]
 * and the depth sort's look-back error flag to k_dev[1] (uint64 each, both in
 * stream order), so a caller can queue the rest of the frame at once and
 * check them later.  k_dev is device memory or pinned host memory that the
 * device can address (hipHostMalloc): the kernels store to it directly, and
 * the host reads it once the stream has passed the call (an event).  The lists are valid only if
 * k_dev[0] <= capacity and k_dev[1] == 0 (then they equal gs_bin_sort's);
 * otherwise they are undefined, no out-of-bounds access happens, and the
 * caller grows the buffers and redoes the frame.  Until it knows K the caller
 * passes `capacity` as k to gs_render_ckpt_floats, gs_render_fwd,
 * gs_render_bwd_workspace, gs_render_bwd and their _2d forms (an upper bound serves every
 * layout and launch there).  Only for frames of at most 16384 tiles (the
 * direct emission; gs_bin_sort takes a radix tile sort beyond); larger frames
 * return GS_ERR_UNSUPPORTED before any device work.
 * Other errors as gs_bin_sort. */
gs_status gs_bin_sort_async(int64_t n, const gs_projected* proj, const gs_camera* cam, void* ws, size_t ws_bytes,
                            uint32_t* point_list, int64_t capacity, uint32_t* ranges, uint64_t* k_dev,
                            gs_stream stream);

/* Work split of the compositing kernels (Sec. IV: workload imbalance between
 * dense and sparse tiles, adaptive merging of thread blocks).  PLAIN: one
 * workgroup per tile, tiles mapped so that neighbours share an XCD.
 * BALANCED: the backward gives every 256-entry batch of a tile's walk its
 * own workgroup -- (tile, batch) items planned on the device from the
 * largest n_contrib of each tile, which the forward leaves in t_ckpt -- and
 * starts each batch's walk from the forward's checkpoints at the batch end
 * (the transmittance and the per-batch colour sums, so the light behind is
 * a sum of non-negative terms); tiles with nothing to walk are skipped.  The
 * forward, which has no work count before it runs, stays PLAIN.  MERGED:
 * BALANCED plus light tiles (at most 64 entries to walk) merged four to a
 * workgroup, one wave per tile and four pixels per lane, in both directions.
 * Per-pixel arithmetic is the same in all three, so they give the same image
 * (bit for bit) and the same gradients up to rounding (order of the atomic
 * sums; the light behind from batch sums). */
#define GS_SCHEDULE_PLAIN 0
#define GS_SCHEDULE_BALANCED 1
#define GS_SCHEDULE_MERGED 2

/* Colour-hash sampling (Sec. IV-C.1, similarity-based sampling with colour
 * hashing): an APPROXIMATE mode of the compositing, selected by or-ing this
 * flag into the schedule argument of gs_render_fwd, gs_render_bwd and
 * gs_render_bwd_2d (the forward and its backward must both carry it).  Each
 * Gaussian's colour is quantised per channel to its 8-bit value
 * v8 = floor(255 clamp(c, 0, 1) + 1/2) (FP32) and then to 4 bits,
 * c_q = floor(v8 / 256 * 16); the bucket is R_q 256 + G_q 16 + B_q (4096
 * buckets).  In every 256-entry window of a tile's list (windows start at the
 * tile's first entry) the entries whose buckets agree form a group; a group of
 * two or more is composited as its front-most member with the members' mean
 * colour and the accumulated opacity 1 - prod (1 - o_j), and its other
 * members are not composited (groups of one are unchanged).  The backward
 * hands the gradient of a group's opacity and colour to its members by the
 * chain rule and the footprint's gradient to the representative.  Results
 * differ from the exact method; the image is still deterministic.  Needs
 * schedule PLAIN or BALANCED and, in the backward, deterministic = 0
 * (GS_ERR_UNSUPPORTED otherwise). */
#define GS_RENDER_COLOUR_HASH 0x100

/* Forward compositing (Sec. II-A, C = sum_i c_i alpha_i prod_{j<i} (1 - alpha_j)
 * over the tile's depth-ordered list).  Per pixel: power = -1/2 (A dx^2 +
 * C dy^2) - B dx dy, alpha = min(0.99, o exp(power)); entries with power > 0 or
 * alpha < 1/255 are skipped; the walk stops before an entry that would take
 * the transmittance below 1e-4.  Outputs image[3][H][W] = colour + T bg,
 * final_T[H][W] and n_contrib[H][W] (1 + position in the tile list of the last
 * blended entry, 0 if none).  t_ckpt (gs_render_ckpt_floats floats, or NULL
 * when no backward follows and schedule is PLAIN) receives every pixel's
 * transmittance at each 256-entry boundary of its tile list, which the
 * backward restarts from, the forward's tile plan and each tile's work count.
 * Deterministic. */
gs_status gs_render_fwd(int64_t n, const gs_projected* proj, const uint32_t* point_list, const uint32_t* ranges,
                        int64_t k, const gs_camera* cam, float* image, float* final_T, uint32_t* n_contrib,
                        float* t_ckpt, int32_t schedule, gs_stream stream);

/* Work counter for measurement: runs the forward's per-pixel decisions
 * without producing an image and writes counts[0] = pairs whose alpha is
 * evaluated before each pixel's walk ends, counts[1] = pairs blended (device
 * uint64[2], overwritten).  Sum over pixels of n_contrib is the number of
 * pairs the backward walks. */
gs_status gs_render_count(int64_t n, const gs_projected* proj, const uint32_t* point_list, const uint32_t* ranges,
                          int64_t k, const gs_camera* cam, uint64_t* counts, gs_stream stream);

/* The colour-hash sampling mode's bucket table for a binned frame (the
 * bucket-wise aggregation of Sec. IV-C.1, two-stage: each window's groups are
 * summed in LDS, then each group is added to the frame's table in device
 * memory), over every list entry:
 *   count[4096] (uint32, overwritten): list entries per bucket;
 *   sums[4096][4] (float, overwritten): sums of their colour (r, g, b) and
 *     opacity, so count and sums give each bucket's representative colour;
 *   bucket[k] (uint16): each list entry's bucket;
 *   rep[k] (uint32): list position of each entry's group representative (its
 *     own position for groups of one).
 * Any output may be NULL.  proj, point_list, ranges and k as for
 * gs_render_fwd.  count and bucket/rep are exact; the float sums depend on
 * the order of the device atomics. */
gs_status gs_colour_hash_table(int64_t n, const gs_projected* proj, const uint32_t* point_list,
                               const uint32_t* ranges, int64_t k, const gs_camera* cam, uint32_t* count,
                               float* sums, uint16_t* bucket, uint32_t* rep, gs_stream stream);

/* Floats of the transmittance checkpoint buffer for K entries. Host-only. */
gs_status gs_render_ckpt_floats(int64_t k, const gs_camera* cam, size_t* floats);

/* Per-Gaussian statistics that densification reads (the adaptive density
 * control of 3DGS that Sec. III builds on), accumulated by gs_render_bwd over
 * the views of an interval: grad_norm_sum[i] += |(dL/du, dL/dv)| of the view
 * (pixel units) and visible_count[i] += 1 for every view in which Gaussian i
 * meets at least one tile.  Device arrays [n], added to (never cleared by the
 * library). */
typedef struct {
  float* grad_norm_sum;
  uint32_t* visible_count;
} gs_densify_stats;

/* Workspace bytes for gs_render_bwd (depends on the Gaussian set's n and
 * colour mode, K and the camera). Host-only. */
gs_status gs_render_bwd_workspace(const gs_gaussians* g, int64_t k, const gs_camera* cam, int32_t deterministic,
                                  size_t* bytes);

/* Backward of the whole splatting step (Sec. II-A, the blending sum and the
 * EWA projection differentiated): dL/dimage -> gradients of the raw
 * parameters, the compositing backward followed by the projection backward in
 * one call.  The compositing part is the exact derivative of gs_render_fwd
 * with its skip/stop decisions held fixed: each pixel's list is walked back to
 * front from its n_contrib, the transmittance before each entry is recovered
 * by division from the forward's value at the end of the entry's 256-entry
 * batch (t_ckpt, or final_T for the last batch) -- never stored per pair --
 * and the light behind it is accumulated on the way.  The projection part
 * applies the chain rule through gs_project, recomputing its forward
 * quantities from the parameters.
 *   g, cam: the Gaussian set and camera of the forward; proj, point_list,
 *     ranges, k, final_T, n_contrib, t_ckpt: that forward's outputs (k as
 *     passed to gs_render_fwd); dL_dimage[3][H][W].
 *   grad: every array overwritten, same layouts as g (colour_mode 0: means,
 *     log_scales, quats, logits, sh; colour_mode 1: means, log_scales, quats,
 *     logits, latents [n][16] FP32 and mlp [GS_MLP_PARAMS] FP32 summed over
 *     Gaussians in a fixed order, plus the view direction's share of means).
 *     Culled Gaussians get zero gradients.
 *   stats: densification statistics to accumulate into, or NULL.
 *   deterministic = 1: no atomics, one partial per (tile, Gaussian) entry
 *     summed per Gaussian in the row-major order of its tile rectangle: the
 *     same bits on every run for a given schedule; 0: device atomics.
 *   schedule: as for gs_render_fwd (BALANCED plans from the work counts the
 *     forward left in t_ckpt).
 *   ws: gs_render_bwd_workspace bytes, 256-byte aligned, caller-owned.
 * Errors: INVALID_ARG for NULL arrays, bad sizes, an unknown schedule or a
 * small workspace (before any device work); HIP for launch failures. */
gs_status gs_render_bwd(const gs_gaussians* g, const gs_camera* cam, const gs_projected* proj,
                        const uint32_t* point_list, const uint32_t* ranges, int64_t k, const float* final_T,
                        const uint32_t* n_contrib, const float* t_ckpt, const float* dL_dimage,
                        gs_gaussians_grad* grad, gs_densify_stats* stats, void* ws, size_t ws_bytes,
                        int32_t deterministic, int32_t schedule, gs_stream stream);

/* The compositing half of gs_render_bwd on its own, stopping at the
 * per-Gaussian record gradients: g2d[9][n] (overwritten) =
 * dL/d(u, v, a, b, c, opacity, r, g, b), where Sigma' = [[a, b], [b, c]] is
 * the 2D covariance whose inverse is the record's conic (b counted in both
 * off-diagonal places).  Each pixel's conic gradient is carried to Sigma'
 * before the sum over pixels, which stays well conditioned where the conic is
 * nearly singular (elongated footprints).  Same decisions, arguments and
 * determinism as gs_render_bwd; ws as sized by gs_render_bwd_2d_workspace. */
gs_status gs_render_bwd_2d_workspace(int64_t n, int64_t k, const gs_camera* cam, int32_t deterministic,
                                     size_t* bytes);
gs_status gs_render_bwd_2d(int64_t n, const gs_projected* proj, const uint32_t* point_list, const uint32_t* ranges,
                           int64_t k, const gs_camera* cam, const float* final_T, const uint32_t* n_contrib,
                           const float* t_ckpt, const float* dL_dimage, float* g2d, void* ws, size_t ws_bytes,
                           int32_t deterministic, int32_t schedule, gs_stream stream);

/* The projection half of gs_render_bwd on its own: chain rule from g2d[9][n]
 * (the layout gs_render_bwd_2d writes) to the raw parameters through the
 * steps of gs_project (Sec. II-A, the EWA projection and the SH colour).
 * Every gradient array is overwritten; culled Gaussians get zero gradients.
 * colour_mode 1 (learned colour) instead fills grad->latents [n][16] FP32,
 * grad->mlp [GS_MLP_PARAMS] FP32 (summed over Gaussians in a fixed order) and
 * adds the view direction's share to grad->means; grad->sh may be NULL.  It
 * reads proj->radius (live = radius > 0, as in gs_project) and needs ws of
 * gs_project_bwd_workspace bytes; colour_mode 0 reads only proj->colour_grad
 * (proj may be NULL: the SH coefficients are then re-read) and ignores ws
 * (may be NULL / 0). */
gs_status gs_project_bwd_workspace(const gs_gaussians* g, size_t* bytes);
gs_status gs_project_bwd(const gs_gaussians* g, const gs_camera* cam, const gs_projected* proj, const float* g2d,
                         gs_gaussians_grad* grad, void* ws, size_t ws_bytes, gs_stream stream);

/* ------------------------------------------------------- optimiser step
 * Writable parameter arrays of a Gaussian set (same layouts as gs_gaussians);
 * also used for the Adam moments, which have the parameters' shapes. */
typedef struct {
  float* means;
  float* log_scales;
  float* quats;
  float* logits;
  float* sh;
} gs_param_arrays;

/* Adam hyper-parameters of a Gaussian set: one learning rate per parameter
 * group (the SH coefficients split into the degree-0 term and the rest),
 * shared moments decay rates, epsilon, and the step number (from 1). */
typedef struct {
  float lr_means, lr_log_scales, lr_quats, lr_logits, lr_sh_dc, lr_sh_rest;
  float beta1, beta2, eps;
  int32_t step;
} gs_adam_config;

/* One Adam step (bias-corrected) over every parameter array of a Gaussian set
 * in one launch -- the optimiser step that follows gs_render_bwd in training:
 *   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
 *   p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps)
 * with the group's lr.  params, m and v are updated in place; grad as written
 * by gs_render_bwd (colour_mode 0 fields).  n Gaussians, SH degree in 0..3.
 * Errors: INVALID_ARG for NULL arrays, step < 1, betas outside [0, 1),
 * eps <= 0 or a non-finite learning rate. */
gs_status gs_adam_gaussians(int64_t n, int32_t sh_degree, const gs_param_arrays* params, const gs_gaussians_grad* grad,
                            const gs_param_arrays* m, const gs_param_arrays* v, const gs_adam_config* cfg,
                            gs_stream stream);

/* ------------------------------------------------------- density control
 * Workload-sensitive density control (Sec. III-C), one round per call: each
 * Gaussian's local density rho = number of other centres within `radius`
 * (the decision d^2 <= r^2 taken in FP32, each operation rounded), the
 * thresholds rho_low = mu - alpha sigma and rho_high = mu + beta sigma over all
 * densities (population statistics in FP64 from the exact integer sums), the
 * mean distance d_bar to the `knn` nearest other centres (nearest by FP32
 * squared distance, then index), then
 *   - densification: every Gaussian with rho < rho_low gets a new neighbour at
 *     p + (spread d_bar) z + jitter e, with z and e the Gaussian's rows of
 *     noise[6][n] (z ~ N(0, I3) in rows 0-2, e ~ U(-1, 1)^3 in rows 3-5, drawn
 *     by the caller), its other parameters copied from it;
 *   - merging: two Gaussians with rho > rho_high that are each other's nearest
 *     neighbour within d_merge = mu_d + gamma sigma_d (statistics of every
 *     Gaussian's nearest-neighbour distance) become one at the lower index:
 *     opacity-weighted mean position and SH coefficients, scales the mean of
 *     the two scales (log of the mean of exp(log_scale) per axis), opacity
 *     1 - (1 - o_i)(1 - o_j), the more opaque one's rotation.
 * The output holds the surviving Gaussians in index order, then the new ones
 * in the order of the Gaussians that spawned them. */
typedef struct {
  float radius;           /* r > 0 */
  float alpha, beta;      /* threshold factors >= 0 (the paper's example: 1, 1) */
  int32_t knn;            /* k in 1..8 */
  float spread;           /* a > 1: sigma_p = a d_bar */
  float jitter;           /* half-width of the uniform perturbation, >= 0 */
  float gamma;            /* merge-radius factor (the paper's example: 1) */
} gs_density_params;

/* Filled on return (also on GS_ERR_CAPACITY). */
typedef struct {
  int64_t n_in, n_merged, n_new, n_out;        /* n_out = n_in - n_merged + n_new */
  double rho_mean, rho_std, rho_low, rho_high;
  double d_mean, d_std, d_merge;
} gs_density_report;

/* Optional per-Gaussian outputs of a round (any pointer may be NULL):
 * rho[n], cls[n] (0 neither, 1 below rho_low, 2 above rho_high), nn[n]
 * (nearest other Gaussian, -1 if none), dbar[n], fate[n] (output index, -1
 * if merged away). */
typedef struct {
  int32_t* rho;
  uint8_t* cls;
  int32_t* nn;
  float* dbar;
  int32_t* fate;
} gs_density_points;

/* Workspace bytes for n Gaussians. Host-only. */
gs_status gs_density_control_workspace(int64_t n, size_t* bytes);

/* One round on g (colour_mode 0; n <= 2^30) into out (same layouts as
 * gs_gaussians with `capacity` in place of n: means[3][capacity], ...).
 * Synchronises the stream once to read the counts.  Errors: INVALID_ARG for
 * bad parameters or NULL arrays; CAPACITY when n_out > capacity (report->n_out
 * holds the size needed; outputs past the capacity are not written);
 * UNSUPPORTED when a coordinate is not finite or lies 2^18 cells (of 1.07 r)
 * or more from the origin (the grid's FP32 cell guarantees need less). */
gs_status gs_density_control(const gs_gaussians* g, const gs_density_params* prm, const float* noise,
                             gs_param_arrays* out, int64_t capacity, void* ws, size_t ws_bytes,
                             gs_density_report* report, gs_density_points* points, gs_stream stream);

/* ---------------------------------------------------------- learned colour
 * Optional decoder that replaces the SH colour read (not part of the paper):
 * per sample, x = [z (16 BF16 latent values); Y_0..15(d)] with Y the real SH
 * basis of degree 3 at the unit view direction d, then
 *   h1 = ReLU(W1 x + b1) (64), h2 = ReLU(W2 h1 + b2) (64), c = sigmoid(W3 h2 + b3).
 * Weights are BF16 (GS_MLP_PARAMS values, row-major, in the order W1[64][32],
 * b1[64], W2[64][64], b2[64], W3[3][64], b3[3]); products run on the BF16
 * matrix cores with FP32 accumulation; the SH encoding and the hidden
 * activations enter them as a pair of BF16 values (hi + lo, about 2^-17
 * relative), so colours match the BF16-weight definition to near FP32
 * accuracy.  In the backward, gradients entering products and the activations
 * of the weight-gradient products are single BF16 values. */
#define GS_MLP_PACKED_BYTES 31244

/* Lay the BF16 parameters out as the matrix-core operand image used by every
 * decoder kernel (GS_MLP_PACKED_BYTES bytes of device memory, 16-byte
 * aligned).  Call again whenever the parameters change. */
gs_status gs_mlp_pack(const uint16_t* params_bf16, void* packed, gs_stream stream);

/* Decoder colours rgb[S][3] of S samples: sample s uses latent s / per
 * (latents bf16 [S/per][16]) and the unit direction dirs[s][3]. */
gs_status gs_mlp_fwd(int64_t S, int32_t per, const uint16_t* latents, const float* dirs, const void* packed,
                     float* rgb, gs_stream stream);

/* Workspace bytes of gs_mlp_bwd for S samples at `per` samples per latent. */
gs_status gs_mlp_bwd_workspace(int64_t S, int32_t per, size_t* bytes);

/* Backward of gs_mlp_fwd over the same samples (S a multiple of per, per a
 * power of two up to 4096).  dL/drgb comes from dL_drgb[S][3], or, when
 * dL_drgb is NULL, from the distillation loss
 *   L = scale * sum_s |rgb_s - target_s|^2           (target[S][3])
 * whose value goes to *loss (device scalar, may be NULL).  Outputs (FP32,
 * overwritten): dlatents[S/per][16] and dparams[GS_MLP_PARAMS] in the
 * parameter order of gs_mlp_pack.  Weight and latent gradients are summed in
 * a fixed order: bit-reproducible for a given S.  The forward is recomputed
 * (the same BF16 roundings as gs_mlp_fwd); products run on the BF16 matrix
 * cores with FP32 accumulation. */
gs_status gs_mlp_bwd(int64_t S, int32_t per, const uint16_t* latents, const float* dirs, const void* packed,
                     const float* dL_drgb, const float* target, float scale, float* dlatents, float* dparams,
                     float* loss, void* ws, size_t ws_bytes, gs_stream stream);

/* SH colour of Gaussian s / per at the unit direction dirs[s][3]: the colour
 * rule of gs_project (Sec. I, colour from SH coefficients; real basis, +0.5,
 * clamped at 0), clamped to at most 1 as well if clamp01 != 0.  sh as in
 * gs_gaussians ((deg+1)^2 x 3 x n).  The distillation target of the decoder. */
gs_status gs_sh_colour(int64_t S, int32_t per, int64_t n, int32_t sh_degree, const float* sh, const float* dirs,
                       int32_t clamp01, float* rgb, gs_stream stream);

/* One Adam step (bias-corrected, step counted from 1) on n FP32 values:
 *   m = b1 m + (1-b1) g,  v = b2 v + (1-b2) g^2,
 *   p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps),
 * and, if param_bf16 != NULL, its BF16 copy (round to nearest even). */
gs_status gs_adam_step(int64_t n, float* param, const float* grad, float* m, float* v, uint16_t* param_bf16,
                       float lr, float beta1, float beta2, float eps, int32_t step, gs_stream stream);

/* L1 photometric loss over `count` floats: *loss = mean |img - target| (device
 * scalar) and, if grad != NULL, grad = sign(img - target) / count.  partials
 * is caller scratch of GS_L1_PARTIALS floats.  The sum is taken in a fixed
 * order, so the loss is deterministic. */
#define GS_L1_PARTIALS 1024
gs_status gs_l1_loss(const float* img, const float* target, int64_t count, float* loss, float* grad,
                     float* partials, gs_stream stream);

/* gs_l1_loss without caller scratch and without any allocation, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  The partial sums live in
 * a file-scope device array of GS_L1_STATIC_PARTIALS floats (4 KiB), one copy
 * per GPU, held until the process ends; its address is looked up on the first
 * call on each device (with that device current).  Every partial-sum slot is
 * written before it is read, so nothing needs clearing between calls.  The
 * partial sums number min(GS_L1_PARTIALS, ceil(count / 256)), which never
 * exceeds the array (GS_ERR_CAPACITY otherwise), so any count > 0 is taken.
 * Calls that overlap on one GPU (other streams, other threads) share the array
 * and race: serialise them.  Same arguments, result and errors as gs_l1_loss
 * otherwise; GS_ERR_UNSUPPORTED for a device index above 63. */
#define GS_L1_STATIC_PARTIALS 1024
gs_status gs_l1_loss_static(const float* img, const float* target, int64_t count, float* loss, float* grad,
                            gs_stream stream);

/* ------------------------------------------------------------ measurement
 * Kernel timer (for benchmarks; not needed by the path).  After
 * gs_kernel_timer_start, every kernel the library launches is bracketed by
 * two HIP events recorded on its launch stream, until gs_kernel_timer_stop, which waits for those events and writes one line per
 * kernel name, "name launches total_ms", in first-launch order, into buf
 * (size bytes, truncated and NUL-terminated; *needed = the full length + 1;
 * buf may be NULL to query the length).  One timer per process: launches
 * from every host thread are timed (an autograd backward runs on a thread of
 * its own); the events add a few microseconds per launch.  Errors:
 * INVALID_ARG when no timer (start: a timer) is running; HIP if an event
 * failed. */
gs_status gs_kernel_timer_start(void);
gs_status gs_kernel_timer_stop(char* buf, size_t size, size_t* needed);

#ifdef __cplusplus
}
#endif

#endif /* GSPLAT_MI355_H */
