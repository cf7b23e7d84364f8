// Front-to-back compositing over per-tile depth-ordered lists, and its backward.
//
// Paper: Sec. II-A, C = sum_i c_i alpha_i prod_{j<i} (1 - alpha_j) over the
// Gaussians reaching a pixel in depth order, with alpha from the projected
// Gaussian G(x) and the opacity; Sec. IV-C.1, 16x16 pixel tiles sharing one
// list; Sec. V, interleaved per-Gaussian records loaded in batches into fast
// on-chip memory.
//
// One 256-thread workgroup per tile, one pixel per thread (a wave64 covers 4
// rows of 16 pixels).  The tile's records are gathered in batches of 256 into
// LDS (one 48-byte record per thread, three 16-byte loads) and every lane
// reads them back as broadcasts.  The per-pair body is branch-free; a wave
// leaves a batch as soon as all its lanes are done (ballot), and the workgroup
// leaves the tile when all 256 pixels are done.  Tiles are mapped so that
// neighbouring tiles run on the same XCD and share its L2.
//
// This file is compiled with -ffp-contract=off: the forward and the backward
// evaluate alpha through the same inline function with explicit fmaf, so the
// backward re-derives exactly the forward's skip decisions and transmittances.
#include "gs_internal.h"

namespace gs {

constexpr int kBatch = 256;

// Records are staged in LDS with the conic pre-scaled so that
// power = a dx^2 + b dx dy + c dy^2:  p = (u, v, a = -A/2, b = -B),
// q = (c = -C/2, opacity, r, g), blue separately.
__device__ __forceinline__ void stage_record(const float4* __restrict__ rec, uint32_t gid, float4& p, float4& q,
                                             float& blue) {
  const float4 r0 = rec[3 * gid];
  const float4 r1 = rec[3 * gid + 1];
  const float4 r2 = rec[3 * gid + 2];
  p = make_float4(r0.x, r0.y, -0.5f * r0.z, -r0.w);
  q = make_float4(-0.5f * r1.x, r1.y, r1.z, r1.w);
  blue = r2.x;
}

// Transmittance checkpoints: the forward stores every pixel's T at the start of
// each 256-entry batch b >= 1 of its tile, in slot floor(S_t / 256) + t + b
// (S_t = first entry of tile t).  Slots of different tiles never collide and
// all are below floor(K / 256) + T + 1.
__device__ __forceinline__ size_t ckpt_slot0(uint32_t start, int tile) {
  return static_cast<size_t>(start / kBatch) + static_cast<size_t>(tile);
}

// power, e^power and the unclamped o e^power for one (pixel, entry) pair.
__device__ __forceinline__ void eval_pair(const float4& p, const float4& q, float px, float py, float& dx,
                                          float& dy, float& power, float& eg, float& og) {
  dx = p.x - px;
  dy = p.y - py;
  const float dxx = dx * dx, dyy = dy * dy, dxy = dx * dy;
  power = fmaf(p.z, dxx, fmaf(q.x, dyy, p.w * dxy));
  eg = __expf(power);
  og = q.y * eg;
}

// ------------------------------------------------------------------- forward

__global__ __launch_bounds__(256) void k_render_fwd(const uint2* __restrict__ ranges,
                                                    const uint32_t* __restrict__ point_list,
                                                    const float4* __restrict__ rec, DevCam cam,
                                                    float* __restrict__ image, float* __restrict__ final_T,
                                                    uint32_t* __restrict__ n_contrib, float* __restrict__ t_ckpt) {
  __shared__ float4 s_p[kBatch];
  __shared__ float4 s_q[kBatch];
  __shared__ float s_b[kBatch];
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
  const int px_i = tx * kTile + (threadIdx.x & 15);
  const int py_i = ty * kTile + (threadIdx.x >> 4);
  const bool inside = px_i < cam.width && py_i < cam.height;
  const float px = static_cast<float>(px_i) + 0.5f, py = static_cast<float>(py_i) + 0.5f;
  const uint2 rg = ranges[tile];

  float T = 1.0f, acc0 = 0.0f, acc1 = 0.0f, acc2 = 0.0f;
  uint32_t contrib = 0;
  bool done = !inside;
  const size_t slot0 = ckpt_slot0(rg.x, tile);

  for (uint32_t base = rg.x, b = 0; base < rg.y; base += kBatch, ++b) {
    if (__syncthreads_count(done) == 256) break;
    if (b > 0 && t_ckpt) t_ckpt[(slot0 + b) * kBatch + threadIdx.x] = T;
    const uint32_t idx = base + threadIdx.x;
    if (idx < rg.y) {
      float4 p, q;
      float b;
      stage_record(rec, point_list[idx], p, q, b);
      s_p[threadIdx.x] = p;
      s_q[threadIdx.x] = q;
      s_b[threadIdx.x] = b;
    }
    __syncthreads();
    const int cnt = static_cast<int>(min(static_cast<uint32_t>(kBatch), rg.y - base));
    for (int j = 0; j < cnt; ++j) {
      if (__ballot(!done) == 0) break;  // whole wave finished: leave the batch
      const float4 p = s_p[j];
      const float4 q = s_q[j];
      float dx, dy, power, eg, og;
      eval_pair(p, q, px, py, dx, dy, power, eg, og);
      const float alpha = fminf(kAlphaMax, og);
      const bool ok = !done && (power <= 0.0f) && (alpha >= kAlphaMin);
      const float Tn = T * (1.0f - alpha);
      const bool stop = ok && (Tn < kTMin);
      const bool blend = ok && !stop;
      const float w = blend ? alpha * T : 0.0f;
      acc0 = fmaf(q.z, w, acc0);
      acc1 = fmaf(q.w, w, acc1);
      acc2 = fmaf(s_b[j], w, acc2);
      T = blend ? Tn : T;
      contrib = blend ? (base + static_cast<uint32_t>(j) - rg.x + 1u) : contrib;
      done = done || stop;
    }
  }
  if (inside) {
    const int64_t HW = static_cast<int64_t>(cam.width) * cam.height;
    const int64_t pix = static_cast<int64_t>(py_i) * cam.width + px_i;
    image[pix] = fmaf(T, cam.bg[0], acc0);
    image[HW + pix] = fmaf(T, cam.bg[1], acc1);
    image[2 * HW + pix] = fmaf(T, cam.bg[2], acc2);
    final_T[pix] = T;
    n_contrib[pix] = contrib;
  }
}

gs_status launch_render_fwd(const gs_projected& proj, const uint32_t* point_list, const uint32_t* ranges,
                            const DevCam& cam, float* image, float* final_T, uint32_t* n_contrib, float* t_ckpt,
                            hipStream_t s) {
  const int ntiles = cam.tiles_x * cam.tiles_y;
  k_render_fwd<<<ntiles, 256, 0, s>>>(reinterpret_cast<const uint2*>(ranges), point_list,
                                      reinterpret_cast<const float4*>(proj.records), cam, image, final_T, n_contrib,
                                      t_ckpt);
  return check_launch("k_render_fwd");
}

// ------------------------------------------------------------------ backward

// Sum over the 64 lanes of a wave with DPP; the total lands in lane 63.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_src(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}

__device__ __forceinline__ float wave_sum_to_lane63(float v) {
  v += dpp_src<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_src<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_src<0x124, 0xF>(v);  // row_ror:4
  v += dpp_src<0x128, 0xF>(v);  // row_ror:8
  v += dpp_src<0x142, 0xA>(v);  // row_bcast:15 into rows 1, 3
  v += dpp_src<0x143, 0xC>(v);  // row_bcast:31 into rows 2, 3
  return v;
}

__device__ __forceinline__ float lane63(float v) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wave_sum_to_lane63(v)), 63));
}

// Per (pixel, entry) derivative, walked back to front.  Starting from S =
// T_f bg, each blended entry m (going backwards) recovers T_m = T_{m+1} /
// (1 - alpha_m) and uses the light behind it, S_m = sum_{j>m} c_j alpha_j T_j +
// T_f bg, accumulated directly:
//   dL/dalpha_m = sum_k G_k (c_k T_m - S_mk / (1 - alpha_m)),  S += c_m alpha_m T_m.
// Accumulating S (instead of subtracting from the pixel value) keeps its
// rounding error relative to S itself.  T restarts at every batch end from the
// forward's checkpoint (or T_f for the last batch), so the division walks at
// most 256 entries and its rounding cannot build up along long lists.  Skips
// are re-derived from the same alpha evaluation as the forward; entries past
// n_contrib are never touched.
__global__ __launch_bounds__(256) void k_render_bwd(const uint2* __restrict__ ranges,
                                                    const uint32_t* __restrict__ point_list,
                                                    const float4* __restrict__ rec, DevCam cam,
                                                    const float* __restrict__ final_T,
                                                    const uint32_t* __restrict__ n_contrib,
                                                    const float* __restrict__ t_ckpt,
                                                    const float* __restrict__ dL_dimage, int n,
                                                    float* __restrict__ g2d) {
  __shared__ float4 s_p[kBatch];
  __shared__ float4 s_q[kBatch];
  __shared__ float s_b[kBatch];
  __shared__ uint32_t s_gid[kBatch];
  __shared__ uint32_t s_max;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
  const int px_i = tx * kTile + (threadIdx.x & 15);
  const int py_i = ty * kTile + (threadIdx.x >> 4);
  const bool inside = px_i < cam.width && py_i < cam.height;
  const float px = static_cast<float>(px_i) + 0.5f, py = static_cast<float>(py_i) + 0.5f;
  const uint2 rg = ranges[tile];
  const int lane = threadIdx.x & 63;

  float G0 = 0.f, G1 = 0.f, G2 = 0.f, T = 1.0f;
  uint32_t ncon = 0;
  if (inside) {
    const int64_t HW = static_cast<int64_t>(cam.width) * cam.height;
    const int64_t pix = static_cast<int64_t>(py_i) * cam.width + px_i;
    G0 = dL_dimage[pix]; G1 = dL_dimage[HW + pix]; G2 = dL_dimage[2 * HW + pix];
    T = final_T[pix];
    ncon = n_contrib[pix];
  }
  const float T_final = T;
  const size_t slot0 = ckpt_slot0(rg.x, tile);
  float S0 = T * cam.bg[0], S1 = T * cam.bg[1], S2 = T * cam.bg[2];
  if (threadIdx.x == 0) s_max = 0;
  __syncthreads();
  if (ncon) atomicMax(&s_max, ncon);
  __syncthreads();
  const uint32_t len = min(rg.y - rg.x, s_max);  // n_contrib never exceeds the list
  const int nbatch = static_cast<int>((len + kBatch - 1) / kBatch);

  for (int bi = nbatch - 1; bi >= 0; --bi) {
    const uint32_t m0 = static_cast<uint32_t>(bi) * kBatch;
    const int cnt = static_cast<int>(min(static_cast<uint32_t>(kBatch), len - m0));
    T = (bi + 1 < nbatch) ? t_ckpt[(slot0 + bi + 1) * kBatch + threadIdx.x] : T_final;
    __syncthreads();
    if (threadIdx.x < cnt) {
      const uint32_t gid = point_list[rg.x + m0 + threadIdx.x];
      float4 p, q;
      float b;
      stage_record(rec, gid, p, q, b);
      s_p[threadIdx.x] = p;
      s_q[threadIdx.x] = q;
      s_b[threadIdx.x] = b;
      s_gid[threadIdx.x] = gid;
    }
    __syncthreads();
    for (int j = cnt - 1; j >= 0; --j) {
      const uint32_t m = m0 + static_cast<uint32_t>(j);
      if (__ballot(m < ncon) == 0) continue;  // no lane of this wave reaches entry m yet
      const float4 p = s_p[j];
      const float4 q = s_q[j];
      const float cb = s_b[j];
      float dx, dy, power, eg, og;
      eval_pair(p, q, px, py, dx, dy, power, eg, og);
      const float alpha = fminf(kAlphaMax, og);
      const bool ok = (m < ncon) && (power <= 0.0f) && (alpha >= kAlphaMin);
      if (__ballot(ok) == 0) continue;
      const float inv = 1.0f / (1.0f - alpha);
      const float Tm = ok ? T * inv : T;
      const float dalpha = G0 * (q.z * Tm - S0 * inv) + G1 * (q.w * Tm - S1 * inv) + G2 * (cb * Tm - S2 * inv);
      const float w = ok ? alpha * Tm : 0.0f;
      S0 = fmaf(q.z, w, S0);
      S1 = fmaf(q.w, w, S1);
      S2 = fmaf(cb, w, S2);
      T = Tm;
      const bool unclamped = og < kAlphaMax;
      const float dpow = (ok && unclamped) ? alpha * dalpha : 0.0f;
      const float dop = (ok && unclamped) ? eg * dalpha : 0.0f;
      // power = a dx^2 + b dx dy + c dy^2 with a = -A/2, b = -B, c = -C/2, so
      // (nkx, nky) = -K d with K the conic and d = (dx, dy).  The pair's conic
      // gradient -1/2 dpow d d^T is carried to Sigma' = K^-1 right here,
      // -K (.) K = 1/2 dpow (K d)(K d)^T, before any summation: converting the
      // summed conic gradient instead cancels badly for elongated footprints.
      const float nkx = 2.0f * p.z * dx + p.w * dy;
      const float nky = p.w * dx + 2.0f * q.x * dy;
      const float du = dpow * nkx;
      const float dv = dpow * nky;
      const float hdp = 0.5f * dpow;
      const float dA = hdp * nkx * nkx;      // dL/dSigma'_xx
      const float dB = dpow * nkx * nky;     // dL/dSigma'_xy (both off-diagonal entries)
      const float dC = hdp * nky * nky;      // dL/dSigma'_yy
      const float dr = G0 * w, dg = G1 * w, db = G2 * w;
      const float s0 = lane63(du), s1 = lane63(dv), s2 = lane63(dA), s3 = lane63(dB), s4 = lane63(dC);
      const float s5 = lane63(dop), s6 = lane63(dr), s7 = lane63(dg), s8 = lane63(db);
      if (lane == 0) {
        const uint32_t gid = s_gid[j];
        unsafeAtomicAdd(&g2d[0 * static_cast<int64_t>(n) + gid], s0);
        unsafeAtomicAdd(&g2d[1 * static_cast<int64_t>(n) + gid], s1);
        unsafeAtomicAdd(&g2d[2 * static_cast<int64_t>(n) + gid], s2);
        unsafeAtomicAdd(&g2d[3 * static_cast<int64_t>(n) + gid], s3);
        unsafeAtomicAdd(&g2d[4 * static_cast<int64_t>(n) + gid], s4);
        unsafeAtomicAdd(&g2d[5 * static_cast<int64_t>(n) + gid], s5);
        unsafeAtomicAdd(&g2d[6 * static_cast<int64_t>(n) + gid], s6);
        unsafeAtomicAdd(&g2d[7 * static_cast<int64_t>(n) + gid], s7);
        unsafeAtomicAdd(&g2d[8 * static_cast<int64_t>(n) + gid], s8);
      }
    }
  }
}

size_t render_bwd_workspace(int64_t n, int64_t k, int ntiles, int deterministic) {
  (void)n; (void)k; (void)ntiles; (void)deterministic;
  return 256;
}

gs_status launch_render_bwd(int64_t n, const gs_projected& proj, const uint32_t* point_list, const uint32_t* ranges,
                            int64_t k, const DevCam& cam, const float* final_T,
                            const uint32_t* n_contrib, const float* t_ckpt, const float* dL_dimage, float* g2d, void* ws,
                            size_t ws_bytes, int deterministic, hipStream_t s) {
  (void)k; (void)ws; (void)ws_bytes;
  if (deterministic) return fail(GS_ERR_UNSUPPORTED, "gs_render_bwd: deterministic reduction not built yet");
  gs_status st = check_hip(hipMemsetAsync(g2d, 0, sizeof(float) * GS_G2D * static_cast<size_t>(n), s),
                           "hipMemsetAsync(g2d)");
  if (st != GS_OK) return st;
  const int ntiles = cam.tiles_x * cam.tiles_y;
  k_render_bwd<<<ntiles, 256, 0, s>>>(reinterpret_cast<const uint2*>(ranges), point_list,
                                      reinterpret_cast<const float4*>(proj.records), cam, final_T, n_contrib,
                                      t_ckpt, dL_dimage, static_cast<int>(n), g2d);
  return check_launch("k_render_bwd");
}

}  // namespace gs
