// Projection of 3D Gaussians to 2D conics with SH colour, and its backward.
//
// Paper: Sec. II-A -- the Gaussian kernel G(x), the EWA projection
// Sigma' = J W Sigma W^T J^T and colour from SH coefficients.  One thread per
// Gaussian; parameters are structure-of-arrays so a wave reads 64 consecutive
// floats per field (256-byte coalesced loads).  The kernel is HBM-bound: it
// reads 44 + 12 (D+1)^2 bytes and writes 60 bytes per Gaussian, plus the 40
// bytes of the colour gradient when the backward asks for it.
#include "gs_internal.h"
#include "gs_sh.h"

namespace gs {

// Geometry of one Gaussian, shared by the forward and the backward so both
// see the same FP32 values.
struct Geo {
  float o;
  float qn[4], qinv;       // unit quaternion and 1/|q|
  float R[9], S[3];        // rotation, scales
  float Sig[6];            // 3D covariance xx xy xz yy yz zz
  float t[3];              // camera-space centre
  float sx, sy;            // (possibly clamped) slopes
  bool clx, cly;
  float T[6];              // J W, 2x3 row-major
  float a, b, c;           // Sigma' (dilated)
  float det, A, B, C;
  int radius;
  float u, v;
};

// Returns false if the Gaussian is culled.
__device__ __forceinline__ bool project_geometry(const float m[3], const float s[3], const float q[4], float logit,
                                                 const DevCam& cam, Geo& g) {
  g.o = 1.0f / (1.0f + expf(-logit));
  const float qq = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
  const float qlen = sqrtf(qq);
  g.qinv = 1.0f / qlen;
  const float w = q[0] * g.qinv, x = q[1] * g.qinv, y = q[2] * g.qinv, z = q[3] * g.qinv;
  g.qn[0] = w; g.qn[1] = x; g.qn[2] = y; g.qn[3] = z;
  float* R = g.R;
  R[0] = 1.0f - 2.0f * (y * y + z * z); R[1] = 2.0f * (x * y - w * z);        R[2] = 2.0f * (x * z + w * y);
  R[3] = 2.0f * (x * y + w * z);        R[4] = 1.0f - 2.0f * (x * x + z * z); R[5] = 2.0f * (y * z - w * x);
  R[6] = 2.0f * (x * z - w * y);        R[7] = 2.0f * (y * z + w * x);        R[8] = 1.0f - 2.0f * (x * x + y * y);
  g.S[0] = expf(s[0]); g.S[1] = expf(s[1]); g.S[2] = expf(s[2]);
  // M = R S ; Sigma = M M^T
  float M[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) M[3 * i + j] = R[3 * i + j] * g.S[j];
  g.Sig[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
  g.Sig[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
  g.Sig[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
  g.Sig[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
  g.Sig[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
  g.Sig[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
  const float* W = cam.R;
#pragma unroll
  for (int i = 0; i < 3; ++i) g.t[i] = W[3 * i] * m[0] + W[3 * i + 1] * m[1] + W[3 * i + 2] * m[2] + cam.t[i];
  const float tz = g.t[2];
  if (!(tz > cam.near_z) || !isfinite(tz)) return false;
  const float itz = 1.0f / tz;
  const float rx = g.t[0] * itz, ry = g.t[1] * itz;
  g.sx = fminf(fmaxf(rx, -cam.lim_x), cam.lim_x);
  g.sy = fminf(fmaxf(ry, -cam.lim_y), cam.lim_y);
  g.clx = (rx > cam.lim_x) || (rx < -cam.lim_x);
  g.cly = (ry > cam.lim_y) || (ry < -cam.lim_y);
  // J = [[fx/tz, 0, -fx sx/tz], [0, fy/tz, -fy sy/tz]];  T = J W
  const float j00 = cam.fx * itz, j02 = -cam.fx * g.sx * itz;
  const float j11 = cam.fy * itz, j12 = -cam.fy * g.sy * itz;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    g.T[k] = j00 * W[k] + j02 * W[6 + k];
    g.T[3 + k] = j11 * W[3 + k] + j12 * W[6 + k];
  }
  // Sigma' = T Sigma T^T (symmetric Sigma stored as 6 values)
  const float* Sg = g.Sig;
  float P0[3], P1[3];  // T Sigma rows
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const float* Tr = g.T + 3 * r;
    float* P = r ? P1 : P0;
    P[0] = Tr[0] * Sg[0] + Tr[1] * Sg[1] + Tr[2] * Sg[2];
    P[1] = Tr[0] * Sg[1] + Tr[1] * Sg[3] + Tr[2] * Sg[4];
    P[2] = Tr[0] * Sg[2] + Tr[1] * Sg[4] + Tr[2] * Sg[5];
  }
  g.a = P0[0] * g.T[0] + P0[1] * g.T[1] + P0[2] * g.T[2] + kDilation;
  g.b = P0[0] * g.T[3] + P0[1] * g.T[4] + P0[2] * g.T[5];
  g.c = P1[0] * g.T[3] + P1[1] * g.T[4] + P1[2] * g.T[5] + kDilation;
  g.det = fmaf(g.a, g.c, -g.b * g.b);
  if (!(g.det > 0.0f) || !isfinite(g.det)) return false;
  const float idet = 1.0f / g.det;
  g.A = g.c * idet; g.B = -g.b * idet; g.C = g.a * idet;
  // largest eigenvalue: mid + sqrt(max(0.1, ((a-c)/2)^2 + b^2)), cancellation-free
  const float mid = 0.5f * (g.a + g.c);
  const float h = 0.5f * (g.a - g.c);
  const float lam = mid + sqrtf(fmaxf(0.1f, h * h + g.b * g.b));
  const float r3 = 3.0f * sqrtf(lam);
  if (!(r3 <= kRadiusMax)) return false;
  g.radius = static_cast<int>(ceilf(r3));
  g.u = cam.fx * g.t[0] * itz + cam.cx;
  g.v = cam.fy * g.t[1] * itz + cam.cy;
  return isfinite(g.u) && isfinite(g.v) && isfinite(g.A) && isfinite(g.B) && isfinite(g.C) && isfinite(g.o);
}

// Half-extents of the axis-aligned box around (u, v) outside which alpha is
// below 1/255 at every point: alpha >= 1/255 needs d^T Sigma'^-1 d <= rho^2 =
// 2 ln(255 o), an ellipse whose x and y half-extents are rho sqrt(Sigma'_xx)
// and rho sqrt(Sigma'_yy).  The FP32 conic's quadratic form may differ from
// the exact one by about 2 eps cond(Sigma') relative, so rho^2 gets 2 %
// (covering cond up to 1e5) plus 2e-4 of slack and the extents 1e-3 px plus
// 1e-6 |u| (rounding of pixel offsets): a pair whose pixel lies outside the
// box is skipped by the per-pixel test anyway, so compositing may skip it
// earlier without changing any result.  Footprints with cond above 1e5 get an
// unbounded box; a Gaussian that can never reach 1/255 gets (-1, -1).
__device__ __forceinline__ void alpha_support(const Geo& g, float& ex, float& ey) {
  const float lo = logf(255.0f * g.o);
  if (!(lo > 0.0f)) { ex = -1.0f; ey = -1.0f; return; }
  const float mid = 0.5f * (g.a + g.c);
  const float h = 0.5f * (g.a - g.c);
  const float disc = sqrtf(h * h + g.b * g.b);
  if (!((mid - disc) * 1e5f > mid + disc)) { ex = 3.0e38f; ey = 3.0e38f; return; }
  const float rho2 = 2.0f * lo * 1.02f + 2e-4f;
  ex = sqrtf(rho2 * g.a) + 1e-3f + 1e-6f * fabsf(g.u);
  ey = sqrtf(rho2 * g.c) + 1e-3f + 1e-6f * fabsf(g.v);
}


constexpr int kProjThreads = 256;

template <int DEG>
__global__ __launch_bounds__(kProjThreads) void k_project(int n, const float* __restrict__ means,
                                                 const float* __restrict__ log_scales,
                                                 const float* __restrict__ quats, const float* __restrict__ logits,
                                                 const float* __restrict__ sh, DevCam cam,
                                                 float4* __restrict__ records, float* __restrict__ depth,
                                                 int* __restrict__ radius, uint32_t* __restrict__ tiles_touched,
                                                 float* __restrict__ cgrad) {
  const int i = blockIdx.x * kProjThreads + threadIdx.x;
  if (i >= n) return;
  const unsigned l = threadIdx.x;
  // element i of row k of a [rows][n] field
  auto at = [&](auto* p, int k) -> auto& { return soa_row<kProjThreads>(p, k, n)[l]; };
  constexpr int NC = DEG < 0 ? 0 : (DEG + 1) * (DEG + 1);
  float m[3], s[3], q[4];
#pragma unroll
  for (int k = 0; k < 3; ++k) { m[k] = at(means, k); s[k] = at(log_scales, k); }
#pragma unroll
  for (int k = 0; k < 4; ++k) q[k] = at(quats, k);
  const float logit = at(logits, 0);
  // the colour coefficients (most of the bytes read) are loaded with the
  // geometry, before it is known whether the Gaussian is live, so that their
  // latency overlaps the projection arithmetic
  float shv[3 * (NC > 0 ? NC : 1)];
#pragma unroll
  for (int j = 0; j < 3 * NC; ++j) shv[j] = at(sh, j);
  Geo g;
  bool live = project_geometry(m, s, q, logit, cam, g);
  float rgb[3] = {0.0f, 0.0f, 0.0f};
  // for the backward (cgrad): d colour / d direction, stored channel by
  // channel as it is formed, and the clamp decisions
  bool jac_done = false;
  uint32_t cmask = 0u;
  if (live && DEG >= 0) {   // DEG < 0: the learned decoder writes the colour afterwards
    float d[3], len;
    view_dir(m, cam, d, len);
    float Y[16];
    sh_basis(DEG, d[0], d[1], d[2], Y);
    // one pass over the basis functions: the colour sums and, for the
    // backward, d colour / d direction (each coefficient used once)
    float acc[3] = {0.0f, 0.0f, 0.0f};
    float jac[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < NC; ++j) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) acc[ch] += Y[j] * shv[3 * j + ch];
      if (cgrad && j > 0) {
        float gx, gy, gz;
        sh_grad_j(j, d[0], d[1], d[2], gx, gy, gz);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
          jac[3 * ch] += gx * shv[3 * j + ch];
          jac[3 * ch + 1] += gy * shv[3 * j + ch];
          jac[3 * ch + 2] += gz * shv[3 * j + ch];
        }
      }
    }
    float raw[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      raw[ch] = acc[ch] + 0.5f;
      rgb[ch] = fmaxf(raw[ch], 0.0f);
    }
    live = isfinite(rgb[0]) && isfinite(rgb[1]) && isfinite(rgb[2]);
    if (cgrad) {
      cmask = (raw[0] >= 0.0f ? 1u : 0u) | (raw[1] >= 0.0f ? 2u : 0u) | (raw[2] >= 0.0f ? 4u : 0u) |
              ((isfinite(raw[0]) && isfinite(raw[1]) && isfinite(raw[2])) ? 8u : 0u);
#pragma unroll
      for (int k = 0; k < 9; ++k) at(cgrad, k) = jac[k];
      jac_done = true;
    }
  }
  if (cgrad) {
    if (!jac_done)
#pragma unroll
      for (int k = 0; k < 9; ++k) at(cgrad, k) = 0.0f;
    at(cgrad, 9) = __uint_as_float(cmask);
  }
  float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0;
  int rad = 0;
  uint32_t cnt = 0;
  float dep = 0.0f;
  if (live) {
    float ex, ey;
    alpha_support(g, ex, ey);
    r0 = make_float4(g.u, g.v, g.A, g.B);
    r1 = make_float4(g.C, g.o, rgb[0], rgb[1]);
    r2 = make_float4(rgb[2], g.t[2], ex, ey);
    rad = g.radius;
    dep = g.t[2];
    int x0, x1, y0, y1;
    cnt = static_cast<uint32_t>(tile_rect(g.u, g.v, rad, cam.tiles_x, cam.tiles_y, x0, x1, y0, y1));
  }
  float4* rec = records + 3 * static_cast<int64_t>(blockIdx.x) * kProjThreads;
  rec[3 * l] = r0;
  rec[3 * l + 1] = r1;
  rec[3 * l + 2] = r2;
  at(depth, 0) = dep;
  at(radius, 0) = rad;
  at(tiles_touched, 0) = cnt;
}

gs_status launch_project(const gs_gaussians& g, const DevCam& cam, gs_projected& out, hipStream_t s) {
  const int n = static_cast<int>(g.n);
  if (n == 0) return GS_OK;
  const dim3 block(kProjThreads), grid(static_cast<unsigned>(ceil_div(n, kProjThreads)));
  float4* rec = reinterpret_cast<float4*>(out.records);
  if (g.colour_mode == 1) {
    { TimedLaunch gs_tl("k_project<-1>", s); k_project<-1><<<grid, block, 0, s>>>(n, g.means, g.log_scales, g.quats, g.logits, nullptr, cam, rec, out.depth,
                                         out.radius, out.tiles_touched, nullptr); }
    gs_status st = check_launch("k_project");
    if (st != GS_OK) return st;
    return launch_mlp_render(n, g.latents, g.means, out.radius, cam, g.mlp, out.records, s);
  }
  switch (g.sh_degree) {
    case 0: { TimedLaunch gs_tl("k_project<0>", s); k_project<0><<<grid, block, 0, s>>>(n, g.means, g.log_scales, g.quats, g.logits, g.sh, cam, rec,
                                                 out.depth, out.radius, out.tiles_touched, out.colour_grad); } break;
    case 1: { TimedLaunch gs_tl("k_project<1>", s); k_project<1><<<grid, block, 0, s>>>(n, g.means, g.log_scales, g.quats, g.logits, g.sh, cam, rec,
                                                 out.depth, out.radius, out.tiles_touched, out.colour_grad); } break;
    case 2: { TimedLaunch gs_tl("k_project<2>", s); k_project<2><<<grid, block, 0, s>>>(n, g.means, g.log_scales, g.quats, g.logits, g.sh, cam, rec,
                                                 out.depth, out.radius, out.tiles_touched, out.colour_grad); } break;
    default: { TimedLaunch gs_tl("k_project<3>", s); k_project<3><<<grid, block, 0, s>>>(n, g.means, g.log_scales, g.quats, g.logits, g.sh, cam, rec,
                                                  out.depth, out.radius, out.tiles_touched, out.colour_grad); } break;
  }
  return check_launch("k_project");
}

// ------------------------------------------------------------------ backward
//
// Chain rule through project_geometry and the SH colour, per Gaussian.
//   Sigma' = [[a, b], [b, c]] arrives as dL/d(a, b, c) (b counted twice),
//                     i.e. the symmetric gradient G' = [[ga, gb/2], [gb/2, gc]];
//   Sigma' = T Sigma T^T:  dL/dSigma = T^T G' T,  dL/dT = 2 G' T Sigma;
//   T = J W:  dL/dJ = dL/dT W^T;  J(t) with the slope clamp;
//   Sigma = M M^T, M = R S:  dL/dM = 2 dL/dSigma M,
//                     dL/ds_k = S_k (R^T dL/dM)_kk,  dL/dR = dL/dM S;
//   R(q^) -> q^ -> q through the normalisation.
//
// The record gradients come as g2d[9][n] (ROWS == false) or, straight from
// the compositing backward, as its accumulator rows acc[n][kAccStride]
// before the per-channel factors grad_scale (ROWS == true).  With stat_grad
// non-NULL, the densification statistics of the view are accumulated:
// stat_grad[i] += |(dL/du, dL/dv)| (pixel units) and stat_count[i] += 1 for
// every Gaussian whose footprint meets a tile.
template <int DEG, bool ROWS>
__global__ __launch_bounds__(kProjThreads) void k_project_bwd(int n, const float* __restrict__ means,
                                                     const float* __restrict__ log_scales,
                                                     const float* __restrict__ quats,
                                                     const float* __restrict__ logits,
                                                     const float* __restrict__ sh, DevCam cam,
                                                     const float* __restrict__ g2d, float* __restrict__ g_means,
                                                     float* __restrict__ g_scales, float* __restrict__ g_quats,
                                                     float* __restrict__ g_logits, float* __restrict__ g_sh,
                                                     const uint32_t* __restrict__ tiles_touched,
                                                     float* __restrict__ stat_grad,
                                                     uint32_t* __restrict__ stat_count,
                                                     const float* __restrict__ cgrad) {
  const int i = blockIdx.x * kProjThreads + threadIdx.x;
  if (i >= n) return;
  const unsigned l = threadIdx.x;
  // element i of row k of a [rows][n] field
  auto at = [&](auto* p, int k) -> auto& { return soa_row<kProjThreads>(p, k, n)[l]; };
  // DEG < 0: colour comes from the learned decoder, whose backward adds its
  // share to dL/dmean afterwards; only the geometry is differentiated here.
  // cgrad (from the projection): d colour / d direction and the clamp
  // decisions, read instead of the SH coefficients.
  constexpr int NC = DEG < 0 ? 0 : (DEG + 1) * (DEG + 1);
  constexpr int NCA = NC > 0 ? NC : 1;
  float m[3], s[3], q[4];
#pragma unroll
  for (int k = 0; k < 3; ++k) { m[k] = at(means, k); s[k] = at(log_scales, k); }
#pragma unroll
  for (int k = 0; k < 4; ++k) q[k] = at(quats, k);
  const float logit = at(logits, 0);
  Geo g;
  bool live = project_geometry(m, s, q, logit, cam, g);
  float d[3] = {0, 0, 0}, len = 1.0f;
  float Y[16];
  float raw[3] = {0, 0, 0};
  float f[NCA][3];
  float jac[9];
  uint32_t cmask = 0u;
  if (DEG >= 0 && cgrad) {
#pragma unroll
    for (int k = 0; k < 9; ++k) jac[k] = at(cgrad, k);
    cmask = __float_as_uint(at(cgrad, 9));
  } else {
#pragma unroll
    for (int j = 0; j < NC; ++j)
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) f[j][ch] = at(sh, 3 * j + ch);
  }
  if (live && DEG >= 0) {
    view_dir(m, cam, d, len);
    sh_basis(DEG, d[0], d[1], d[2], Y);
    if (cgrad) {
      live = (cmask & 8u) != 0u;
    } else {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        float acc = 0.0f;
#pragma unroll
        for (int j = 0; j < NC; ++j) acc += Y[j] * f[j][ch];
        raw[ch] = acc + 0.5f;
      }
      live = isfinite(raw[0]) && isfinite(raw[1]) && isfinite(raw[2]);
      cmask = (raw[0] >= 0.0f ? 1u : 0u) | (raw[1] >= 0.0f ? 2u : 0u) | (raw[2] >= 0.0f ? 4u : 0u);
    }
  }
  if (!live) {
#pragma unroll
    for (int k = 0; k < 3; ++k) { at(g_means, k) = 0.0f; at(g_scales, k) = 0.0f; }
#pragma unroll
    for (int k = 0; k < 4; ++k) at(g_quats, k) = 0.0f;
    at(g_logits, 0) = 0.0f;
#pragma unroll
    for (int j = 0; j < 3 * NC; ++j) at(g_sh, j) = 0.0f;
    return;
  }
  float G[GS_G2D];
  if constexpr (ROWS) {
    const float4* row = reinterpret_cast<const float4*>(g2d + static_cast<int64_t>(blockIdx.x) * kProjThreads * kAccStride) +
                        l * (kAccStride / 4);
    const float4 a = row[0], b = row[1], c = row[2];
    const float v[GS_G2D] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x};
#pragma unroll
    for (int k = 0; k < GS_G2D; ++k) G[k] = v[k] * grad_scale(k);
  } else {
#pragma unroll
    for (int k = 0; k < GS_G2D; ++k) G[k] = at(g2d, k);
  }
  if (stat_grad && at(tiles_touched, 0) > 0) {
    at(stat_grad, 0) += sqrtf(G[0] * G[0] + G[1] * G[1]);
    at(stat_count, 0) += 1u;
  }
  float gm[3] = {0.0f, 0.0f, 0.0f};

  // ---- colour
  if constexpr (DEG >= 0) {
  float gc[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) gc[ch] = ((cmask >> ch) & 1u) ? G[6 + ch] : 0.0f;
  float wj[16];
#pragma unroll
  for (int j = 0; j < NC; ++j) {
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) at(g_sh, 3 * j + ch) = Y[j] * gc[ch];
    if (!cgrad) wj[j] = gc[0] * f[j][0] + gc[1] * f[j][1] + gc[2] * f[j][2];
  }
  if (DEG > 0) {
    float gd[3];
    if (cgrad) {
      // dL/dd = sum over channels of dL/dc times d c / d d
#pragma unroll
      for (int k = 0; k < 3; ++k) gd[k] = gc[0] * jac[k] + gc[1] * jac[3 + k] + gc[2] * jac[6 + k];
    } else {
      sh_basis_vjp(DEG, d[0], d[1], d[2], wj, gd[0], gd[1], gd[2]);
    }
    const float dd = d[0] * gd[0] + d[1] * gd[1] + d[2] * gd[2];
    const float il = 1.0f / len;
#pragma unroll
    for (int k = 0; k < 3; ++k) gm[k] += (gd[k] - d[k] * dd) * il;
  }
  }

  // ---- opacity
  at(g_logits, 0) = G[5] * g.o * (1.0f - g.o);

  // ---- Sigma' gradient: the render backward already converted it from the
  // conic pair by pair; G[3] counts both off-diagonal entries.
  const float ga = G[2], gb = 0.5f * G[3], gcc = G[4];

  // ---- Sigma' = T Sigma T^T
  const float* T = g.T;
  // dL/dSigma = T^T G' T (3x3 symmetric)
  float GT0[3], GT1[3];  // rows of G' T
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    GT0[k] = ga * T[k] + gb * T[3 + k];
    GT1[k] = gb * T[k] + gcc * T[3 + k];
  }
  float gS[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) gS[3 * a + b] = T[a] * GT0[b] + T[3 + a] * GT1[b];
  // dL/dT = 2 G' T Sigma
  const float* Sg = g.Sig;
  const float Sfull[9] = {Sg[0], Sg[1], Sg[2], Sg[1], Sg[3], Sg[4], Sg[2], Sg[4], Sg[5]};
  float gT[6];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    gT[b] = 2.0f * (GT0[0] * Sfull[b] + GT0[1] * Sfull[3 + b] + GT0[2] * Sfull[6 + b]);
    gT[3 + b] = 2.0f * (GT1[0] * Sfull[b] + GT1[1] * Sfull[3 + b] + GT1[2] * Sfull[6 + b]);
  }
  // dL/dJ = dL/dT W^T ; only J00, J02, J11, J12 are non-zero entries of J
  const float* W = cam.R;
  const float gJ00 = gT[0] * W[0] + gT[1] * W[1] + gT[2] * W[2];
  const float gJ02 = gT[0] * W[6] + gT[1] * W[7] + gT[2] * W[8];
  const float gJ11 = gT[3] * W[3] + gT[4] * W[4] + gT[5] * W[5];
  const float gJ12 = gT[3] * W[6] + gT[4] * W[7] + gT[5] * W[8];
  const float tz = g.t[2];
  const float itz = 1.0f / tz, itz2 = itz * itz;
  float gt[3] = {0.0f, 0.0f, 0.0f};
  // J00 = fx/tz, J11 = fy/tz
  gt[2] += -(gJ00 * cam.fx + gJ11 * cam.fy) * itz2;
  // J02 = -fx sx/tz, J12 = -fy sy/tz  (sx = tx/tz unless clamped)
  gt[2] += (gJ02 * cam.fx * g.sx + gJ12 * cam.fy * g.sy) * itz2;
  const float gsx = -gJ02 * cam.fx * itz, gsy = -gJ12 * cam.fy * itz;
  if (!g.clx) { gt[0] += gsx * itz; gt[2] -= gsx * g.t[0] * itz2; }
  if (!g.cly) { gt[1] += gsy * itz; gt[2] -= gsy * g.t[1] * itz2; }
  // (u, v) = (fx tx/tz + cx, fy ty/tz + cy)
  gt[0] += G[0] * cam.fx * itz;
  gt[1] += G[1] * cam.fy * itz;
  gt[2] -= (G[0] * cam.fx * g.t[0] + G[1] * cam.fy * g.t[1]) * itz2;
  // t = W mu + t_cw
#pragma unroll
  for (int k = 0; k < 3; ++k) gm[k] += W[k] * gt[0] + W[3 + k] * gt[1] + W[6 + k] * gt[2];

  // ---- Sigma = M M^T, M = R S
  const float* R = g.R;
  float M[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) M[3 * a + b] = R[3 * a + b] * g.S[b];
  float gM[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      gM[3 * a + b] = 2.0f * (gS[3 * a] * M[b] + gS[3 * a + 1] * M[3 + b] + gS[3 * a + 2] * M[6 + b]);
#pragma unroll
  for (int k = 0; k < 3; ++k)
    at(g_scales, k) = g.S[k] * (R[k] * gM[k] + R[3 + k] * gM[3 + k] + R[6 + k] * gM[6 + k]);
  float gR[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) gR[3 * a + b] = gM[3 * a + b] * g.S[b];
  const float w = g.qn[0], x = g.qn[1], y = g.qn[2], z = g.qn[3];
  float gq[4];
  gq[0] = 2.0f * (z * (gR[3] - gR[1]) + y * (gR[2] - gR[6]) + x * (gR[7] - gR[5]));
  gq[1] = 2.0f * (y * (gR[3] + gR[1]) + z * (gR[6] + gR[2]) + w * (gR[7] - gR[5])) - 4.0f * x * (gR[4] + gR[8]);
  gq[2] = 2.0f * (x * (gR[3] + gR[1]) + w * (gR[2] - gR[6]) + z * (gR[7] + gR[5])) - 4.0f * y * (gR[0] + gR[8]);
  gq[3] = 2.0f * (w * (gR[3] - gR[1]) + x * (gR[6] + gR[2]) + y * (gR[7] + gR[5])) - 4.0f * z * (gR[0] + gR[4]);
  const float qd = w * gq[0] + x * gq[1] + y * gq[2] + z * gq[3];
#pragma unroll
  for (int k = 0; k < 4; ++k) at(g_quats, k) = (gq[k] - g.qn[k] * qd) * g.qinv;
#pragma unroll
  for (int k = 0; k < 3; ++k) at(g_means, k) = gm[k];
}

gs_status launch_project_bwd(const gs_gaussians& g, const DevCam& cam, const int* radius, const float* g2d, bool rows,
                             const uint32_t* tiles_touched, gs_densify_stats* stats, gs_gaussians_grad& gr, void* ws,
                             const float* cgrad, hipStream_t s) {
  const int n = static_cast<int>(g.n);
  if (n == 0) return GS_OK;
  const dim3 block(kProjThreads), grid(static_cast<unsigned>(ceil_div(n, kProjThreads)));
  float* sg = stats ? stats->grad_norm_sum : nullptr;
  uint32_t* sc = stats ? stats->visible_count : nullptr;
#define GS_PB(D, R)                                                                                               \
  k_project_bwd<D, R><<<grid, block, 0, s>>>(n, g.means, g.log_scales, g.quats, g.logits, g.sh, cam, g2d,          \
                                             gr.means, gr.log_scales, gr.quats, gr.logits, gr.sh, tiles_touched, \
                                             sg, sc, cgrad)
  {
    // the kernel's own template name, as profilers report it
    static const char* const kNames[2][4] = {
        {"k_project_bwd<0, false>", "k_project_bwd<1, false>", "k_project_bwd<2, false>", "k_project_bwd<3, false>"},
        {"k_project_bwd<0, true>", "k_project_bwd<1, true>", "k_project_bwd<2, true>", "k_project_bwd<3, true>"}};
    TimedLaunch gs_tl(g.colour_mode == 1 ? (rows ? "k_project_bwd<-1, true>" : "k_project_bwd<-1, false>")
                                         : kNames[rows ? 1 : 0][std::min(std::max(g.sh_degree, 0), 3)], s);
    if (g.colour_mode == 1) {
      if (rows) GS_PB(-1, true);
      else GS_PB(-1, false);
    } else if (rows) {
      switch (g.sh_degree) {
        case 0: GS_PB(0, true); break;
        case 1: GS_PB(1, true); break;
        case 2: GS_PB(2, true); break;
        default: GS_PB(3, true); break;
      }
    } else {
      switch (g.sh_degree) {
        case 0: GS_PB(0, false); break;
        case 1: GS_PB(1, false); break;
        case 2: GS_PB(2, false); break;
        default: GS_PB(3, false); break;
      }
    }
  }
#undef GS_PB
  gs_status st = check_launch("k_project_bwd");
  if (st != GS_OK || g.colour_mode != 1) return st;
  return launch_mlp_render_bwd(n, g.latents, g.means, radius, cam, g.mlp, g2d, rows, gr.latents, gr.means, gr.mlp, ws,
                               s);
}

}  // namespace gs
