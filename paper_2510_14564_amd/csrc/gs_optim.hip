// Adam over every parameter array of a Gaussian set in one launch: the
// optimiser step that follows the backward in a training iteration.
//
// The arrays form six segments (means, log-scales, quaternions, logits, the
// degree-0 SH coefficients, the other SH coefficients), each with its own
// learning rate.  A thread updates four consecutive values of one segment
// with 16-byte loads and stores when the segment's four arrays allow it.  The
// step is bound by HBM: per value it reads the parameter, its gradient and
// both moments and writes the parameter and both moments (28 bytes).
#include <cmath>

#include "gs_internal.h"

namespace gs {

constexpr int kAdamSegs = 6;

struct AdamSeg {
  float* p;
  const float* g;
  float* m;
  float* v;
  int64_t len;     // values in the segment
  int64_t chunk0;  // first 4-value chunk of the segment in the launch
  float lr;
  int vec;         // all four arrays 16-byte aligned and len % 4 == 0
};

struct AdamArgs {
  AdamSeg seg[kAdamSegs];
  int64_t chunks;
  float b1, b2, eps, bc1, bc2;
};

__device__ __forceinline__ void adam_one(float& p, float g, float& m, float& v, float lr, const AdamArgs& a) {
  m = a.b1 * m + (1.0f - a.b1) * g;
  v = a.b2 * v + (1.0f - a.b2) * g * g;
  p = p - lr * (m / a.bc1) / (sqrtf(v / a.bc2) + a.eps);
}

__global__ __launch_bounds__(256) void k_adam_gaussians(AdamArgs a) {
  for (int64_t c = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; c < a.chunks;
       c += static_cast<int64_t>(gridDim.x) * 256) {
    int s = 0;
#pragma unroll
    for (int k = 1; k < kAdamSegs; ++k) s += c >= a.seg[k].chunk0 ? 1 : 0;
    const AdamSeg& sg = a.seg[s];
    const int64_t e = 4 * (c - sg.chunk0);
    if (sg.vec) {
      float4 p = reinterpret_cast<const float4*>(sg.p)[e / 4];
      const float4 g = reinterpret_cast<const float4*>(sg.g)[e / 4];
      float4 m = reinterpret_cast<const float4*>(sg.m)[e / 4];
      float4 v = reinterpret_cast<const float4*>(sg.v)[e / 4];
      adam_one(p.x, g.x, m.x, v.x, sg.lr, a);
      adam_one(p.y, g.y, m.y, v.y, sg.lr, a);
      adam_one(p.z, g.z, m.z, v.z, sg.lr, a);
      adam_one(p.w, g.w, m.w, v.w, sg.lr, a);
      reinterpret_cast<float4*>(sg.p)[e / 4] = p;
      reinterpret_cast<float4*>(sg.m)[e / 4] = m;
      reinterpret_cast<float4*>(sg.v)[e / 4] = v;
    } else {
      const int64_t end = min(e + 4, sg.len);
      for (int64_t i = e; i < end; ++i) {
        float p = sg.p[i], m = sg.m[i], v = sg.v[i];
        adam_one(p, sg.g[i], m, v, sg.lr, a);
        sg.p[i] = p;
        sg.m[i] = m;
        sg.v[i] = v;
      }
    }
  }
}

gs_status launch_adam_gaussians(int64_t n, int sh_degree, const gs_param_arrays& p, const gs_gaussians_grad& g,
                                const gs_param_arrays& m, const gs_param_arrays& v, const gs_adam_config& cfg,
                                hipStream_t s) {
  const int64_t nc = (sh_degree + 1) * (sh_degree + 1);
  AdamArgs a{};
  // (parameter, gradient, first moment, second moment, values, learning rate)
  const struct {
    float* p;
    const float* g;
    float* m;
    float* v;
    int64_t len;
    float lr;
  } segs[kAdamSegs] = {
      {p.means, g.means, m.means, v.means, 3 * n, cfg.lr_means},
      {p.log_scales, g.log_scales, m.log_scales, v.log_scales, 3 * n, cfg.lr_log_scales},
      {p.quats, g.quats, m.quats, v.quats, 4 * n, cfg.lr_quats},
      {p.logits, g.logits, m.logits, v.logits, n, cfg.lr_logits},
      {p.sh, g.sh, m.sh, v.sh, 3 * n, cfg.lr_sh_dc},
      {p.sh + 3 * n, g.sh + 3 * n, m.sh + 3 * n, v.sh + 3 * n, 3 * (nc - 1) * n, cfg.lr_sh_rest},
  };
  int64_t chunks = 0;
  for (int k = 0; k < kAdamSegs; ++k) {
    AdamSeg& d = a.seg[k];
    d.p = segs[k].p;
    d.g = segs[k].g;
    d.m = segs[k].m;
    d.v = segs[k].v;
    d.len = segs[k].len;
    d.lr = segs[k].lr;
    d.chunk0 = chunks;
    const uintptr_t al = reinterpret_cast<uintptr_t>(d.p) | reinterpret_cast<uintptr_t>(d.g) |
                         reinterpret_cast<uintptr_t>(d.m) | reinterpret_cast<uintptr_t>(d.v);
    d.vec = (al % 16 == 0 && d.len % 4 == 0) ? 1 : 0;
    chunks += ceil_div(d.len, 4);
  }
  a.chunks = chunks;
  a.b1 = cfg.beta1;
  a.b2 = cfg.beta2;
  a.eps = cfg.eps;
  a.bc1 = static_cast<float>(1.0 - std::pow(static_cast<double>(cfg.beta1), cfg.step));
  a.bc2 = static_cast<float>(1.0 - std::pow(static_cast<double>(cfg.beta2), cfg.step));
  if (chunks == 0) return GS_OK;
  const unsigned grid = static_cast<unsigned>(std::min<int64_t>(ceil_div(chunks, 256), 1 << 20));
  { TimedLaunch gs_tl("k_adam_gaussians", s); k_adam_gaussians<<<grid, 256, 0, s>>>(a); }
  return check_launch("k_adam_gaussians");
}

}  // namespace gs
