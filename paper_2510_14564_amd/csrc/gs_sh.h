// Real spherical-harmonic basis (degree <= 3) and the unit view direction,
// shared by the projection and the learned colour decoder of the HIP path.
#pragma once

#include "gs_internal.h"

namespace gs {

// Real SH basis, Condon-Shortley phase kept, ordered by l then m = -l..l.
// Constants are the closed-form normalisations:
//   l=0: 1/(2 sqrt(pi));  l=1: sqrt(3/(4 pi));
//   l=2: (1/2) sqrt(15/pi), (1/4) sqrt(5/pi), (1/4) sqrt(15/pi);
//   l=3: (1/4) sqrt(35/(2 pi)), (1/2) sqrt(105/pi), (1/4) sqrt(21/(2 pi)),
//        (1/4) sqrt(7/pi), (1/4) sqrt(105/pi).
constexpr float kSH0 = 0.28209479177387814f;
constexpr float kSH1 = 0.48860251190291992f;
constexpr float kSH2a = 1.0925484305920792f;
constexpr float kSH2c = 0.31539156525252005f;
constexpr float kSH2e = 0.54627421529603959f;
constexpr float kSH3a = 0.59004358992664352f;
constexpr float kSH3b = 2.8906114426405538f;
constexpr float kSH3c = 0.45704579946446572f;
constexpr float kSH3d = 0.37317633259011540f;
constexpr float kSH3f = 1.4453057213202769f;

__device__ __forceinline__ void sh_basis(int deg, float x, float y, float z, float* Y) {
  Y[0] = kSH0;
  if (deg < 1) return;
  Y[1] = -kSH1 * y;
  Y[2] = kSH1 * z;
  Y[3] = -kSH1 * x;
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = kSH2a * x * y;
  Y[5] = -kSH2a * y * z;
  Y[6] = kSH2c * (2.0f * zz - xx - yy);
  Y[7] = -kSH2a * x * z;
  Y[8] = kSH2e * (xx - yy);
  if (deg < 3) return;
  Y[9] = -kSH3a * y * (3.0f * xx - yy);
  Y[10] = kSH3b * x * y * z;
  Y[11] = -kSH3c * y * (4.0f * zz - xx - yy);
  Y[12] = kSH3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
  Y[13] = -kSH3c * x * (4.0f * zz - xx - yy);
  Y[14] = kSH3f * z * (xx - yy);
  Y[15] = -kSH3a * x * (xx - 3.0f * yy);
}

// g = sum_j w_j grad Y_j(d) for the Cartesian forms above.
__device__ __forceinline__ void sh_basis_vjp(int deg, float x, float y, float z, const float* w, float& gx,
                                             float& gy, float& gz) {
  gx = gy = gz = 0.0f;
  if (deg < 1) return;
  gy += -kSH1 * w[1];
  gz += kSH1 * w[2];
  gx += -kSH1 * w[3];
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  gx += kSH2a * y * w[4];             gy += kSH2a * x * w[4];
  gy += -kSH2a * z * w[5];            gz += -kSH2a * y * w[5];
  gx += -2.0f * kSH2c * x * w[6];     gy += -2.0f * kSH2c * y * w[6];   gz += 4.0f * kSH2c * z * w[6];
  gx += -kSH2a * z * w[7];            gz += -kSH2a * x * w[7];
  gx += 2.0f * kSH2e * x * w[8];      gy += -2.0f * kSH2e * y * w[8];
  if (deg < 3) return;
  gx += -6.0f * kSH3a * x * y * w[9];
  gy += -kSH3a * (3.0f * xx - 3.0f * yy) * w[9];
  gx += kSH3b * y * z * w[10];  gy += kSH3b * x * z * w[10];  gz += kSH3b * x * y * w[10];
  gx += 2.0f * kSH3c * x * y * w[11];
  gy += -kSH3c * (4.0f * zz - xx - 3.0f * yy) * w[11];
  gz += -8.0f * kSH3c * y * z * w[11];
  gx += -6.0f * kSH3d * x * z * w[12];
  gy += -6.0f * kSH3d * y * z * w[12];
  gz += kSH3d * (6.0f * zz - 3.0f * xx - 3.0f * yy) * w[12];
  gx += -kSH3c * (4.0f * zz - 3.0f * xx - yy) * w[13];
  gy += 2.0f * kSH3c * x * y * w[13];
  gz += -8.0f * kSH3c * x * z * w[13];
  gx += 2.0f * kSH3f * x * z * w[14];
  gy += -2.0f * kSH3f * y * z * w[14];
  gz += kSH3f * (xx - yy) * w[14];
  gx += -kSH3a * (3.0f * xx - 3.0f * yy) * w[15];
  gy += 6.0f * kSH3a * x * y * w[15];
}

// grad Y_j(d) of one basis function (j a compile-time constant once the
// caller's loop is unrolled), the terms of sh_basis_vjp for that j.
__device__ __forceinline__ void sh_grad_j(int j, float x, float y, float z, float& gx, float& gy, float& gz) {
  const float xx = x * x, yy = y * y, zz = z * z;
  gx = gy = gz = 0.0f;
  switch (j) {
    case 1: gy = -kSH1; break;
    case 2: gz = kSH1; break;
    case 3: gx = -kSH1; break;
    case 4: gx = kSH2a * y; gy = kSH2a * x; break;
    case 5: gy = -kSH2a * z; gz = -kSH2a * y; break;
    case 6: gx = -2.0f * kSH2c * x; gy = -2.0f * kSH2c * y; gz = 4.0f * kSH2c * z; break;
    case 7: gx = -kSH2a * z; gz = -kSH2a * x; break;
    case 8: gx = 2.0f * kSH2e * x; gy = -2.0f * kSH2e * y; break;
    case 9: gx = -6.0f * kSH3a * x * y; gy = -kSH3a * (3.0f * xx - 3.0f * yy); break;
    case 10: gx = kSH3b * y * z; gy = kSH3b * x * z; gz = kSH3b * x * y; break;
    case 11: gx = 2.0f * kSH3c * x * y; gy = -kSH3c * (4.0f * zz - xx - 3.0f * yy); gz = -8.0f * kSH3c * y * z; break;
    case 12: gx = -6.0f * kSH3d * x * z; gy = -6.0f * kSH3d * y * z; gz = kSH3d * (6.0f * zz - 3.0f * xx - 3.0f * yy); break;
    case 13: gx = -kSH3c * (4.0f * zz - 3.0f * xx - yy); gy = 2.0f * kSH3c * x * y; gz = -8.0f * kSH3c * x * z; break;
    case 14: gx = 2.0f * kSH3f * x * z; gy = -2.0f * kSH3f * y * z; gz = kSH3f * (xx - yy); break;
    case 15: gx = -kSH3a * (3.0f * xx - 3.0f * yy); gy = 6.0f * kSH3a * x * y; break;
    default: break;
  }
}

__device__ __forceinline__ void view_dir(const float m[3], const DevCam& cam, float d[3], float& len) {
  const float dx = m[0] - cam.centre[0], dy = m[1] - cam.centre[1], dz = m[2] - cam.centre[2];
  len = sqrtf(dx * dx + dy * dy + dz * dz);
  const float il = 1.0f / len;
  d[0] = dx * il; d[1] = dy * il; d[2] = dz * il;
}

}  // namespace gs
