// Real spherical harmonics up to degree 3 (Condon-Shortley phase, coefficient l^2 + l + m),
// written as polynomials of the unit direction (x, y, z), and their gradients.
#pragma once

#include <hip/hip_runtime.h>

namespace sof {

// Normalisation constants of the real SH basis, K_l^m sqrt(2) P_l^m reduced to polynomials.
constexpr float kY00 = 0.28209479177387814f;   // 1 / (2 sqrt(pi))
constexpr float kY1 = 0.48860251190291992f;    // sqrt(3 / (4 pi))
constexpr float kY2a = 1.09254843059207907f;   // sqrt(15 / (4 pi))
constexpr float kY2b = 0.31539156525252001f;   // sqrt(5 / (16 pi))
constexpr float kY2c = 0.54627421529603954f;   // sqrt(15 / (16 pi))
constexpr float kY3a = 0.59004358992664352f;   // sqrt(35 / (32 pi))
constexpr float kY3b = 2.89061144264055406f;   // sqrt(105 / (4 pi))
constexpr float kY3c = 0.45704579946446572f;   // sqrt(21 / (32 pi))
constexpr float kY3d = 0.37317633259011540f;   // sqrt(7 / (16 pi))
constexpr float kY3e = 1.44530572132027703f;   // sqrt(105 / (16 pi))

// Basis values Y[0..(deg+1)^2).
__device__ inline void sh_basis(int deg, float x, float y, float z, float* Y) {
  Y[0] = kY00;
  if (deg < 1) return;
  Y[1] = -kY1 * y;
  Y[2] = kY1 * z;
  Y[3] = -kY1 * x;
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = kY2a * x * y;
  Y[5] = -kY2a * y * z;
  Y[6] = kY2b * (2.f * zz - xx - yy);
  Y[7] = -kY2a * x * z;
  Y[8] = kY2c * (xx - yy);
  if (deg < 3) return;
  Y[9] = -kY3a * y * (3.f * xx - yy);
  Y[10] = kY3b * x * y * z;
  Y[11] = -kY3c * y * (4.f * zz - xx - yy);
  Y[12] = kY3d * z * (2.f * zz - 3.f * xx - 3.f * yy);
  Y[13] = -kY3c * x * (4.f * zz - xx - yy);
  Y[14] = kY3e * z * (xx - yy);
  Y[15] = -kY3a * x * (xx - 3.f * yy);
}

// Gradient of sum_k w_k Y_k with respect to (x, y, z) of the polynomial (not yet projected
// onto the sphere's tangent plane).
__device__ inline void sh_basis_grad(int deg, float x, float y, float z, const float* w, float& gx,
                                     float& gy, float& gz) {
  gx = gy = gz = 0.f;
  if (deg < 1) return;
  gy += -kY1 * w[1];
  gz += kY1 * w[2];
  gx += -kY1 * w[3];
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  gx += kY2a * y * w[4];
  gy += kY2a * x * w[4];
  gy += -kY2a * z * w[5];
  gz += -kY2a * y * w[5];
  gx += -2.f * kY2b * x * w[6];
  gy += -2.f * kY2b * y * w[6];
  gz += 4.f * kY2b * z * w[6];
  gx += -kY2a * z * w[7];
  gz += -kY2a * x * w[7];
  gx += 2.f * kY2c * x * w[8];
  gy += -2.f * kY2c * y * w[8];
  if (deg < 3) return;
  gx += -6.f * kY3a * x * y * w[9];
  gy += -kY3a * (3.f * xx - 3.f * yy) * w[9];
  gx += kY3b * y * z * w[10];
  gy += kY3b * x * z * w[10];
  gz += kY3b * x * y * w[10];
  gx += 2.f * kY3c * x * y * w[11];
  gy += -kY3c * (4.f * zz - xx - 3.f * yy) * w[11];
  gz += -8.f * kY3c * y * z * w[11];
  gx += -6.f * kY3d * x * z * w[12];
  gy += -6.f * kY3d * y * z * w[12];
  gz += kY3d * (6.f * zz - 3.f * xx - 3.f * yy) * w[12];
  gx += -kY3c * (4.f * zz - 3.f * xx - yy) * w[13];
  gy += 2.f * kY3c * x * y * w[13];
  gz += -8.f * kY3c * x * z * w[13];
  gx += 2.f * kY3e * x * z * w[14];
  gy += -2.f * kY3e * y * z * w[14];
  gz += kY3e * (xx - yy) * w[14];
  gx += -kY3a * (3.f * xx - 3.f * yy) * w[15];
  gy += 6.f * kY3a * x * y * w[15];
}

// Rotation matrix (row-major) of a unit quaternion (w, x, y, z), Hamilton convention.
template <typename T>
__host__ __device__ inline void quat_rot(T w, T x, T y, T z, T* R) {
  R[0] = T(1) - T(2) * (y * y + z * z);
  R[1] = T(2) * (x * y - w * z);
  R[2] = T(2) * (x * z + w * y);
  R[3] = T(2) * (x * y + w * z);
  R[4] = T(1) - T(2) * (x * x + z * z);
  R[5] = T(2) * (y * z - w * x);
  R[6] = T(2) * (x * z - w * y);
  R[7] = T(2) * (y * z + w * x);
  R[8] = T(1) - T(2) * (x * x + y * y);
}

// Index of the smallest scale, lowest index on ties.
template <typename T>
__host__ __device__ inline int argmin3(T a, T b, T c) {
  if (a <= b && a <= c) return 0;
  if (b <= c) return 1;
  return 2;
}

}  // namespace sof
