// Reduction of per-instance gradient partials and the chain rule back to the Gaussian
// parameters (adjoint of sof_project).  One thread per Gaussian: for every camera it sums
// the partials of the Gaussian's instances (contiguous in emission order, summed in a fixed
// order, so the result is deterministic), maps the camera-space (mu_c, P_c) gradients to
// world space, adds the view-dependent colour and normal terms, and finally chains the
// world precision P = R diag(1/s^2) R^T to scales and the quaternion.
#include "launch.h"
#include "sh_eval.h"

namespace sof {

__global__ __launch_bounds__(128) void k_project_bwd(ProjectBwdArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int deg = a.sh_degree;
  const int K = (deg + 1) * (deg + 1);
  const int64_t kinst = *a.count_total < a.cap ? *a.count_total : a.cap;

  const double mx = a.means[3 * i], my = a.means[3 * i + 1], mzw = a.means[3 * i + 2];
  double qw = a.quats[4 * i], qx = a.quats[4 * i + 1], qy = a.quats[4 * i + 2], qz = a.quats[4 * i + 3];
  const double qnorm = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  qw /= qnorm; qx /= qnorm; qy /= qnorm; qz /= qnorm;
  double Rg[9];
  quat_rot<double>(qw, qx, qy, qz, Rg);
  const double s[3] = {a.scales[3 * i], a.scales[3 * i + 1], a.scales[3 * i + 2]};
  const int jmin = argmin3(s[0], s[1], s[2]);
  const float* f = a.sh + (size_t)i * K * 3;

  double dmu[3] = {0, 0, 0};
  double dPw[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  double dRg[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  double dop = 0.0;
  float dsh[kMaxShCoeffs * 3];
  for (int k = 0; k < K * 3; ++k) dsh[k] = 0.f;

  for (int c = 0; c < a.n_cams; ++c) {
    const int64_t vg = (int64_t)c * a.n + i;
    const int cnt = a.counts[vg];
    if (cnt == 0) continue;
    const int64_t e0 = a.offsets[vg];
    const int64_t e1 = (e0 + cnt < kinst) ? e0 + cnt : kinst;
    float gsum[kGradFields];
#pragma unroll
    for (int f4 = 0; f4 < kGradFields; ++f4) gsum[f4] = 0.f;
    for (int64_t e = e0; e < e1; ++e) {
      const float4* src = (const float4*)(a.grads + (size_t)e * kGradFields);
#pragma unroll
      for (int f4 = 0; f4 < kGradFields / 4; ++f4) {
        const float4 v = src[f4];
        gsum[4 * f4] += v.x; gsum[4 * f4 + 1] += v.y; gsum[4 * f4 + 2] += v.z; gsum[4 * f4 + 3] += v.w;
      }
    }
    const sof_camera cam = a.cams[c];
    double Rc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Rc[k] = cam.R[k];
    // mu_c = Rc mu + t  ->  dmu += Rc^T dmu_c
    for (int r = 0; r < 3; ++r) dmu[r] += Rc[r] * gsum[0] + Rc[3 + r] * gsum[1] + Rc[6 + r] * gsum[2];
    // P_c = Rc P Rc^T  ->  dP += Rc^T G Rc  (G symmetric, full-matrix entries)
    const double G[9] = {gsum[3], gsum[4], gsum[5], gsum[4], gsum[6], gsum[7], gsum[5], gsum[7], gsum[8]};
    double GR[9];
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) GR[3 * r + k] = G[3 * r] * Rc[k] + G[3 * r + 1] * Rc[3 + k] + G[3 * r + 2] * Rc[6 + k];
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) dPw[3 * r + k] += Rc[r] * GR[k] + Rc[3 + r] * GR[3 + k] + Rc[6 + r] * GR[6 + k];
    dop += gsum[9];

    // camera centre and view direction, evaluated exactly as in the forward pass
    const double ccx = -(Rc[0] * cam.t[0] + Rc[3] * cam.t[1] + Rc[6] * cam.t[2]);
    const double ccy = -(Rc[1] * cam.t[0] + Rc[4] * cam.t[1] + Rc[7] * cam.t[2]);
    const double ccz = -(Rc[2] * cam.t[0] + Rc[5] * cam.t[1] + Rc[8] * cam.t[2]);
    const double ddx = mx - ccx, ddy = my - ccy, ddz = mzw - ccz;
    const double dn = rsqrt(ddx * ddx + ddy * ddy + ddz * ddz);
    const float dx = (float)(ddx * dn), dy = (float)(ddy * dn), dz = (float)(ddz * dn);
    float Y[kMaxShCoeffs];
    sh_basis(deg, dx, dy, dz, Y);
    float cr = 0.5f, cg = 0.5f, cb = 0.5f;
    for (int k = 0; k < K; ++k) {
      cr = fmaf(Y[k], f[3 * k], cr);
      cg = fmaf(Y[k], f[3 * k + 1], cg);
      cb = fmaf(Y[k], f[3 * k + 2], cb);
    }
    const float gc[3] = {cr > 0.f ? gsum[10] : 0.f, cg > 0.f ? gsum[11] : 0.f, cb > 0.f ? gsum[12] : 0.f};
    float wk[kMaxShCoeffs];
    for (int k = 0; k < K; ++k) {
      dsh[3 * k] += Y[k] * gc[0];
      dsh[3 * k + 1] += Y[k] * gc[1];
      dsh[3 * k + 2] += Y[k] * gc[2];
      wk[k] = f[3 * k] * gc[0] + f[3 * k + 1] * gc[1] + f[3 * k + 2] * gc[2];
    }
    float gx, gy, gz;
    sh_basis_grad(deg, dx, dy, dz, wk, gx, gy, gz);
    // d dir / d mu = (I - dir dir^T) / |mu - centre|
    const double dot = (double)gx * dx + (double)gy * dy + (double)gz * dz;
    dmu[0] += ((double)gx - dot * dx) * dn;
    dmu[1] += ((double)gy - dot * dy) * dn;
    dmu[2] += ((double)gz - dot * dz) * dn;

    // normal: +-column jmin of Rg, flipped to face the camera
    const double nx = Rg[jmin], ny = Rg[3 + jmin], nz = Rg[6 + jmin];
    const double sg = (nx * (ccx - mx) + ny * (ccy - my) + nz * (ccz - mzw) < 0.0) ? -1.0 : 1.0;
    dRg[jmin] += sg * gsum[13];
    dRg[3 + jmin] += sg * gsum[14];
    dRg[6 + jmin] += sg * gsum[15];
  }

  // P = Rg D Rg^T, D = diag(1/s^2):  dRg += 2 dP Rg D,  dD_kk = (Rg^T dP Rg)_kk
  const double D[3] = {1.0 / (s[0] * s[0]), 1.0 / (s[1] * s[1]), 1.0 / (s[2] * s[2])};
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k)
      dRg[3 * r + k] += 2.0 * (dPw[3 * r] * Rg[k] + dPw[3 * r + 1] * Rg[3 + k] + dPw[3 * r + 2] * Rg[6 + k]) * D[k];
  double ds[3];
  for (int k = 0; k < 3; ++k) {
    double v = 0.0;
    for (int r = 0; r < 3; ++r)
      for (int l = 0; l < 3; ++l) v += Rg[3 * r + k] * dPw[3 * r + l] * Rg[3 * l + k];
    ds[k] = v * (-2.0 * D[k] / s[k]);
  }
  // rotation matrix of the unit quaternion -> quaternion, then through the normalisation
  const double w = qw, x = qx, y = qy, z = qz;
  const double* g = dRg;
  double dq[4];
  dq[0] = 2.0 * (-z * g[1] + y * g[2] + z * g[3] - x * g[5] - y * g[6] + x * g[7]);
  dq[1] = 2.0 * (y * g[1] + z * g[2] + y * g[3] - 2.0 * x * g[4] - w * g[5] + z * g[6] + w * g[7] - 2.0 * x * g[8]);
  dq[2] = 2.0 * (-2.0 * y * g[0] + x * g[1] + w * g[2] + x * g[3] + z * g[5] - w * g[6] + z * g[7] - 2.0 * y * g[8]);
  dq[3] = 2.0 * (-2.0 * z * g[0] - w * g[1] + x * g[2] + w * g[3] - 2.0 * z * g[4] + y * g[5] + x * g[6] + y * g[7]);
  const double qd = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
  const double qv[4] = {w, x, y, z};
  for (int k = 0; k < 4; ++k) a.d_quats[4 * i + k] = (float)((dq[k] - qv[k] * qd) / qnorm);
  for (int k = 0; k < 3; ++k) {
    a.d_means[3 * i + k] = (float)dmu[k];
    a.d_scales[3 * i + k] = (float)ds[k];
  }
  a.d_opac[i] = (float)dop;
  for (int k = 0; k < K * 3; ++k) a.d_sh[(size_t)i * K * 3 + k] = dsh[k];
}

hipError_t launch_project_bwd(const ProjectBwdArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  const int th = 128;
  hipLaunchKernelGGL(k_project_bwd, dim3((unsigned)div_up(a.n, th)), dim3(th), 0, s, a);
  return hipGetLastError();
}

}  // namespace sof
