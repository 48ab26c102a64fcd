// 3D filter (App. "Dead Gaussians"): Sigma + s I and o_hat = o sqrt(|Sigma| / |Sigma + s I|).
// The filter size s of each Gaussian follows the filter the paper adopts: (k z / f)^2 for the
// camera that samples the centre most finely (largest f / z among cameras whose image holds
// the projected centre beyond the near plane), 0 when no camera sees it.  Adding s I keeps
// the rotation and adds s to every squared scale, and |Sigma| / |Sigma + s I| =
// prod s_j^2 / prod (s_j^2 + s).  One thread per Gaussian; the adjoint holds s constant.
#include "launch.h"

namespace sof {

__global__ __launch_bounds__(256) void k_filter3d(const float* means, const float* scales, const float* opac,
                                                  int64_t n, const sof_camera* cams, int n_cams, float near_plane,
                                                  float k, float* var, float* scales_out, float* opac_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float mx = means[3 * i], my = means[3 * i + 1], mz = means[3 * i + 2];
  float best = 0.f;                                     // largest f / z over cameras seeing the centre
  for (int c = 0; c < n_cams; ++c) {
    const sof_camera& cam = cams[c];
    const float x = fmaf(cam.R[0], mx, fmaf(cam.R[1], my, fmaf(cam.R[2], mz, cam.t[0])));
    const float y = fmaf(cam.R[3], mx, fmaf(cam.R[4], my, fmaf(cam.R[5], mz, cam.t[1])));
    const float z = fmaf(cam.R[6], mx, fmaf(cam.R[7], my, fmaf(cam.R[8], mz, cam.t[2])));
    if (!(z > near_plane)) continue;
    const float u = cam.fx * x / z + cam.cx, v = cam.fy * y / z + cam.cy;
    if (u >= 0.f && u < (float)cam.width && v >= 0.f && v < (float)cam.height) best = fmaxf(best, cam.fx / z);
  }
  const float s = best > 0.f ? (k / best) * (k / best) : 0.f;
  float ratio = 1.f;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const float sj = scales[3 * i + j];
    const float nj = sqrtf(fmaf(sj, sj, s));
    scales_out[3 * i + j] = nj;
    ratio *= sj / nj;
  }
  var[i] = s;
  opac_out[i] = opac[i] * ratio;
}

__global__ __launch_bounds__(256) void k_filter3d_bwd(const float* scales, const float* opac, const float* var,
                                                      int64_t n, const float* d_scales_out, const float* d_opac_out,
                                                      float* d_scales, float* d_opac) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float s = var[i];
  float sj[3], nj[3], ratio = 1.f;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    sj[j] = scales[3 * i + j];
    nj[j] = sqrtf(fmaf(sj[j], sj[j], s));
    ratio *= sj[j] / nj[j];
  }
  const float go = d_opac_out ? d_opac_out[i] : 0.f;
  const float oh = opac[i] * ratio;
  d_opac[i] = go * ratio;
  // d n_j / d s_j = s_j / n_j;  d log(ratio) / d s_j = 1 / s_j - s_j / n_j^2 = s / (s_j n_j^2)
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const float gs = d_scales_out ? d_scales_out[3 * i + j] : 0.f;
    d_scales[3 * i + j] = gs * sj[j] / nj[j] + go * oh * s / (sj[j] * nj[j] * nj[j]);
  }
}

hipError_t launch_filter3d(const float* means, const float* scales, const float* opac, int64_t n,
                           const sof_camera* cams, int n_cams, float near_plane, float k, float* var,
                           float* scales_out, float* opac_out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_filter3d, dim3((unsigned)div_up(n, 256)), dim3(256), 0, s, means, scales, opac, n, cams, n_cams,
                     near_plane, k, var, scales_out, opac_out);
  return hipGetLastError();
}

hipError_t launch_filter3d_bwd(const float* scales, const float* opac, const float* var, int64_t n,
                               const float* d_scales_out, const float* d_opac_out, float* d_scales, float* d_opac,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_filter3d_bwd, dim3((unsigned)div_up(n, 256)), dim3(256), 0, s, scales, opac, var, n,
                     d_scales_out, d_opac_out, d_scales, d_opac);
  return hipGetLastError();
}

}  // namespace sof
