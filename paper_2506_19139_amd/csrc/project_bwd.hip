// Reduction of per-instance gradient partials and the chain rule back to the Gaussian
// parameters (adjoint of sof_project), in two kernels.  k_grad_reduce: the lane of each
// (camera, Gaussian) gets the sum of the partials of its instances (contiguous in emission
// order; added in a fixed order, so this sum adds no order dependence of its own) in the slot
// of its first instance, its wave streaming the partials through LDS.
// k_project_bwd: one thread per Gaussian reads those sums for every camera, maps the
// camera-space (mu_c, P_c) gradients to world space, adds the view-dependent colour and normal
// terms, and finally chains the world precision P = R diag(1/s^2) R^T to scales and the
// quaternion.
#include "launch.h"
#include "sh_eval.h"

namespace sof {

constexpr int kPbThreads = 128;

// Copy a [rows, width] float block staged in LDS to consecutive rows of a global array
// with coalesced stores (one row per thread would stride the writes).
__device__ inline void store_rows(const float* lds, float* dst, int64_t row0, int rows, int width) {
  const int total = rows * width;
  float* out = dst + row0 * width;
  for (int k = threadIdx.x; k < total; k += kPbThreads) out[k] = lds[k];
}

constexpr int kGrThreads = 256;
constexpr int kGrWindow = 64;                   // instances per LDS window of a wave
constexpr int kGrRow = kGradFields + 4;         // LDS row stride (16-B aligned; rows start in
                                                // different banks)
constexpr int kGrLoads = kGrWindow * kGradFields / 4 / 64;   // float4 loads per lane and window
typedef float f32x4 __attribute__((ext_vector_type(4)));       // kept in registers (an array of
                                                               // HIP's float4 went to scratch)

// The partials of instances [w0, min(w0 + kGrWindow, Eend)) of a wave's run, one float4 per
// lane and load; every load unconditional (the index clamped into the window), so that they
// are in flight together (predicated loads were each waited for on their own).
__device__ __attribute__((always_inline)) inline void gr_load_window(const float* grads, int64_t w0, int64_t Eend,
                                                                     int lane, f32x4 (&buf)[kGrLoads]) {
  const int nf = (int)((Eend - w0 < kGrWindow ? Eend - w0 : kGrWindow) * (kGradFields / 4));
  const f32x4* src = (const f32x4*)(grads + (size_t)w0 * kGradFields);
#pragma unroll
  for (int r = 0; r < kGrLoads; ++r) {
    const int f = lane + 64 * r;
    buf[r] = src[f < nf ? f : nf - 1];
  }
}

__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A wave owns 64 consecutive (camera, Gaussian) pairs, whose instances are one contiguous run
// of partials.  The run streams through an LDS window of kGrWindow instances with coalesced
// loads (the next window's loads in flight while the current one is summed).  Inside a window
// the sums run across lanes, so that no lane waits for the Gaussian with the most instances:
// lane r finds the owner of row r (a binary search over the wave's prefix of counts); lane
// (f, q) adds field f over the 16 rows of quarter q, one run per owner, and leaves each run's
// sum in the run's first row; the owner's lane then adds its (at most four) runs in order.
// Every sum has a fixed order (rows in emission order inside a run, runs and windows in
// order), so the result does not depend on scheduling.  (A lane adding its own rows one by
// one took 67 us at 1M Gaussians 1080p, as long as the wave's largest count; each lane
// loading its own instances from global memory 145 us.)
__global__ __launch_bounds__(kGrThreads) void k_grad_reduce(const int32_t* counts, const int64_t* offsets,
                                                           const int64_t* count_total, int64_t cap, int64_t vn,
                                                           float* grads) {
  __shared__ __align__(16) float win[kGrThreads / 64][kGrWindow * kGrRow];
  __shared__ __align__(16) int32_t own[kGrThreads / 64][kGrWindow];
  static_assert(kGrWindow == 64 && kGradFields == 16, "one row per lane; 16 fields x 4 quarters of 16 rows");
  const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
  const int64_t base = ((int64_t)blockIdx.x * (kGrThreads / 64) + w) * 64;
  if (base >= vn) return;                                 // wave-uniform
  const int64_t vg = base + lane;
  const int64_t kinst = *count_total < cap ? *count_total : cap;
  const int cnt = vg < vn ? counts[vg] : 0;
  const int64_t e0 = vg < vn ? offsets[vg] : 0;
  const int64_t e1 = (e0 + cnt < kinst) ? e0 + cnt : kinst;
  const bool need = e1 - e0 >= 2;                         // one instance is its own sum
  if (__ballot(need) == 0) return;
  int incl = cnt;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  const int total = __shfl(incl, 63, 64);
  const int64_t E0 = offsets[base];
  const int64_t Eend = (E0 + total < kinst) ? E0 + total : kinst;
  float* lw = win[w];
  int32_t* lo_own = own[w];
  const int f = lane & 15, q = lane >> 4;                 // field and quarter of the run sums
  float4 s[kGradFields / 4];
#pragma unroll
  for (int f4 = 0; f4 < kGradFields / 4; ++f4) s[f4] = make_float4(0.f, 0.f, 0.f, 0.f);
  f32x4 buf[kGrLoads];
  gr_load_window(grads, E0, Eend, lane, buf);
  for (int64_t w0 = E0; w0 < Eend; w0 += kGrWindow) {
#pragma unroll
    for (int r = 0; r < kGrLoads; ++r) {
      const int fi = lane + 64 * r;
      *(f32x4*)&lw[(fi >> 2) * kGrRow + (fi & 3) * 4] = buf[r];
    }
    {
      // owner of row `lane`: the first lane whose inclusive prefix exceeds the row's offset
      const int j = (int)(w0 - E0) + lane;
      int lo = 0, hi = 63;
#pragma unroll
      for (int it = 0; it < 6; ++it) {
        const int mid = (lo + hi) >> 1;
        const bool right = __shfl(incl, mid, 64) <= j;
        lo = right ? mid + 1 : lo;
        hi = right ? hi : mid;
      }
      lo_own[lane] = (w0 + lane < Eend) ? lo : -1;
    }
    wave_lds_sync();
    // the next window's loads (the last window re-reads itself: no branch around the loads,
    // which would keep buf out of registers)
    gr_load_window(grads, w0 + kGrWindow < Eend ? w0 + kGrWindow : w0, Eend, lane, buf);
    {
      int ow[16];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int4 o4 = *(const int4*)&lo_own[16 * q + 4 * k];
        ow[4 * k] = o4.x; ow[4 * k + 1] = o4.y; ow[4 * k + 2] = o4.z; ow[4 * k + 3] = o4.w;
      }
      float run = 0.f;
      int cur = -1, start = 0;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int r = 16 * q + k;
        const float v = lw[r * kGrRow + f];
        if (ow[k] != cur) {
          if (cur >= 0) lw[start * kGrRow + f] = run;     // a row this lane has already read
          cur = ow[k];
          start = r;
          run = 0.f;
        }
        run += v;
      }
      if (cur >= 0) lw[start * kGrRow + f] = run;
    }
    wave_lds_sync();
    if (need) {
      const int a = (int)((e0 > w0 ? e0 : w0) - w0);
      const int b = (int)((e1 < w0 + kGrWindow ? e1 : w0 + kGrWindow) - w0);
      if (a < b) {
        for (int qq = a >> 4; qq <= (b - 1) >> 4; ++qq) {
          const int r = a > 16 * qq ? a : 16 * qq;        // the first row of this lane's run in quarter qq
          const float4* row = (const float4*)&lw[r * kGrRow];
#pragma unroll
          for (int f4 = 0; f4 < kGradFields / 4; ++f4) {
            const float4 v = row[f4];
            s[f4].x += v.x; s[f4].y += v.y; s[f4].z += v.z; s[f4].w += v.w;
          }
        }
      }
    }
    wave_lds_sync();
  }
  if (need) {
    float4* dst = (float4*)(grads + (size_t)e0 * kGradFields);
#pragma unroll
    for (int f4 = 0; f4 < kGradFields / 4; ++f4) dst[f4] = s[f4];
  }
}

template <int DEG>
__global__ __launch_bounds__(kPbThreads) void k_project_bwd(ProjectBwdArgs a) {
  __shared__ float s_sh[kPbThreads * kMaxShCoeffs * 3];
  __shared__ float s_small[kPbThreads * 11];        // dmu 3, ds 3, dq 4, do 1
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t row0 = (int64_t)blockIdx.x * blockDim.x;
  const int rows = (int)((a.n - row0) < kPbThreads ? (a.n - row0) : kPbThreads);
  constexpr int K = (DEG + 1) * (DEG + 1);
  constexpr int K3 = 3 * K;
  constexpr int deg = DEG;
  if (i < a.n) {
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
  float dsh[K3];
#pragma unroll
  for (int k = 0; k < K3; ++k) dsh[k] = 0.f;

  bool touched = false;                     // some camera has an instance of this Gaussian
  for (int c = 0; c < a.n_cams; ++c) {
    const int64_t vg = (int64_t)c * a.n + i;
    const int cnt = a.counts[vg];
    if (cnt == 0) continue;
    touched = true;
    // the sum over this camera's instances, left in the first one's slot by k_grad_reduce
    // (none when the instances were dropped at the capacity)
    const int64_t e0 = a.offsets[vg];
    float gsum[kGradFields];
#pragma unroll
    for (int f4 = 0; f4 < kGradFields; ++f4) gsum[f4] = 0.f;
    if (e0 < kinst) {
      const float4* src = (const float4*)(a.grads + (size_t)e0 * kGradFields);
#pragma unroll
      for (int f4 = 0; f4 < kGradFields / 4; ++f4) {
        const float4 v = src[f4];
        gsum[4 * f4] = 0.f + v.x; gsum[4 * f4 + 1] = 0.f + v.y; gsum[4 * f4 + 2] = 0.f + v.z;
        gsum[4 * f4 + 3] = 0.f + v.w;
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
#pragma unroll
    for (int k = 0; k < K; ++k) {
      cr = fmaf(Y[k], f[3 * k], cr);
      cg = fmaf(Y[k], f[3 * k + 1], cg);
      cb = fmaf(Y[k], f[3 * k + 2], cb);
    }
    const float gc[3] = {cr > 0.f ? gsum[10] : 0.f, cg > 0.f ? gsum[11] : 0.f, cb > 0.f ? gsum[12] : 0.f};
    float wk[kMaxShCoeffs];
#pragma unroll
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
  float* sm = s_small + threadIdx.x * 11;
  // an untouched Gaussian (culled everywhere, possibly for non-finite parameters) gets exact
  // zeros rather than 0 times its own non-finite chain-rule factors
  for (int k = 0; k < 3; ++k) {
    sm[k] = touched ? (float)dmu[k] : 0.f;
    sm[3 + k] = touched ? (float)ds[k] : 0.f;
  }
  for (int k = 0; k < 4; ++k) sm[6 + k] = touched ? (float)((dq[k] - qv[k] * qd) / qnorm) : 0.f;
  sm[10] = touched ? (float)dop : 0.f;
#pragma unroll
  for (int k = 0; k < K3; ++k) s_sh[threadIdx.x * K3 + k] = touched ? dsh[k] : 0.f;
  }
  __syncthreads();
  if (rows <= 0) return;
  // coalesced write-out of the block's rows
  for (int k = threadIdx.x; k < rows * 3; k += kPbThreads) {
    const int r = k / 3, c = k - 3 * r;
    a.d_means[row0 * 3 + k] = s_small[r * 11 + c];
    a.d_scales[row0 * 3 + k] = s_small[r * 11 + 3 + c];
  }
  for (int k = threadIdx.x; k < rows * 4; k += kPbThreads) a.d_quats[row0 * 4 + k] = s_small[(k >> 2) * 11 + 6 + (k & 3)];
  for (int k = threadIdx.x; k < rows; k += kPbThreads) a.d_opac[row0 + k] = s_small[k * 11 + 10];
  store_rows(s_sh, a.d_sh, row0, rows, K3);
}

hipError_t launch_project_bwd(const ProjectBwdArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  const int64_t vn = a.n * a.n_cams;
  hipLaunchKernelGGL(k_grad_reduce, dim3((unsigned)div_up(vn, kGrThreads)), dim3(kGrThreads), 0, s, a.counts,
                     a.offsets, a.count_total, a.cap, vn, a.grads);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int th = kPbThreads;
  const dim3 grid((unsigned)div_up(a.n, th)), block(th);
  switch (a.sh_degree) {
    case 0: hipLaunchKernelGGL(k_project_bwd<0>, grid, block, 0, s, a); break;
    case 1: hipLaunchKernelGGL(k_project_bwd<1>, grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_project_bwd<2>, grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL(k_project_bwd<3>, grid, block, 0, s, a); break;
  }
  return hipGetLastError();
}

}  // namespace sof
