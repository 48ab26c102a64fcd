// Per (camera, Gaussian) preprocessing: liveness, the cancellation-free per-ray quadric
// constants (Sec. 3.1 Eq. (7)-(10), App. A.1), the opacity-aware bound E (Eq. (3)), the
// screen rectangle of the E-ellipsoid, colour (SH), normal and the z_min key (Eq. (15)).
//
// One thread per (camera, Gaussian); consecutive threads take consecutive Gaussians of one
// camera so that the parameter reads are coalesced.  The geometry is set up in float64 and
// stored in float32 (HBM-bound kernel: ~236 B read and ~140 B written per pair at SH 3).
#include "sof_internal.h"
#include "sh_eval.h"

namespace sof {

struct ProjectArgs {
  const float* means;
  const float* scales;
  const float* quats;
  const float* opac;
  const float* sh;
  int sh_degree;
  int64_t n;
  const sof_camera* cams;
  int n_cams;
  float near_plane;
  float4* geom;
  float4* app;
  float4* bwdr;
  short4* rect;
  float* zmin;
  float4* world;      // query layout only (else null): per-Gaussian S^-1 R^T rows and mean
  int query;          // 1: skip colour / normal / backward records
};

__device__ inline int clamp_floor(double v) {
  const double lim = 1.0e7;
  v = v < -lim ? -lim : (v > lim ? lim : v);
  return (int)floor(v);
}

// Templated on the SH degree so that the coefficient loop is unrolled and its loads are all in
// flight together (with a runtime degree each of its 16 iterations waited for its own load:
// 82 us at 1M Gaussians 1080p).  DEG < 0: the query layout (no colour).
template <int DEG>
__global__ __launch_bounds__(256) void k_project(ProjectArgs a) {
  const int64_t vn = a.n * (int64_t)a.n_cams;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= vn) return;
  const int c = (int)(idx / a.n);
  const int64_t i = idx - (int64_t)c * a.n;
  const sof_camera cam = a.cams[c];

  const float o = a.opac[i];
  const double mx = a.means[3 * i], my = a.means[3 * i + 1], mz_w = a.means[3 * i + 2];
  double Rc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) Rc[k] = cam.R[k];
  const double mcx = Rc[0] * mx + Rc[1] * my + Rc[2] * mz_w + cam.t[0];
  const double mcy = Rc[3] * mx + Rc[4] * my + Rc[5] * mz_w + cam.t[1];
  const double mcz = Rc[6] * mx + Rc[7] * my + Rc[8] * mz_w + cam.t[2];

  // a Gaussian with a non-finite or degenerate parameter (scale <= 0, zero quaternion) is
  // culled like a dead one, so that it can neither poison a pixel nor waste tile instances
  double qw = a.quats[4 * i], qx = a.quats[4 * i + 1], qy = a.quats[4 * i + 2], qz = a.quats[4 * i + 3];
  const double s0 = a.scales[3 * i], s1 = a.scales[3 * i + 1], s2 = a.scales[3 * i + 2];
  const double qq = qw * qw + qx * qx + qy * qy + qz * qz;
  const bool sane = isfinite(mcx) && isfinite(mcy) && isfinite(mcz) && isfinite(o) && s0 > 0.0 && s1 > 0.0 && s2 > 0.0 &&
                    isfinite(s0 * s1 * s2) && qq > 0.0 && isfinite(qq);
  const bool live = sane && (o >= kAlphaMin) && (mcz > (double)a.near_plane);
  if (!live) {
    a.rect[idx] = make_short4(0, 0, -1, -1);
    a.zmin[idx] = 0.f;
    return;
  }

  // rotation of the Gaussian and its camera-space frame T = Rc Rg
  const double qn = rsqrt(qq);
  qw *= qn; qx *= qn; qy *= qn; qz *= qn;
  double Rg[9];
  quat_rot<double>(qw, qx, qy, qz, Rg);
  double T[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) T[3 * r + k] = Rc[3 * r] * Rg[k] + Rc[3 * r + 1] * Rg[3 + k] + Rc[3 * r + 2] * Rg[6 + k];
  const double v0 = s0 * s0, v1 = s1 * s1, v2 = s2 * s2;
  const double w0 = 1.0 / v0, w1 = 1.0 / v1, w2 = 1.0 / v2;
  // Sigma_c = T diag(v) T^T, P = T diag(1/v) T^T (symmetric; index pairs 00 01 02 11 12 22)
  double S[6], P[6];
  {
    int p = 0;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int k = r; k < 3; ++k) {
        S[p] = T[3 * r] * T[3 * k] * v0 + T[3 * r + 1] * T[3 * k + 1] * v1 + T[3 * r + 2] * T[3 * k + 2] * v2;
        P[p] = T[3 * r] * T[3 * k] * w0 + T[3 * r + 1] * T[3 * k + 1] * w1 + T[3 * r + 2] * T[3 * k + 2] * w2;
        ++p;
      }
  }
  const double E = sqrt(2.0 * log(255.0 * (double)o));
  const double E2 = E * E;
  const double zmin = mcz - E * sqrt(S[5]);

  // ---- screen bound of the E-ellipsoid
  double xl, xh, yl, yh;
  if (zmin > (double)a.near_plane) {
    // exact silhouette: image of the dual quadric, N = mu mu^T - E^2 Sigma
    const double N00 = mcx * mcx - E2 * S[0], N02 = mcx * mcz - E2 * S[2];
    const double N11 = mcy * mcy - E2 * S[3], N12 = mcy * mcz - E2 * S[4];
    const double N22 = mcz * mcz - E2 * S[5];
    const double dx = sqrt(fmax(0.0, N02 * N02 - N00 * N22));
    const double dy = sqrt(fmax(0.0, N12 * N12 - N11 * N22));
    xl = (N02 - dx) / N22; xh = (N02 + dx) / N22;
    yl = (N12 - dy) / N22; yh = (N12 + dy) / N22;
  } else {
    // crosses the near plane: camera-space box clipped to z >= near, projected
    const double ex = E * sqrt(S[0]), ey = E * sqrt(S[3]), ez = E * sqrt(S[5]);
    const double z0 = (double)a.near_plane, z1 = mcz + ez;
    const double xa = mcx - ex, xb = mcx + ex, ya = mcy - ey, yb = mcy + ey;
    xl = fmin(fmin(xa / z0, xa / z1), fmin(xb / z0, xb / z1));
    xh = fmax(fmax(xa / z0, xa / z1), fmax(xb / z0, xb / z1));
    yl = fmin(fmin(ya / z0, ya / z1), fmin(yb / z0, yb / z1));
    yh = fmax(fmax(ya / z0, ya / z1), fmax(yb / z0, yb / z1));
  }
  int x0 = clamp_floor(cam.fx * xl + cam.cx) - 1, x1 = clamp_floor(cam.fx * xh + cam.cx) + 1;
  int y0 = clamp_floor(cam.fy * yl + cam.cy) - 1, y1 = clamp_floor(cam.fy * yh + cam.cy) + 1;
  x0 = max(x0, 0); y0 = max(y0, 0);
  x1 = min(x1, cam.width - 1); y1 = min(y1, cam.height - 1);
  if (x0 > x1 || y0 > y1) { x0 = 0; y0 = 0; x1 = -1; y1 = -1; }
  a.rect[idx] = make_short4((short)x0, (short)y0, (short)x1, (short)y1);
  a.zmin[idx] = (float)zmin;
  if (x1 < x0) return;   // off screen: nothing reads the records

  // ---- per-ray quadric constants relative to the projected centre
  const double iz = 1.0 / mcz;
  const double dmx = mcx * iz, dmy = mcy * iz;
  double u = cam.fx * dmx + cam.cx, v = cam.fy * dmy + cam.cy;
  const double lim = 1.0e9;
  u = fmin(fmax(u, -lim), lim);
  v = fmin(fmax(v, -lim), lim);
  const double ui = floor(u), vi = floor(v);
  // g = P dm, a = dm^T P dm, M = a P_xy - g_xy g_xy^T
  const double g0 = P[0] * dmx + P[1] * dmy + P[2];
  const double g1 = P[1] * dmx + P[3] * dmy + P[4];
  const double g2 = P[2] * dmx + P[4] * dmy + P[5];
  const double aa = dmx * g0 + dmy * g1 + g2;
  const double M00 = aa * P[0] - g0 * g0, M01 = aa * P[1] - g0 * g1, M11 = aa * P[3] - g1 * g1;
  const double ifx = 1.0 / cam.fx, ify = 1.0 / cam.fy;
  const double ia = 1.0 / aa;
  const double km = (double)kHalfLog2e * mcz * mcz * ia;
  float4 r0, r1, r2, r3;
  r0.x = __int_as_float((int)ui);
  r0.y = (float)(u - ui);
  r0.z = __int_as_float((int)vi);
  r0.w = (float)(v - vi);
  r1.x = (float)(g0 * ia * ifx);
  r1.y = (float)(g1 * ia * ify);
  r1.z = (float)(P[0] * ia * ifx * ifx);
  r1.w = (float)(2.0 * P[1] * ia * ifx * ify);
  r2.x = (float)(P[3] * ia * ify * ify);
  r2.y = (float)(km * M00 * ifx * ifx);
  r2.z = (float)(2.0 * km * M01 * ifx * ify);
  r2.w = (float)(km * M11 * ify * ify);
  r3.x = (float)mcz;
  r3.y = o;
  r3.z = (float)log2(255.0 * (double)o);
  r3.w = (float)aa;
  a.geom[4 * idx + 0] = r0;
  a.geom[4 * idx + 1] = r1;
  a.geom[4 * idx + 2] = r2;
  a.geom[4 * idx + 3] = r3;
  if (DEG < 0 || a.query) return;
  a.bwdr[2 * idx + 0] = make_float4((float)P[0], (float)P[1], (float)P[2], (float)P[3]);
  a.bwdr[2 * idx + 1] = make_float4((float)P[4], (float)P[5], (float)dmx, (float)dmy);

  // ---- colour: max(0, SH(dir) + 1/2), dir from the camera centre to the mean
  const double ccx = -(Rc[0] * cam.t[0] + Rc[3] * cam.t[1] + Rc[6] * cam.t[2]);
  const double ccy = -(Rc[1] * cam.t[0] + Rc[4] * cam.t[1] + Rc[7] * cam.t[2]);
  const double ccz = -(Rc[2] * cam.t[0] + Rc[5] * cam.t[1] + Rc[8] * cam.t[2]);
  double ddx = mx - ccx, ddy = my - ccy, ddz = mz_w - ccz;
  const double dn = rsqrt(ddx * ddx + ddy * ddy + ddz * ddz);
  float Y[kMaxShCoeffs];
  constexpr int deg = DEG < 0 ? 0 : DEG;
  sh_basis(deg, (float)(ddx * dn), (float)(ddy * dn), (float)(ddz * dn), Y);
  constexpr int K = (deg + 1) * (deg + 1);
  const float* f = a.sh + (size_t)i * K * 3;
  float cr = 0.5f, cg = 0.5f, cb = 0.5f;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    cr = fmaf(Y[k], f[3 * k], cr);
    cg = fmaf(Y[k], f[3 * k + 1], cg);
    cb = fmaf(Y[k], f[3 * k + 2], cb);
  }
  // ---- normal: rotation column of the smallest scale, facing the camera
  const int j = argmin3(s0, s1, s2);
  double nx = Rg[j], ny = Rg[3 + j], nz = Rg[6 + j];
  if (nx * (ccx - mx) + ny * (ccy - my) + nz * (ccz - mz_w) < 0.0) { nx = -nx; ny = -ny; nz = -nz; }
  a.app[2 * idx + 0] = make_float4(fmaxf(cr, 0.f), fmaxf(cg, 0.f), fmaxf(cb, 0.f), o);
  a.app[2 * idx + 1] = make_float4((float)nx, (float)ny, (float)nz, 0.f);
  if (!isfinite(cr + cg + cb)) a.rect[idx] = make_short4(0, 0, -1, -1);   // non-finite SH: culled too
}

// World record for point queries: row k of S^-1 R^T is (column k of R) / s_k.
__global__ __launch_bounds__(256) void k_world(const float* means, const float* scales, const float* quats, int64_t n,
                                               float4* world) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double qw = quats[4 * i], qx = quats[4 * i + 1], qy = quats[4 * i + 2], qz = quats[4 * i + 3];
  const double qn = rsqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  double R[9];
  quat_rot<double>(qw * qn, qx * qn, qy * qn, qz * qn, R);
  const double is0 = 1.0 / scales[3 * i], is1 = 1.0 / scales[3 * i + 1], is2 = 1.0 / scales[3 * i + 2];
  world[4 * i + 0] = make_float4((float)(R[0] * is0), (float)(R[3] * is0), (float)(R[6] * is0), (float)(R[1] * is1));
  world[4 * i + 1] = make_float4((float)(R[4] * is1), (float)(R[7] * is1), (float)(R[2] * is2), (float)(R[5] * is2));
  world[4 * i + 2] = make_float4((float)(R[8] * is2), means[3 * i], means[3 * i + 1], means[3 * i + 2]);
  world[4 * i + 3] = make_float4(0.f, 0.f, 0.f, 0.f);
}

hipError_t launch_project(const sof_gaussians* g, const sof_camera* d_cams, int n_cams, float near_plane,
                          void* proj, hipStream_t stream, bool query) {
  const int64_t vn = g->n * (int64_t)n_cams;
  if (vn == 0) return hipSuccess;
  ProjLayout L = ProjLayout::make(vn, query, g->n);
  char* base = (char*)proj;
  ProjectArgs a;
  a.means = g->means; a.scales = g->scales; a.quats = g->quats; a.opac = g->opacities; a.sh = g->sh;
  a.sh_degree = g->sh_degree; a.n = g->n; a.cams = d_cams; a.n_cams = n_cams; a.near_plane = near_plane;
  a.geom = (float4*)(base + L.geom);
  a.app = (float4*)(base + L.app);
  a.bwdr = (float4*)(base + L.bwdr);
  a.rect = (short4*)(base + L.rect);
  a.zmin = (float*)(base + L.zmin);
  a.world = query ? (float4*)(base + L.world) : nullptr;
  a.query = query ? 1 : 0;
  const int threads = 256;
  const int64_t blocks = div_up(vn, threads);
  const dim3 grid((unsigned)blocks), block(threads);
  if (query) hipLaunchKernelGGL(k_project<-1>, grid, block, 0, stream, a);
  else switch (a.sh_degree) {
    case 0: hipLaunchKernelGGL(k_project<0>, grid, block, 0, stream, a); break;
    case 1: hipLaunchKernelGGL(k_project<1>, grid, block, 0, stream, a); break;
    case 2: hipLaunchKernelGGL(k_project<2>, grid, block, 0, stream, a); break;
    default: hipLaunchKernelGGL(k_project<3>, grid, block, 0, stream, a); break;
  }
  if (query)
    hipLaunchKernelGGL(k_world, dim3((unsigned)div_up(g->n, threads)), dim3(threads), 0, stream, g->means, g->scales,
                       g->quats, g->n, a.world);
  return hipGetLastError();
}

}  // namespace sof
