// Opacity field at the rendered depth (Sec. 3.3, direct opacity-field supervision): for each
// pixel with a 0.5 crossing, O_N(x) at x = o + t_r d, t_r the depth the forward wrote, over
// the Gaussians that pixel blends, each evaluated at min(t*, t_r) as in Eq. (12).  Whether a
// Gaussian peaks in front of x is only known once t_r is, so this is a second pass that
// replays the forward's per-pixel order (same tile lists, candidate test and window).  As in
// the paper, O_N = O_k + T_k sum_{i >= k} alpha_i prod_{k <= j < i} (1 - alpha_j): when the
// forward ran with the loss outputs it already accumulated the factor from the crossing
// Gaussian k on (1 - that sum = prod_{i >= k} (1 - alpha_i(x))), and this pass visits only
// the Gaussians in front of k; without them it replays the whole blended sequence.  Only
// products are accumulated (O_N does not depend on the order, App. A.2).  With the forward's
// recorded blend order (LIST) the pass reads the blended Gaussians' list positions instead of
// replaying the candidate test and the window; tiles the forward flagged are replayed.
#include "launch.h"
#include "render_common.h"

namespace sof {

// Eight waves per SIMD for windows up to 8 (64 VGPRs, 5 spilled): 1.06 -> 1.00 ms at 1080p.
template <int TS, int W, bool LIST>
__global__ __launch_bounds__(TS * TS, W <= 8 ? 8 : 1) void k_render_opa(RenderOpaArgs A) {
  constexpr int NT = TS * TS;
  constexpr int B = NT < 256 ? NT : 256;
  __shared__ StageEntry stage[LIST ? 1 : B];
  __shared__ uint2 srect[LIST ? 1 : B];
  __shared__ int32_t gring[LIST ? 2 * B : 1];          // Gaussian of the last two batches' positions
  const RenderFwdArgs& a = A.f;
  const int tile = blockIdx.x;
  if (a.order) {
    if (LIST == (a.order_flags[tile] != 0)) return;   // the other kernel's tile
  }
  const int c = find_cam(a.cam_info, a.n_cams, tile);
  const CamInfo ci = a.cam_info[c];
  const sof_camera& cam = a.cams[c];
  const int width = cam.width, height = cam.height;
  const int lt = tile - ci.tile_off;
  const int tx = lt % ci.tiles_x, ty = lt / ci.tiles_x;
  int lx, ly;
  lane_pixel<TS>((int)threadIdx.x, lx, ly);
  const int x0 = tx * TS, y0 = ty * TS;
  const int px = x0 + lx, py = y0 + ly;
  const int sx = x0 + (lx & ~7), sy = y0 + (ly & ~7);
  const int sxu = __builtin_amdgcn_readfirstlane(sx), syu = __builtin_amdgcn_readfirstlane(sy);
  const bool inside = px < width && py < height;
  const int2 rg = a.ranges[tile];
  const int64_t cam_base = (int64_t)c * a.n;
  const float near_plane = a.near_plane;

  // per pixel: the forward's blend count, crossing and depth (as a view z along this ray)
  const int64_t hw = (int64_t)width * height;
  const int64_t pix = (int64_t)py * width + px;
  int n_emit = 0, kgid = -1;
  float s_r = 0.f, tail = 1.f;
  if (inside) {
    const float* aux = a.aux + kAuxChannels * ci.pix_off;
    n_emit = __float_as_int(aux[hw + pix]);
    kgid = __float_as_int(aux[2 * hw + pix]);
    if (A.tail) {                                        // stop in front of k; the rest is known
      const float* L = A.tail + kLossChannels * ci.pix_off;
      tail = L[4 * hw + pix];
      n_emit = __float_as_int(L[5 * hw + pix]);
    }
    const float rx = (px + 0.5f - cam.cx) / cam.fx, ry = (py + 0.5f - cam.cy) / cam.fy;
    const float dn = sqrtf(fmaf(rx, rx, fmaf(ry, ry, 1.f)));
    s_r = a.depth[ci.pix_off + pix] / dn;
  }
  float P = 1.f;                       // prod (1 - alpha_j(x)) over the counted Gaussians
  int emitted = 0;
  bool done = !inside || kgid < 0 || n_emit <= 0;     // (k first in the order: nothing in front)
  Window<W> win;
  win.init();

  // window payload: key = peak view z s*, a = unclamped o G*, t = bits of A (= d^T P d)
  auto count = [&](float sstar, float araw, uint32_t abits) {
    float ax = fminf(kAlphaMax, araw);
    bool keep = true;                                    // a candidate: alpha >= 1/255, s* > near
    if (sstar > s_r) {                                   // peak beyond x: evaluate at x
      const float ds = s_r - sstar;
      ax = fminf(kAlphaMax, araw * __builtin_amdgcn_exp2f(-kHalfLog2e * __uint_as_float(abits) * ds * ds));
      keep = ax >= kAlphaMin && s_r > near_plane;
    }
    P = keep ? P * (1.f - ax) : P;
    if (++emitted >= n_emit) done = true;
  };

  if constexpr (LIST) {
    // the recorded order (as in the backward): per batch, each lane counts its next blended
    // Gaussians whose list position lies in the staged batches, evaluated from the record as the
    // candidate test and the window payload are (same offset, quadric, reciprocal and exp2)
    const uint16_t* recw =
        a.order + ((int64_t)tile * (NT / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) * a.order_slots * 64 +
        (threadIdx.x & 63);
    const int len = rg.y - rg.x;
    const int n_rec = done ? 0 : min(n_emit, a.order_slots);
    int kd = 0;
    uint32_t nxt = n_rec > 0 ? (uint32_t)recw[0] : 0xFFFFFFFFu;
    int cur_b = -1;
    for (int bs = rg.x; bs < rg.y; bs += B) {
      if (__syncthreads_count(kd < n_rec) == 0) break;
      ++cur_b;
      const int i = bs + (int)threadIdx.x;
      if (threadIdx.x < B && i < rg.y) gring[(i - rg.x) % (2 * B)] = a.gid[a.vals[i]];
      __syncthreads();
      const uint32_t lim = (uint32_t)min((cur_b + 1) * B, len);
      while (kd < n_rec && nxt < lim) {
        const int pos = (int)nxt;
        ++kd;
        nxt = kd < n_rec ? (uint32_t)recw[(int64_t)kd * 64] : 0xFFFFFFFFu;
        int32_t g = gring[pos % (2 * B)];
        __asm__ volatile("" : "+v"(g));                  // keep the LDS read apart from the list read
        if (pos < (cur_b - 1) * B) g = a.gid[a.vals[rg.x + pos]];
        const int64_t vg = cam_base + g;
        const float4 r0 = a.geom[4 * vg], r1 = a.geom[4 * vg + 1], r2 = a.geom[4 * vg + 2], r3 = a.geom[4 * vg + 3];
        const float2 d = pixel_offset(r0, px, py);
        const Quad q = quad_terms(r1.x, r1.y, r1.z, r1.w, r2.x, r2.y, r2.z, r2.w, d.x, d.y);
        const float r = __builtin_amdgcn_rcpf(q.den);
        const float x = fmaxf(q.num * r, 0.f);
        count(r3.x * (1.f + q.b) * r, r3.y * __builtin_amdgcn_exp2f(-x), __float_as_uint(r3.w * q.den));
      }
    }
  } else {
    for (int bs = rg.x; bs < rg.y; bs += B) {
      if (__syncthreads_count(!done) == 0) break;
      const int i = bs + (int)threadIdx.x;
      if (threadIdx.x < B && i < rg.y) {
        const int32_t g = a.gid[a.vals[i]];
        const int64_t vg = cam_base + g;
        stage_entry(a.geom, a.rect, vg, x0, y0, 0u, &stage[threadIdx.x], &srect[threadIdx.x]);
        stage[threadIdx.x].tag = a.geom[4 * vg + 3].w;     // the record's a = dm^T P dm
      }
      __syncthreads();
      const int nb = min(B, rg.y - bs);
      for (int j = 0; j < nb; ++j) {
        if (!__any(!done)) break;
        if (misses_subtile(uniform_rect(srect[j]), sxu, syu)) continue;
        const StageEntry e = stage[j];
        const Cand1 c1 = candidate_stage1(e, lx, ly, near_plane);
        if (!__any(c1.pre && !done)) continue;
        float key, al;
        const bool cand = candidate_stage2(e, c1, key, al) && !done;
        if (!__any(cand)) continue;
        if (cand) {
          const float x = fmaxf(c1.q.num * __builtin_amdgcn_rcpf(c1.q.den), 0.f);
          const float araw = e.o * __builtin_amdgcn_exp2f(-x);
          float ea, ek;
          uint32_t et;
          if (win.push(key, araw, __float_as_uint(e.tag * c1.q.den), ea, et, ek)) count(ek, ea, et);
        }
      }
    }
    if constexpr (W > 0) {
      while (!done && win.count > 0) {
        float ea, ek;
        uint32_t et;
        win.pop_front(ea, et, ek);
        count(ek, ea, et);
      }
    }
  }
  if (!inside) return;
  A.opa[ci.pix_off + pix] = kgid >= 0 ? 1.f - P * tail : 0.f;
}

// With a recorded order: the order-reading kernel over the recorded tiles, then the replay
// over the flagged ones (each leaves the other's tiles at once).
template <int TS>
static hipError_t launch_opa_ts(const RenderOpaArgs& a, int window, int64_t n_tiles, hipStream_t s) {
  const dim3 grid((unsigned)n_tiles), block(TS * TS);
  if (a.f.order) {
    hipLaunchKernelGGL((k_render_opa<TS, 0, true>), grid, block, 0, s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  switch (window) {
    case 0: hipLaunchKernelGGL((k_render_opa<TS, 0, false>), grid, block, 0, s, a); break;
    case 1: hipLaunchKernelGGL((k_render_opa<TS, 1, false>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_render_opa<TS, 2, false>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_render_opa<TS, 4, false>), grid, block, 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_render_opa<TS, 8, false>), grid, block, 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_render_opa<TS, 16, false>), grid, block, 0, s, a); break;
    case 32: hipLaunchKernelGGL((k_render_opa<TS, 32, false>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_render_opa(const RenderOpaArgs& a, int tile, int window, int64_t n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  switch (tile) {
    case 8: return launch_opa_ts<8>(a, window, n_tiles, s);
    case 16: return launch_opa_ts<16>(a, window, n_tiles, s);
    case 32: return launch_opa_ts<32>(a, window, n_tiles, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sof
