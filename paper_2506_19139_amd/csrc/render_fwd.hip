// Forward rasteriser: one workgroup per screen tile (TS x TS lanes, one pixel per lane).
// The tile's list is staged through LDS in batches of up to 128 entries with one coalesced
// 64-byte record load per lane; every lane then walks the batch from LDS (broadcast reads),
// tests candidates, feeds its register window and blends what the window emits front to
// back (Eq. (1)).  The workgroup leaves the list once no lane is still accumulating.
// Outputs per pixel: colour, accumulated opacity, exact depth (Sec. 3.2), normal, the
// replay state the backward pass needs and two work counters (list entries tested,
// candidates that passed the alpha cut); optionally the blend order itself (the list
// position of every blended Gaussian), which spares the backward the replay.
#include "render_common.h"

namespace sof {

struct PixFwd {
  float T, r, g, b, nx, ny, nz, Tk;
  float A, mu, M, E;         // losses only: sum w, weighted mean and central second moment of
                             // d = NDC(t*) (updated one Gaussian at a time), sum w extent
  float sr, Pt;              // losses only: view z of the rendered depth on this ray and the
                             // product of (1 - alpha_i(x)) from the crossing Gaussian on
  int n_emit, k, kpos, walked, cands;   // kpos: position of k in the blend order
  bool done;
};

// Output depth of the crossing Gaussian (record r3, quadric terms q at this pixel, T_k):
// the exact depth of the 0.5 level set (Sec. 3.2, App. A.3), or t*_k with SOF_DEPTH_MEDIAN.
__device__ inline float crossing_depth(const float4& r3, const Quad& q, float Tk, float dn, uint32_t flags) {
  const float sstar = r3.x * (1.f + q.b) / q.den;
  if (flags & SOF_DEPTH_MEDIAN) return dn * sstar;
  const float x = fmaxf(q.num / q.den, 0.f);                 // K q*
  const float g = (Tk - 0.5f) / (Tk * r3.y);
  const float L = fmaxf(2.f * (-x * kLn2 - logf(g)), 0.f);  // 2 ln(G*/g)
  const float A = r3.w * q.den;                              // d^T P d, d = (x_n, y_n, 1)
  return dn * (sstar - sqrtf(L / A));
}

// Blends Gaussian `gid` with colour c and normal nn; returns the blend weight (0 when the
// Gaussian was not blended).
__device__ inline float blend(PixFwd& p, float alpha, uint32_t gid, const float4& c, const float4& nn) {
  const float test_T = p.T * (1.f - alpha);
  if (test_T < kTMin) {
    p.done = true;
    return 0.f;
  }
  const float w = alpha * p.T;
  p.r = fmaf(w, c.x, p.r);
  p.g = fmaf(w, c.y, p.g);
  p.b = fmaf(w, c.z, p.b);
  p.nx = fmaf(w, nn.x, p.nx);
  p.ny = fmaf(w, nn.y, p.ny);
  p.nz = fmaf(w, nn.z, p.nz);
  if (p.k < 0 && test_T <= 0.5f) {
    p.k = (int)gid;
    p.kpos = p.n_emit;
    p.Tk = p.T;
  }
  p.T = test_T;
  ++p.n_emit;
  return w;
}

// Distortion and extent terms of one blended Gaussian (Sec. 3.3; App. C.1, C.2): its NDC
// depth d = NDC(t*) and the extent e = eps / t*^2 of its 1/255 contour along the ray,
// eps = sqrt((E^2 - q*) / A) on the unit ray; in the stored view-z units
// e = sqrt((E^2 - q*) / A_s) / (|d~| s*^2) with A_s = d~^T P d~.
//
// The same pass accumulates the tail of the opacity field at the rendered depth (Sec. 3.3,
// direct opacity-field supervision): once the crossing Gaussian k is blended, its depth is
// known, and from k on every blended Gaussian's alpha at x = o + t_r d (t_eval = min(t*,
// t_r), the 1/255 and near-plane rules of Eq. (12)) multiplies Pt = prod_{i >= k} (1 -
// alpha_i(x)); the second pass then needs only the Gaussians in front of k.
__device__ inline void loss_terms(PixFwd& p, float w, float sstar, const float4& r0, const float4& r1, const float4& r2,
                                  const float4& r3, int px, int py, float dn, bool crossed_here, uint32_t flags,
                                  float near_plane) {
  const float2 d2 = pixel_offset(r0, px, py);
  const Quad q = quad_terms(r1.x, r1.y, r1.z, r1.w, r2.x, r2.y, r2.z, r2.w, d2.x, d2.y);
  // hardware reciprocals (1 ulp): these values only enter the losses, never a decision
  // E^2 - q* = 2 ln 2 (log2(255 o) - x*): the record keeps log2(255 o) (the 1/255 cut)
  const float xs = fmaxf(q.num * __builtin_amdgcn_rcpf(q.den), 0.f);
  if (crossed_here) p.sr = crossing_depth(r3, q, p.Tk, dn, flags) / dn;   // as the stored depth / |d~|
  if (p.k >= 0) {
    // alpha at x: at the peak (the blend alpha) when it lies in front of x, else at x
    const float araw = r3.y * __builtin_amdgcn_exp2f(-xs);
    float ax = fminf(kAlphaMax, araw);
    bool keep = true;
    if (sstar > p.sr) {
      const float ds = p.sr - sstar;
      ax = fminf(kAlphaMax, araw * __builtin_amdgcn_exp2f(-kHalfLog2e * (r3.w * q.den) * ds * ds));
      keep = ax >= kAlphaMin && p.sr > near_plane;
    }
    p.Pt = keep ? p.Pt * (1.f - ax) : p.Pt;
  }
  const float u = (2.f * kLn2) * fmaxf(r3.z - xs, 0.f);
  const float t = dn * sstar, it = __builtin_amdgcn_rcpf(t);
  const float e = sqrtf(u * __builtin_amdgcn_rcpf(r3.w * q.den)) * it * __builtin_amdgcn_rcpf(sstar);
  const float d = (kNdcFar / (kNdcFar - kNdcNear)) * (t - kNdcNear) * it;
  // weighted running mean and second moment (numerically stable; the distortion
  // sum_ij w_i w_j (d_i - d_j)^2 = 2 A sum w (d - mean)^2 would cancel as 2 (A DD - D^2))
  p.A += w;
  const float delta = d - p.mu;
  p.mu = fmaf(w * __builtin_amdgcn_rcpf(p.A), delta, p.mu);
  p.M = fmaf(w * delta, d - p.mu, p.M);
  p.E = fmaf(w, e, p.E);
}

// Depth of the crossing Gaussian and the per-pixel output writes.
template <bool LOSS>
__device__ inline void write_pixel(const RenderFwdArgs& a, const PixFwd& p, const sof_camera& cam, const CamInfo& ci,
                                   int64_t cam_base, int px, int py) {
  const int width = cam.width, height = cam.height;
  // exact depth of the 0.5 level set on the crossing Gaussian (Sec. 3.2, App. A.3)
  const float rx = (px + 0.5f - cam.cx) / cam.fx, ry = (py + 0.5f - cam.cy) / cam.fy;
  const float dn = sqrtf(fmaf(rx, rx, fmaf(ry, ry, 1.f)));
  float depth = 0.f;
  if (p.k >= 0) {
    const int64_t vg = cam_base + p.k;
    const float4 r0 = a.geom[4 * vg], r1 = a.geom[4 * vg + 1], r2 = a.geom[4 * vg + 2], r3 = a.geom[4 * vg + 3];
    const float2 d = pixel_offset(r0, px, py);
    const Quad q = quad_terms(r1.x, r1.y, r1.z, r1.w, r2.x, r2.y, r2.z, r2.w, d.x, d.y);
    depth = crossing_depth(r3, q, p.Tk, dn, a.flags);
  }
  const int64_t hw = (int64_t)width * height;
  const int64_t pix = (int64_t)py * width + px;
  const float T = p.T;
  if (a.rgb) {
    float* o = a.rgb + 3 * ci.pix_off;
    o[pix] = fmaf(a.bg[0], T, p.r);
    o[hw + pix] = fmaf(a.bg[1], T, p.g);
    o[2 * hw + pix] = fmaf(a.bg[2], T, p.b);
  }
  if (a.acc) a.acc[ci.pix_off + pix] = 1.f - T;
  if (a.depth) a.depth[ci.pix_off + pix] = depth;
  if (a.normal) {
    float* o = a.normal + 3 * ci.pix_off;
    o[pix] = p.nx;
    o[hw + pix] = p.ny;
    o[2 * hw + pix] = p.nz;
  }
  if (a.aux) {
    float* o = a.aux + kAuxChannels * ci.pix_off;
    o[pix] = T;
    o[hw + pix] = __int_as_float(p.n_emit);
    o[2 * hw + pix] = __int_as_float(p.k);
    o[3 * hw + pix] = p.Tk;
    o[4 * hw + pix] = __int_as_float(p.walked);
    o[5 * hw + pix] = __int_as_float(p.cands);
  }
  if constexpr (LOSS) {
    // distortion sum_ij w_i w_j (d_i - d_j)^2 = 2 A M; extent f n / (f - n) sum w e
    float* o = a.losses + kLossChannels * ci.pix_off;
    o[pix] = 2.f * p.A * p.M;
    o[hw + pix] = kNdcFar * kNdcNear / (kNdcFar - kNdcNear) * p.E;
    o[2 * hw + pix] = p.mu;
    o[3 * hw + pix] = p.M;
    o[4 * hw + pix] = p.Pt;
    o[5 * hw + pix] = __int_as_float(p.k >= 0 ? p.kpos : -1);
  }
}

// Kernel variants: the plain forward, the forward with the loss moments, and the forward
// that also writes the per-pixel order (debug output of sof_render_order; the same code
// with stores added, so its decisions are those of the plain forward).
enum FwdMode { kFwdPlain = 0, kFwdLoss = 1, kFwdDump = 2 };

// Six waves per SIMD (80 VGPRs) for windows up to 8: seven (72 VGPRs) spill the blend
// accumulators (1.81 vs 1.25 ms at 1080p), five measure 1.33 ms; four (128 VGPRs) for a
// window of 16 (no spills).  8x8 tiles (held by LDS to four one-wave workgroups per SIMD), a
// window of 32 and the variants with the loss moments or the order output keep the default.
template <int TS, int W, int MODE>
__global__ __launch_bounds__(TS * TS, (MODE != kFwdPlain || TS < 16) ? 1 : (W <= 8 ? 6 : (W == 16 ? 4 : 1)))
    void k_render_fwd(RenderFwdArgs a) {
  constexpr bool LOSS = MODE == kFwdLoss;
  constexpr bool DUMP = MODE == kFwdDump;
  // the window's tag: the entry's list position, from which the recorded order is written,
  // except in the order output, which reports Gaussian indices.  With positions, the Gaussian
  // index, colour and normal of the last two batches' entries are kept in LDS rings, so that
  // a blend reads them there (an older entry, rare, is looked up in the list and gathered)
  constexpr bool POS = !DUMP;
  constexpr int NT = TS * TS;
  constexpr int B = NT < 128 ? NT : 128;         // list entries staged per batch
  constexpr int NR = POS ? 2 * B : 1;            // ring entries
  __shared__ StageEntry stage[B];
  __shared__ uint2 srect[B];
  __shared__ int32_t gring[NR];
  __shared__ float4 aring[2 * NR];               // colour, normal
  __shared__ float4 lring[LOSS ? 4 * NR : 1];    // geometry record (the loss terms read it)
  const int tile = blockIdx.x;
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
  const int sx = x0 + (lx & ~7), sy = y0 + (ly & ~7);     // this wave's 8x8 sub-tile
  const int sxu = __builtin_amdgcn_readfirstlane(sx), syu = __builtin_amdgcn_readfirstlane(sy);
  const bool inside = px < width && py < height;
  const int2 rg = a.ranges[tile];
  const int64_t cam_base = (int64_t)c * a.n;
  const float near_plane = a.near_plane;

  PixFwd p;
  p.T = 1.f; p.r = p.g = p.b = 0.f; p.nx = p.ny = p.nz = 0.f; p.Tk = 0.f; p.n_emit = 0; p.k = -1; p.kpos = -1;
  p.A = p.mu = p.M = p.E = 0.f;
  p.sr = 0.f;
  p.Pt = 1.f;
  float dn = 1.f;
  if constexpr (LOSS) {
    const float rx = (px + 0.5f - cam.cx) / cam.fx, ry = (py + 0.5f - cam.cy) / cam.fy;
    dn = sqrtf(fmaf(rx, rx, fmaf(ry, ry, 1.f)));
  }
  p.walked = 0; p.cands = 0;
  p.done = !inside;
  Window<W> win;
  win.init();
  // order output: this pixel's slot (-1: none), candidates fed to the window and entries
  // that left it
  int64_t dslot = -1;
  int n_fed = 0, n_out = 0;
  if constexpr (DUMP) {
    if (inside) {
      const int32_t sl = a.dump.slot[ci.pix_off + (int64_t)py * width + px];
      if (sl >= 0 && sl < a.dump.n_slots) dslot = sl;
    }
  }
  auto record_fed = [&](uint32_t tag, float key) {
    if constexpr (DUMP) {
      if (dslot >= 0) {
        if (n_fed < a.dump.max_entries) {
          a.dump.stream_ids[dslot * a.dump.max_entries + n_fed] = (int32_t)tag;
          a.dump.stream_keys[dslot * a.dump.max_entries + n_fed] = key;
        }
        ++n_fed;
      }
    }
  };
  auto record_out = [&](uint32_t tag) {
    if constexpr (DUMP) {
      if (dslot >= 0) {
        if (n_out < a.dump.max_entries) a.dump.emit_ids[dslot * a.dump.max_entries + n_out] = (int32_t)tag;
        ++n_out;
      }
    }
  };

  // recorded order: this wave's rows (row e = each lane's e-th blended Gaussian; a
  // wave-uniform base, the lane's column added at the store)
  uint16_t* recw = nullptr;
  if constexpr (POS) {
    if (a.order)
      recw = a.order + ((int64_t)tile * (NT / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) * a.order_slots * 64;
  }
  int cur_b = -1;
  // blend the entry that left the window (tag et, alpha ea, key ek)
  // (its Gaussian: the tag itself, or for a list position the ring entry of the last two
  // batches or, for an older entry, the list)
  auto emit = [&](uint32_t et, float ea, float ek) {
    record_out(et);
    uint32_t g = et;
    float4 cc, nn;
    if constexpr (POS) {
      const int r = (int)(et % NR);
      uint32_t g0 = (uint32_t)gring[r];
      float4 c0 = aring[2 * r], n0 = aring[2 * r + 1];
      // (the empty asm keeps the LDS reads here: sunk into the blend branch, they would merge
      // with the global reads below into generic loads)
      __asm__ volatile("" : "+v"(g0), "+v"(c0.x), "+v"(c0.y), "+v"(c0.z), "+v"(n0.x), "+v"(n0.y), "+v"(n0.z));
      if ((int)et < (cur_b - 1) * B) {
        g0 = (uint32_t)a.gid[a.vals[rg.x + (int)et]];
        c0 = a.app[2 * (cam_base + g0)];
        n0 = a.app[2 * (cam_base + g0) + 1];
      }
      g = g0;
      cc = c0;
      nn = n0;
    } else {
      cc = a.app[2 * (cam_base + g)];
      nn = a.app[2 * (cam_base + g) + 1];
    }
    const int k_before = p.k, n_before = p.n_emit;
    const float w = blend(p, ea, g, cc, nn);
    if constexpr (POS) {
      if (recw && p.n_emit > n_before && n_before < a.order_slots)
        recw[n_before * 64 + (int)(threadIdx.x & 63)] = (uint16_t)et;
    }
    if constexpr (LOSS) {
      if (w > 0.f) {
        const int r = (int)(et % NR);
        float4 r0 = lring[4 * r], r1 = lring[4 * r + 1], r2 = lring[4 * r + 2], r3 = lring[4 * r + 3];
        if ((int)et < (cur_b - 1) * B) {                 // older than the ring
          const int64_t vg = cam_base + g;
          r0 = a.geom[4 * vg]; r1 = a.geom[4 * vg + 1]; r2 = a.geom[4 * vg + 2]; r3 = a.geom[4 * vg + 3];
        }
        loss_terms(p, w, ek, r0, r1, r2, r3, px, py, dn, k_before < 0 && p.k >= 0, a.flags, near_plane);
      }
    }
  };

  for (int bs = rg.x; bs < rg.y; bs += B) {
    if (__syncthreads_count(!p.done) == 0) break;
    ++cur_b;
    const int i = bs + (int)threadIdx.x;
    if (threadIdx.x < B && i < rg.y) {
      const int32_t g = a.gid[a.vals[i]];
      stage_entry(a.geom, a.rect, cam_base + g, x0, y0, POS ? (uint32_t)(i - rg.x) : (uint32_t)g, &stage[threadIdx.x],
                  &srect[threadIdx.x]);
      if constexpr (POS) {
        const int r = (i - rg.x) % NR;
        gring[r] = g;
        aring[2 * r] = a.app[2 * (cam_base + g)];
        aring[2 * r + 1] = a.app[2 * (cam_base + g) + 1];
        if constexpr (LOSS) {
          const int64_t vg = cam_base + g;
#pragma unroll
          for (int k = 0; k < 4; ++k) lring[4 * r + k] = a.geom[4 * vg + k];
        }
      }
    }
    __syncthreads();
    const int nb = min(B, rg.y - bs);
    for (int j = 0; j < nb; ++j) {
      if (!__any(!p.done)) break;
      if (misses_subtile(uniform_rect(srect[j]), sxu, syu)) continue;      // wave-uniform
      const StageEntry e = stage[j];
      p.walked += p.done ? 0 : 1;
      const Cand1 c1 = candidate_stage1(e, lx, ly, near_plane);
      if (!__any(c1.pre && !p.done)) continue;
      float key, al;
      const bool cand = candidate_stage2(e, c1, key, al) && !p.done;
      if (!__any(cand)) continue;
      if (cand) {
        ++p.cands;
        float ea, ek;
        uint32_t et;
        record_fed(__float_as_uint(e.tag), key);
        if (win.push(key, al, __float_as_uint(e.tag), ea, et, ek)) emit(et, ea, ek);
      }
    }
  }
  if constexpr (W > 0) {
    while (!p.done && win.count > 0) {
      float ea, ek;
      uint32_t et;
      win.pop_front(ea, et, ek);
      emit(et, ea, ek);
    }
  }
  if constexpr (POS) {
    if (a.order) {
      const int over = __syncthreads_or(p.n_emit > a.order_slots);
      if (threadIdx.x == 0) a.order_flags[tile] = (over || rg.y - rg.x > kMaxOrderListLength) ? 1 : 0;
    }
  }
  if (!inside) return;
  if constexpr (DUMP) {
    if (dslot >= 0) {
      a.dump.counts[2 * dslot] = n_fed;
      a.dump.counts[2 * dslot + 1] = n_out;
    }
  }
  write_pixel<LOSS>(a, p, cam, ci, cam_base, px, py);
}

template <int TS, int MODE>
static hipError_t launch_fwd_tsl(const RenderFwdArgs& a, int window, int64_t n_tiles, hipStream_t s) {
  const dim3 grid((unsigned)n_tiles), block(TS * TS);
  switch (window) {
    case 0: hipLaunchKernelGGL((k_render_fwd<TS, 0, MODE>), grid, block, 0, s, a); break;
    case 1: hipLaunchKernelGGL((k_render_fwd<TS, 1, MODE>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_render_fwd<TS, 2, MODE>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_render_fwd<TS, 4, MODE>), grid, block, 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_render_fwd<TS, 8, MODE>), grid, block, 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_render_fwd<TS, 16, MODE>), grid, block, 0, s, a); break;
    case 32: hipLaunchKernelGGL((k_render_fwd<TS, 32, MODE>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int TS>
static hipError_t launch_fwd_ts(const RenderFwdArgs& a, int window, int64_t n_tiles, hipStream_t s) {
  if (a.dump.slot) return launch_fwd_tsl<TS, kFwdDump>(a, window, n_tiles, s);
  return a.losses ? launch_fwd_tsl<TS, kFwdLoss>(a, window, n_tiles, s) : launch_fwd_tsl<TS, kFwdPlain>(a, window, n_tiles, s);
}

bool render_supported(int tile, int window) {
  const bool w = window == 0 || window == 1 || window == 2 || window == 4 || window == 8 || window == 16 || window == 32;
  return w && (tile == 8 || tile == 16 || tile == 32);
}

hipError_t launch_render_fwd(const RenderFwdArgs& a, int tile, int window, int64_t n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  switch (tile) {
    case 8: return launch_fwd_ts<8>(a, window, n_tiles, s);
    case 16: return launch_fwd_ts<16>(a, window, n_tiles, s);
    case 32: return launch_fwd_ts<32>(a, window, n_tiles, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sof
