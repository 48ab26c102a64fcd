// Backward rasteriser: the adjoint of render_fwd, without per-sample state.
//
// Each lane walks its pixel's forward order front to back: read from the order the forward
// recorded (the list position of every blended Gaussian), or, without it and for the tiles
// the forward could not record, replayed exactly (same staging, candidate test and window
// code).  It recomputes the transmittance T_j on the way.  Contributions behind j
// come from the stored totals: for F in {colour, normal}, dF/dalpha_j = T_j f_j -
// (F_total - F_<=j) / (1 - alpha_j); d acc / d alpha_j = T_end / (1 - alpha_j).
// The exact-depth correction (App. A.3) is either treated as a constant, as in the paper
// (d depth = |d| d s*_k), or differentiated fully (SOF_DEPTH_GRAD_FULL), which adds a term
// through T_k to every Gaussian in front of the crossing.
//
// Gradients are taken with respect to the camera-space mean mu_c and precision P_c of the
// emitted Gaussian: with r = mu_c - s* d the peak-to-mean offset,
//   dq*/dmu = 2 P r,  dq*/dP = r r^T,  ds*/dmu = P d / A,  ds*/dP = sym(d r^T) / A,
//   dA/dP = d d^T,  A = d^T P d, d = (x_n, y_n, 1).
// Per lane the 16 partials (dmu 3, dP 6, do, dcolour 3, dnormal 3) are added into LDS slots
// of the instance (two batches of slots stay resident); slots are written to the
// per-instance buffer once, in list order, and the rare emission of an entry older than
// two batches adds to the buffer atomically.  A separate kernel reduces the per-instance
// partials of each Gaussian in a fixed order.
#include "render_common.h"

namespace sof {

// Pending slots a lane may hold before a round is forced (see the emission loop).
template <int W>
constexpr int kPendingDepth = W >= 16 ? 1 : 4;

struct PixBwd {
  float T;
  float S;                        // prefix sum of w (g_c . c + g_n . n)
  bool crossed;
};

// Cross-lane read inside a row of 16 lanes (DPP, no LDS round trip).
constexpr int kDppRowMirror = 0x140;       // lane i reads lane 15 - i of its row
constexpr int kDppRowHalfMirror = 0x141;   // lane i reads lane 7 - i of its half-row (i ^ 7)
constexpr int kDppQuadXor2 = 0x4E;         // quad permutation (2, 3, 0, 1)
constexpr int kDppQuadXor1 = 0xB1;         // quad permutation (1, 0, 3, 2)
template <int CTRL>
__device__ inline float dpp_pull(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Sum over the lanes where `mine` holds of 16 per-lane fields; every lane of the wave must be
// active.  A reduce-scatter that halves the fields a lane carries at each stage, starting with
// the two cross-row exchanges of gfx950: a half-wave swap (lanes l and l ^ 32) adds field k
// of the pair in the lower half and field k + 8 in the upper half with one swap and one add
// per field pair, a swap of neighbouring rows (l and l ^ 16) does the same for the next bit,
// then two DPP stages inside each row (partners i ^ 15 and i ^ 7: bits 3 and 2 differ) and two
// plain quad sums.  On return lane l holds the wave total of field (l >> 2) & 15.
__device__ inline float wave_field_sums16(const float* gv, bool mine) {
  const int lane = (int)(threadIdx.x & 63);
  const bool b3 = (lane & 8) != 0, b2 = (lane & 4) != 0;
  float m[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) m[k] = mine ? gv[k] : 0.f;
  // lanes l, l ^ 32: the first operand's upper half is swapped with the second's lower half
  float s8[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(m[k]), __float_as_uint(m[k + 8]), false, false);
    s8[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  // lanes l, l ^ 16: odd rows of the first operand are swapped with even rows of the second
  float s4[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(s8[k]), __float_as_uint(s8[k + 4]), false, false);
    s4[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  float s2[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) s2[k] = (b3 ? s4[k + 2] : s4[k]) + dpp_pull<kDppRowMirror>(b3 ? s4[k] : s4[k + 2]);
  float s1 = (b2 ? s2[1] : s2[0]) + dpp_pull<kDppRowHalfMirror>(b2 ? s2[0] : s2[1]);
  s1 += dpp_pull<kDppQuadXor2>(s1);
  s1 += dpp_pull<kDppQuadXor1>(s1);
  return s1;
}

// Five waves per SIMD (96 VGPRs; LDS allows five 256-lane workgroups per CU) hide more of the
// gather latency than four; the variant with the optional opacity and loss terms gets four.
// Windows above 8 keep the default (their window registers would spill under either bound), and
// so do 8x8 tiles, whose one-wave workgroups are held to three waves per SIMD by LDS.
//
// LIST: the pixel's order is read from the forward's recorded order instead of being replayed
// (no staging, candidate test or window); the kernel then runs on the tiles whose order was
// recorded, the replay kernel on the others.
template <int TS, int W, bool EXT, bool LIST>
__global__ __launch_bounds__(TS * TS, (TS >= 16 && W <= 8) ? (EXT ? 4 : 5) : 1) void k_render_bwd(RenderBwdArgs A) {
  constexpr int NT = TS * TS;
  constexpr int B = NT < 128 ? NT : 128;         // list entries per batch
  constexpr int NS = 2 * B;                      // resident gradient slots (two batches)
  __shared__ StageEntry stage[LIST ? 1 : B];
  __shared__ uint2 srect[LIST ? 1 : B];
  constexpr int kSlotStride = kGradFields + 1;   // padded: fields of one slot and equal fields
                                                 // of neighbouring slots fall in distinct banks
  // lanes sharing an instance: reduce first (3 measured 2.62 against 2.69 ms with 4 at 1080p;
  // the variant with the loss and opacity terms keeps 4: 3.29 against 3.23 ms)
  constexpr int kGroupReduce = EXT ? 4 : 3;
  __shared__ float gsl[kSlotStride * NS];
  __shared__ uint2 ring[NS];                     // (emission index, Gaussian) of each resident list slot
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
  const int sx = x0 + (lx & ~7), sy = y0 + (ly & ~7);     // this wave's 8x8 sub-tile
  const int sxu = __builtin_amdgcn_readfirstlane(sx), syu = __builtin_amdgcn_readfirstlane(sy);
  const bool inside = px < width && py < height;
  const int2 rg = A.f.ranges[tile];
  const int len = rg.y - rg.x;
  const int64_t cam_base = (int64_t)c * a.n;
  const float near_plane = a.near_plane;
  const float ifx = 1.f / cam.fx, ify = 1.f / cam.fy;

  for (int s = threadIdx.x; s < kSlotStride * NS; s += NT) gsl[s] = 0.f;

  // ---- per-pixel forward state and upstream gradients
  const int64_t hw = (int64_t)width * height;
  const int64_t pix = (int64_t)py * width + px;
  float T_end = 1.f, Tk = 0.f;
  int n_emit = 0, kgid = -1;
  float G0 = 0.f;                 // g_c . C + g_n . N - g_acc T_end over the forward's totals
  float gr = 0, gg = 0, gb = 0, ga = 0, gd = 0, gnx = 0, gny = 0, gnz = 0;
  if (inside) {
    const float* aux = a.aux + kAuxChannels * ci.pix_off;
    T_end = aux[pix];
    n_emit = __float_as_int(aux[hw + pix]);
    kgid = __float_as_int(aux[2 * hw + pix]);
    Tk = aux[3 * hw + pix];
    const int64_t o3 = 3 * ci.pix_off;
    if (A.d_rgb) {
      gr = A.d_rgb[o3 + pix]; gg = A.d_rgb[o3 + hw + pix]; gb = A.d_rgb[o3 + 2 * hw + pix];
      G0 = gr * A.out_rgb[o3 + pix] + gg * A.out_rgb[o3 + hw + pix] + gb * A.out_rgb[o3 + 2 * hw + pix];
    }
    if (A.d_normal) {
      gnx = A.d_normal[o3 + pix]; gny = A.d_normal[o3 + hw + pix]; gnz = A.d_normal[o3 + 2 * hw + pix];
      G0 += gnx * A.out_normal[o3 + pix] + gny * A.out_normal[o3 + hw + pix] + gnz * A.out_normal[o3 + 2 * hw + pix];
    }
    if (A.d_acc) ga = A.d_acc[ci.pix_off + pix];
    if (A.d_depth) gd = A.d_depth[ci.pix_off + pix];
    G0 -= ga * T_end;
  }
  const float rx = (px + 0.5f - cam.cx) * ifx, ry = (py + 0.5f - cam.cy) * ify;
  const float dn = sqrtf(fmaf(rx, rx, fmaf(ry, ry, 1.f)));

  // ---- opacity at the rendered depth: x at view z s_r on this ray, dL/dalpha_j(x) =
  //      g_opa prod_{i != j} (1 - alpha_i(x)) = g_opa (1 - O_N) / (1 - alpha_j(x))
  float s_r = 0.f, gopaP = 0.f;
  bool opa_on = false;
  if constexpr (EXT) {
    if (A.d_opa && inside && kgid >= 0) {
      const float go = A.d_opa[ci.pix_off + pix];
      s_r = A.out_depth[ci.pix_off + pix] / dn;
      gopaP = go * (1.f - A.opa[ci.pix_off + pix]);
      opa_on = go != 0.f;
    }
  }

  // ---- distortion and extent losses: upstream gradients, the forward's totals A = sum w,
  //      mean mu and central moment M = sum w (d - mu)^2 of d = NDC(t*), E = sum w e, and
  //      running prefixes of w (d - mu)^2 and w e
  constexpr float kKappa = kNdcFar * kNdcNear / (kNdcFar - kNdcNear);
  float g_dist = 0.f, g_ext = 0.f, Atot = 0.f, mu = 0.f, Mtot = 0.f, Etot = 0.f;
  float Mp = 0.f, Ep = 0.f;
  bool loss_on = false;
  if constexpr (EXT) {
    if (A.d_losses && inside) {
      const float* L = A.losses + kLossChannels * ci.pix_off;
      g_dist = A.d_losses[2 * ci.pix_off + pix];
      g_ext = A.d_losses[2 * ci.pix_off + hw + pix];
      Atot = 1.f - T_end;
      Etot = L[hw + pix] / kKappa;
      mu = L[2 * hw + pix];
      Mtot = L[3 * hw + pix];
      loss_on = g_dist != 0.f || g_ext != 0.f;
    }
  }

  // ---- exact-depth terms of the crossing Gaussian (full mode)
  const bool full = (a.flags & SOF_DEPTH_GRAD_FULL) && !(a.flags & SOF_DEPTH_MEDIAN);
  float cT = 0.f, dq_k = 0.f, dA_k = 0.f, do_k = 0.f;
  if (full && inside && kgid >= 0 && gd != 0.f) {
    const int64_t vg = cam_base + kgid;
    const float4 r0 = a.geom[4 * vg], r1 = a.geom[4 * vg + 1], r2 = a.geom[4 * vg + 2], r3 = a.geom[4 * vg + 3];
    const float2 d = pixel_offset(r0, px, py);
    const Quad q = quad_terms(r1.x, r1.y, r1.z, r1.w, r2.x, r2.y, r2.z, r2.w, d.x, d.y);
    const float x = fmaxf(q.num / q.den, 0.f);
    const float g = (Tk - 0.5f) / (Tk * r3.y);
    const float L = fmaxf(2.f * (-x * kLn2 - logf(g)), 0.f);
    const float Am = r3.w * q.den;
    const float S = sqrtf(L / Am);
    if (S > 1e-7f * r3.x) {
      const float inv = gd * dn / (S * Am);
      cT = inv * (1.f / (Tk - 0.5f) - 1.f / Tk);
      dq_k = 0.5f * inv;
      dA_k = 0.5f * gd * dn * S / Am;
      do_k = -inv / r3.y;
    }
  }

  PixBwd p;
  p.T = 1.f; p.S = 0.f;
  p.crossed = false;
  Window<W> win;
  win.init();

  // Emission, in the forward's order.  The window holds (key, list slot) only: an entry that
  // leaves it is queued in a short per-lane FIFO of pending slots.  A round takes the oldest
  // pending slot of every lane that has one: it gathers the Gaussian, recomputes its alpha
  // (bit-identical to the candidate test: same pixel offset, quadric terms, reciprocal and
  // exp2), advances the transmittance and prefix sums and forms all partials, which are then
  // added wave-cooperatively, so lanes holding the same Gaussian are summed across the wave
  // before touching LDS.  A round costs the same whatever number of lanes take part, so rounds
  // are deferred until every lane that can still emit has a pending slot, or one lane's FIFO
  // is full; each lane still handles its slots in emission order.
  constexpr int D = kPendingDepth<W>;
  uint32_t fifo[D];              // pending list slots, oldest first
#pragma unroll
  for (int i = 0; i < D; ++i) fifo[i] = 0u;
  int nq = 0;                    // pending count
  int n_out = 0;                 // slots emitted so far (queued or done)
  bool has = false;              // this round's slot (fifo head) and its lane
  uint32_t qpos = 0u;
  uint32_t qe = 0u;              // its instance (emission index)
  int32_t qg = 0;                // and Gaussian (stale on lanes without a pending slot)
  auto queue = [&](uint32_t pos) {
#pragma unroll
    for (int i = 0; i < D; ++i) fifo[i] = nq == i ? pos : fifo[i];
    ++nq;
    ++n_out;
  };
  // the forward blended n_emit entries; the lane emits no more once that many have left
  auto emit_done = [&]() { return n_out >= n_emit; };

  // Gaussian of list slot `pos`: from the LDS ring while its batch is resident
  auto slot_gaussian = [&](uint32_t pos, int cur_b, uint32_t& e) -> int32_t {
    if ((int)pos >= (cur_b - 1) * B) {
      const uint2 r = ring[pos % NS];
      e = r.x;
      return (int32_t)r.y;
    }
    e = A.f.vals[rg.x + (int)pos];
    return A.f.gid[e];
  };

  // One emitted Gaussian: blend state, dL/dalpha, and the gradients with respect to mu_c,
  // P_c, the opacity, the colour and the normal.  `live` is false on lanes that compute on a
  // stale Gaussian only to keep the wave's control flow uniform: their state is left as is.
  auto adjoint = [&](bool live, float* gv) {
    const int64_t vg = cam_base + qg;
    const float4 r0 = a.geom[4 * vg], r1 = a.geom[4 * vg + 1], r2 = a.geom[4 * vg + 2], r3 = a.geom[4 * vg + 3];
    const float4 p0 = A.bwdr[2 * vg], p1 = A.bwdr[2 * vg + 1];
    const float4 col = a.app[2 * vg], nrm = a.app[2 * vg + 1];
    const float2 dd = pixel_offset(r0, px, py);
    const float dx = dd.x, dy = dd.y;
    const Quad q = quad_terms(r1.x, r1.y, r1.z, r1.w, r2.x, r2.y, r2.z, r2.w, dx, dy);
    const float iden = __builtin_amdgcn_rcpf(q.den);
    const float xs = fmaxf(q.num * iden, 0.f);
    const float Gs = __builtin_amdgcn_exp2f(-xs);
    const float o = r3.y;
    const float al = fminf(kAlphaMax, o * Gs);

    // ---- blend state and dL/dalpha
    const float Tj = p.T;
    const float w = al * Tj;
    const float om = 1.f - al;
    const float iom = __builtin_amdgcn_rcpf(om);
    // dF/dalpha_j = T_j f_j - (F - F_<=j) / (1 - alpha_j) for F in {colour, normal}, and
    // T_end / (1 - alpha_j) for acc, contracted with the upstream gradients: only the scalar
    // prefix S of w (g . f) is carried, the contracted totals sit in G0
    const float gc = gr * col.x + gg * col.y + gb * col.z + gnx * nrm.x + gny * nrm.y + gnz * nrm.z;
    const float S = fmaf(w, gc, p.S);
    const float testT = Tj * om;
    const bool is_k = live && !p.crossed && testT <= 0.5f;
    const float suffix = (!p.crossed && !is_k) ? (G0 - S) + cT * Tk : G0 - S;
    float dal = gc * Tj - suffix * iom;
    const bool clamped = al >= kAlphaMax;                 // alpha = min(0.99, o G*)
    float dq = clamped ? 0.f : -0.5f * al * dal;          // dalpha/dq* = -alpha/2
    float dop = clamped ? 0.f : dal * Gs;                 // dalpha/do = G*
    float ds = 0.f, dA = 0.f;
    if (is_k) {
      ds = gd * dn;
      dA = dA_k;
      dq += dq_k;
      dop += do_k;
    }
    if (live) {
      p.S = S;
      p.T = testT;
      if (is_k) p.crossed = true;
    }

    // ---- chain rule to (mu_c, P_c)
    const float mz = r3.x, aa = r3.w;
    const float sstar = mz * (1.f + q.b) * iden;
    const float dnx = dx * ifx, dny = dy * ify;
    const float dmx = p1.z, dmy = p1.w;
    const float dvx = dmx + dnx, dvy = dmy + dny;               // d = (dvx, dvy, 1)
    const float mzs = mz * (q.b + q.c) * iden;                  // mu_z - s*
    const float rxv = mzs * dmx - sstar * dnx, ryv = mzs * dmy - sstar * dny, rzv = mzs;
    const float P00 = p0.x, P01 = p0.y, P02 = p0.z, P11 = p0.w, P12 = p1.x, P22 = p1.y;
    const float Prx = P00 * rxv + P01 * ryv + P02 * rzv;
    const float Pry = P01 * rxv + P11 * ryv + P12 * rzv;
    const float Prz = P02 * rxv + P12 * ryv + P22 * rzv;
    const float Am = aa * q.den;
    // distortion and extent losses (App. C.1, C.2), in blend order: dL/dalpha through the
    // weights (prefix sums from the running totals), plus the direct terms of d = NDC(t*)
    // and of the extent e = sqrt((E^2 - q*) / A) / (|d~| s*^2)
    if constexpr (EXT) {
      if (loss_on) {
        // hardware reciprocals (1 ulp) throughout: nothing here decides an integer
        const float t = dn * sstar, it = __builtin_amdgcn_rcpf(t);
        const float d = (kNdcFar / (kNdcFar - kNdcNear)) * (t - kNdcNear) * it;
        const float ndcp = kKappa * it * it;
        const float Tn = testT;
        // L_dist = sum_ij w_i w_j (d_i - d_j)^2: dL/dw_k = 2 (A (d_k - mu)^2 + M), and the
        // suffix sum_{i>k} w_i dL/dw_i = 2 (A (M - prefix_k) + M (A - A_k))
        const float dc = d - mu;
        const float cd = 2.f * (Atot * dc * dc + Mtot);
        Mp = fmaf(w * dc, dc, Mp);
        const float Sd = 2.f * (Atot * (Mtot - Mp) + Mtot * (Atot - (1.f - Tn)));
        float dal_x = g_dist * (cd * Tj - Sd * iom);
        ds += g_dist * 4.f * w * Atot * dc * ndcp * dn;                   // dL/dd_k = 4 w_k A (d_k - mu)
        // E^2 - q* = 2 ln 2 (log2(255 o) - x*), log2(255 o) being the record's 1/255 cut.
        // Where that is not positive (an alpha that passed the cut by rounding) the forward
        // clamps it to 0, so the extent is 0 there and has no direct terms either
        const float uraw = (2.f * kLn2) * (r3.z - xs);
        const bool ext_pos = uraw > 0.f;
        const float iu = __builtin_amdgcn_rcpf(ext_pos ? uraw : 1.f), iAm = __builtin_amdgcn_rcpf(Am);
        const float e = ext_pos ? sqrtf(uraw * iAm) * it * __builtin_amdgcn_rcpf(sstar) : 0.f;
        Ep = fmaf(w, e, Ep);
        dal_x += g_ext * kKappa * (e * Tj - (Etot - Ep) * iom);
        const float ce = g_ext * kKappa * w, cee = ce * e;
        dq -= 0.5f * cee * iu;
        dA -= 0.5f * cee * iAm;
        ds -= 2.f * cee * it * dn;                                          // 1 / s* = |d~| / t
        dop += cee * iu * __builtin_amdgcn_rcpf(o);
        if (al < kAlphaMax) {                                                // alpha / o = G*
          dq -= 0.5f * al * dal_x;
          dop += dal_x * Gs;
        }
      }
    }
    // opacity at the rendered depth, peak in front of x: alpha_j(x) is the blend alpha
    if constexpr (EXT) {
      if (opa_on && sstar <= s_r && al < kAlphaMax) {
        const float dl = gopaP * iom;
        dq -= 0.5f * al * dl;
        dop += dl * Gs;                                                      // alpha / o = G*
      }
    }
    const float dq2 = 2.f * dq;
    gv[0] = dq2 * Prx;
    gv[1] = dq2 * Pry;
    gv[2] = dq2 * Prz;
    gv[3] = dq * rxv * rxv;
    gv[4] = dq * rxv * ryv;
    gv[5] = dq * rxv * rzv;
    gv[6] = dq * ryv * ryv;
    gv[7] = dq * ryv * rzv;
    gv[8] = dq * rzv * rzv;
    // terms of the peak depth s* and of A = d^T P d: only the crossing Gaussian (exact depth)
    // and the optional losses have them, so the wave takes this branch rarely otherwise
    if (__any(ds != 0.f || dA != 0.f)) {
      const float Pdx = P00 * dvx + P01 * dvy + P02;
      const float Pdy = P01 * dvx + P11 * dvy + P12;
      const float Pdz = P02 * dvx + P12 * dvy + P22;
      const float sA = ds * __builtin_amdgcn_rcpf(Am), hA = 0.5f * sA;
      gv[0] = fmaf(sA, Pdx, gv[0]);
      gv[1] = fmaf(sA, Pdy, gv[1]);
      gv[2] = fmaf(sA, Pdz, gv[2]);
      gv[3] += hA * 2.f * dvx * rxv + dA * dvx * dvx;
      gv[4] += hA * (dvx * ryv + rxv * dvy) + dA * dvx * dvy;
      gv[5] += hA * (dvx * rzv + rxv) + dA * dvx;
      gv[6] += hA * 2.f * dvy * ryv + dA * dvy * dvy;
      gv[7] += hA * (dvy * rzv + ryv) + dA * dvy;
      gv[8] += hA * 2.f * rzv + dA;
    }
    gv[9] = dop;
    gv[10] = gr * w; gv[11] = gg * w; gv[12] = gb * w;
    gv[13] = gnx * w; gv[14] = gny * w; gv[15] = gnz * w;
    // opacity at the rendered depth, peak beyond x: alpha_j(x) = o exp(-q(x)/2) with
    // q(x) = u^T P u, u = mu_c - x (x = s_r (dm + delta)); dq/dmu_c = 2 P u, dq/dP_c = u u^T
    if constexpr (EXT) {
      if (opa_on && sstar > s_r) {
        const float dsr = s_r - sstar;
        const float araw = o * exp2f(-(xs + kHalfLog2e * Am * dsr * dsr));
        const float ax = fminf(kAlphaMax, araw);
        if (ax >= kAlphaMin && s_r > near_plane && araw < kAlphaMax) {
          const float dl = gopaP * __builtin_amdgcn_rcpf(1.f - ax);
          const float dqx = -0.5f * ax * dl, dqx2 = 2.f * dqx;
          const float mzr = mz - s_r;
          const float ux = mzr * dmx - s_r * dnx, uy = mzr * dmy - s_r * dny, uz = mzr;
          gv[0] += dqx2 * (P00 * ux + P01 * uy + P02 * uz);
          gv[1] += dqx2 * (P01 * ux + P11 * uy + P12 * uz);
          gv[2] += dqx2 * (P02 * ux + P12 * uy + P22 * uz);
          gv[3] += dqx * ux * ux;
          gv[4] += dqx * ux * uy;
          gv[5] += dqx * ux * uz;
          gv[6] += dqx * uy * uy;
          gv[7] += dqx * uy * uz;
          gv[8] += dqx * uz * uz;
          gv[9] += dl * ax * __builtin_amdgcn_rcpf(o);
        }
      }
    }
  };

  // Every lane with a pending slot computes its partials; they are then added
  // wave-cooperatively.  Lanes of one wave often hold the same instance (neighbouring
  // pixels share Gaussians), and float atomics to one LDS address serialise, so lanes are
  // grouped by instance: small groups add directly, a larger group is first summed across
  // the wave (wave_field_sums16: each field total ends in one quad of lanes) and adds
  // once.  Entries older than the two resident batches add to the global buffer.
  auto round = [&](int cur_b) {
    float gv[kGradFields];
    if (has) qg = slot_gaussian(qpos, cur_b, qe);
    const uint32_t pos = has ? qpos : 0xFFFFFFFFu;
    const uint32_t e = qe;
    if constexpr (EXT) {
#pragma unroll
      for (int f = 0; f < kGradFields; ++f) gv[f] = 0.f;
      if (has) adjoint(true, gv);                        // the loss prefixes advance on emission only
    } else {
      // lanes without a pending slot compute on their last (or the first) Gaussian; every
      // use of gv below is masked by has, so their values are never read
      adjoint(has, gv);
    }
    const int resident_from = (cur_b - 1) * B;
    const bool resident = has && (int)pos >= resident_from;
    if (has && !resident) {
      float* dst = A.grads + (size_t)e * kGradFields;
#pragma unroll
      for (int f = 0; f < kGradFields; ++f) atomicAdd(dst + f, gv[f]);
    }
    // group the resident lanes by instance (wave-uniform masks: the loop is scalar work apart
    // from one compare per group)
    uint64_t todo = __ballot(resident);
    uint64_t big = 0ull;
    while (todo) {
      const uint32_t lp = __builtin_amdgcn_readlane(pos, __ffsll((unsigned long long)todo) - 1);
      const uint64_t m = __ballot(resident && pos == lp);
      if (__popcll(m) >= kGroupReduce) big |= m;
      todo &= ~m;
    }
    const int lane = (int)(threadIdx.x & 63);
    if (resident && !((big >> lane) & 1ull)) {
      float* dst = &gsl[((int)pos % NS) * kSlotStride];
#pragma unroll
      for (int f = 0; f < kGradFields; ++f) atomicAdd(dst + f, gv[f]);
    }
    while (big) {
      const int leader = __ffsll((unsigned long long)big) - 1;
      const uint32_t lp = __builtin_amdgcn_readlane(pos, leader);
      const bool mine = resident && pos == lp;           // the whole group is big
      big &= ~__ballot(mine);
      const float v = wave_field_sums16(gv, mine);
      if ((lane & 3) == 0) atomicAdd(&gsl[((int)lp % NS) * kSlotStride + ((lane >> 2) & 15)], v);
    }
  };
  // the oldest pending slot of each lane is this round's
  auto take_head = [&]() {
    has = nq > 0;
    qpos = fifo[0];
#pragma unroll
    for (int i = 0; i < D - 1; ++i) fifo[i] = fifo[i + 1];
    nq = has ? nq - 1 : 0;
  };
  // after a list step: a round once every lane that can still emit has a pending slot, or when
  // a FIFO is full (the next step may queue one more).  Deeper FIFOs measured slower (depth 6:
  // 3.29 -> 3.46 ms at 1M Gaussians 1080p), and so did a 3/4 quorum (3.33 ms)
  auto maybe_round = [&](int cur_b) {
    const uint64_t pend = __ballot(nq > 0);
    if (!pend) return;
    const uint64_t act = __ballot(nq > 0 || !emit_done());
    if (__any(nq >= D) || pend == act) {
      take_head();
      round(cur_b);
    }
  };

  // write the resident slots of batch b to the per-instance buffer and clear them
  auto flush = [&](int b) {
    if (b < 0 || threadIdx.x >= B) return;
    const int pos = b * B + (int)threadIdx.x;
    if (pos >= len) return;
    float* src = &gsl[(pos % NS) * kSlotStride];
    const uint32_t e = A.f.vals[rg.x + pos];
    float4* dst = (float4*)(A.grads + (size_t)e * kGradFields);
#pragma unroll
    for (int f4 = 0; f4 < kGradFields / 4; ++f4) {
      dst[f4] = make_float4(src[4 * f4], src[4 * f4 + 1], src[4 * f4 + 2], src[4 * f4 + 3]);
#pragma unroll
      for (int k = 0; k < 4; ++k) src[4 * f4 + k] = 0.f;
    }
  };

  int cur_b = -1;
  if constexpr (LIST) {
    // this lane's recorded order: row e of the wave's rows is its e-th blended Gaussian.  Each
    // batch takes the lane's next entries in blend order while their list position lies in
    // the batches staged so far (a Gaussian leaves the window at or after its own position),
    // so the slots of the last two batches stay resident as in the replay
    const uint16_t* recw =
        a.order + ((int64_t)tile * (NT / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) * a.order_slots * 64 +
        (threadIdx.x & 63);
    // (the forward flags a tile with more than order_slots blended Gaussians in a pixel, so
    // n_rec = n_emit here; the bounds only keep inconsistent inputs inside the buffers)
    const int n_rec = min(n_emit, a.order_slots);
    int kd = 0;                                           // entries taken
    uint32_t nxt = n_rec > 0 ? (uint32_t)recw[0] : 0xFFFFFFFFu;
    for (int bs = rg.x; bs < rg.y; bs += B) {
      if (__syncthreads_count(kd < n_rec) == 0) break;
      ++cur_b;
      flush(cur_b - 2);
      const int i = bs + (int)threadIdx.x;
      if (threadIdx.x < B && i < rg.y) {
        const uint32_t e = A.f.vals[i];
        ring[(i - rg.x) % NS] = make_uint2(e, (uint32_t)A.f.gid[e]);
      }
      __builtin_amdgcn_s_waitcnt(0x0F70);               // vmcnt(0): see the replay below
      __syncthreads();
      const uint32_t lim = (uint32_t)min((cur_b + 1) * B, len);
      while (true) {
        const bool go = kd < n_rec && nxt < lim;
        if (!__any(go)) break;
        has = go;
        qpos = nxt;
        if (go) {
          ++kd;
          nxt = kd < n_rec ? (uint32_t)recw[(int64_t)kd * 64] : 0xFFFFFFFFu;
        }
        round(cur_b);
      }
    }
  } else {
    for (int bs = rg.x; bs < rg.y; bs += B) {
      if (__syncthreads_count(!emit_done()) == 0) break;  // window and FIFO are drained after the loop
      ++cur_b;
      flush(cur_b - 2);
      const int i = bs + (int)threadIdx.x;
      if (threadIdx.x < B && i < rg.y) {
        const uint32_t e = A.f.vals[i];
        const int32_t g = A.f.gid[e];
        stage_entry(a.geom, a.rect, cam_base + g, x0, y0, (uint32_t)(i - rg.x), &stage[threadIdx.x],
                    &srect[threadIdx.x]);
        ring[(i - rg.x) % NS] = make_uint2(e, (uint32_t)g);
      }
      // The flushed slots and any later global atomics on them (entries emitted after their
      // batch left the ring) come from this workgroup only: waiting until this lane's stores
      // are acknowledged by L2 and then the barrier order them, without the L2 write-back and
      // invalidation of a device-scope fence.
      __builtin_amdgcn_s_waitcnt(0x0F70);                 // vmcnt(0)
      __syncthreads();
      const int nb = min(B, rg.y - bs);
      for (int j = 0; j < nb; ++j) {
        // a wave whose lanes have all emitted their count finishes its FIFOs after the list
        if (!__any(!emit_done())) break;
        if (misses_subtile(uniform_rect(srect[j]), sxu, syu)) continue;      // wave-uniform
        const StageEntry e = stage[j];
        const Cand1 c1 = candidate_stage1(e, lx, ly, near_plane);
        if (!__any(c1.pre && !emit_done())) continue;
        float key, al;
        const bool cand = candidate_stage2(e, c1, key, al) && !emit_done();
        if (__any(cand)) {
          if (cand) {
            float ea;
            uint32_t et;
            // alpha is recomputed on emission, so the window carries none (its moves fold away)
            if (win.push(key, 0.f, __float_as_uint(e.tag), ea, et)) queue(et);
          }
          maybe_round(cur_b);
        }
      }
    }
    // the rest of the window (in order) behind the pending slots: one new slot per lane and round
    while (__any(nq > 0 || (W > 0 && !emit_done() && win.count > 0))) {
      if constexpr (W > 0) {
        if (!emit_done() && win.count > 0 && nq < D) {
          float ea;
          uint32_t et;
          win.pop_front(ea, et);
          queue(et);
        }
      }
      take_head();
      round(cur_b);
    }
  }
  __syncthreads();
  flush(cur_b - 1);
  flush(cur_b);
  // entries never staged (the whole tile finished early) get zero partials
  for (int pos = (cur_b + 1) * B + (int)threadIdx.x; pos < len; pos += NT) {
    float4* dst = (float4*)(A.grads + (size_t)A.f.vals[rg.x + pos] * kGradFields);
#pragma unroll
    for (int f4 = 0; f4 < kGradFields / 4; ++f4) dst[f4] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

// With a recorded order: the order-reading kernel over the recorded tiles, then the replay
// over the flagged ones (each kernel leaves the other's tiles at once; they share no instance).
template <int TS, bool EXT>
static hipError_t launch_bwd_tso(const RenderBwdArgs& a, int window, int64_t n_tiles, hipStream_t s) {
  const dim3 grid((unsigned)n_tiles), block(TS * TS);
  if (a.f.order) {
    hipLaunchKernelGGL((k_render_bwd<TS, 0, EXT, true>), grid, block, 0, s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  switch (window) {
    case 0: hipLaunchKernelGGL((k_render_bwd<TS, 0, EXT, false>), grid, block, 0, s, a); break;
    case 1: hipLaunchKernelGGL((k_render_bwd<TS, 1, EXT, false>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_render_bwd<TS, 2, EXT, false>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_render_bwd<TS, 4, EXT, false>), grid, block, 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_render_bwd<TS, 8, EXT, false>), grid, block, 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_render_bwd<TS, 16, EXT, false>), grid, block, 0, s, a); break;
    case 32: hipLaunchKernelGGL((k_render_bwd<TS, 32, EXT, false>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int TS>
static hipError_t launch_bwd_ts(const RenderBwdArgs& a, int window, int64_t n_tiles, hipStream_t s) {
  const bool ext = a.d_opa || a.d_losses;
  return ext ? launch_bwd_tso<TS, true>(a, window, n_tiles, s) : launch_bwd_tso<TS, false>(a, window, n_tiles, s);
}

hipError_t launch_render_bwd(const RenderBwdArgs& a, int tile, int window, int64_t n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  switch (tile) {
    case 8: return launch_bwd_ts<8>(a, window, n_tiles, s);
    case 16: return launch_bwd_ts<16>(a, window, n_tiles, s);
    case 32: return launch_bwd_ts<32>(a, window, n_tiles, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sof
