// Per-pixel machinery shared by the forward rasteriser and the backward replay, so that both
// make bit-identical decisions: candidate test, ray depth of the peak and the bounded
// resort window.
//
// Hierarchical resort (the paper adopts StopThePop's per-pixel resorting, Sec. 3.1): level
// 0 is the tile list already sorted by (view depth of the mean, index); level 1 is a
// per-pixel window of W entries kept sorted in registers.  While the window has room a
// candidate is inserted; once full, the smallest of window + newcomer (by peak depth, ties
// to the earlier stream position) is emitted for blending and the other stays.  At the end
// of the list the window is emitted in order.
#pragma once

#include "launch.h"

namespace sof {

// LDS copy of a tile-list entry (16 words): integer and fractional parts of the pixel
// offset of the tile origin from the projected centre, the quadric constants and a 32-bit
// tag (Gaussian index or list slot).  A pixel's offset is (float)(ix + lx) + hx: exact
// integer arithmetic and a single rounding, independent of the tile size.  The entry's
// pixel rectangle is staged separately (8 bytes) so that a wave whose sub-tile it misses
// reads nothing else.
struct __align__(16) StageEntry {
  int ix, iy;
  float hx, hy, gx, gy;
  float cxx, cxy2, cyy, mxx;
  float mxy2, myy, mz, o;
  float thr, tag;
};

__device__ inline void stage_entry(const float4* geom, const short4* rect, int64_t vg, int x0, int y0, uint32_t tag,
                                   StageEntry* dst, uint2* dst_rect) {
  const float4 r0 = geom[4 * vg + 0], r1 = geom[4 * vg + 1], r2 = geom[4 * vg + 2], r3 = geom[4 * vg + 3];
  const short4 rc = rect[vg];
  StageEntry e;
  e.ix = x0 - __float_as_int(r0.x);
  e.iy = y0 - __float_as_int(r0.z);
  e.hx = 0.5f - r0.y;
  e.hy = 0.5f - r0.w;
  e.gx = r1.x; e.gy = r1.y; e.cxx = r1.z; e.cxy2 = r1.w;
  e.cyy = r2.x; e.mxx = r2.y; e.mxy2 = r2.z; e.myy = r2.w;
  e.mz = r3.x; e.o = r3.y; e.thr = r3.z; e.tag = __uint_as_float(tag);
  *dst = e;
  *dst_rect = make_uint2((uint32_t)(uint16_t)rc.x | ((uint32_t)(uint16_t)rc.z << 16),
                         (uint32_t)(uint16_t)rc.y | ((uint32_t)(uint16_t)rc.w << 16));
}

// Pixel-to-lane layout inside a TS x TS tile: wave w owns the 8x8 sub-tile
// (w mod TS/8, w div TS/8); lane l is pixel (l mod 8, l div 8) of it.
template <int TS>
__device__ inline void lane_pixel(int tid, int& lx, int& ly) {
  const int w = tid >> 6, l = tid & 63;
  lx = (w % (TS / 8)) * 8 + (l & 7);
  ly = (w / (TS / 8)) * 8 + (l >> 3);
}

// True when the entry's rectangle misses the 8x8 sub-tile with origin (sx, sy) (then no
// pixel of the sub-tile can have it as a candidate).
__device__ inline bool misses_subtile(uint2 r, int sx, int sy) {
  const int rx0 = (int)(r.x & 0xFFFFu), rx1 = (int)(r.x >> 16);
  const int ry0 = (int)(r.y & 0xFFFFu), ry1 = (int)(r.y >> 16);
  return rx1 < sx || rx0 > sx + 7 || ry1 < sy || ry0 > sy + 7;
}

// Offset (pixels) of pixel centre (px, py) from the projected centre stored in `r0`.
__device__ inline float2 pixel_offset(float4 r0, int px, int py) {
  return make_float2((float)(px - __float_as_int(r0.x)) + (0.5f - r0.y),
                     (float)(py - __float_as_int(r0.z)) + (0.5f - r0.w));
}

struct Quad {
  float b, c, den, num;
};

// Quadric terms of a pixel at offset (dx, dy) pixels from the projected centre.
__device__ inline Quad quad_terms(float gx, float gy, float cxx, float cxy2, float cyy, float mxx, float mxy2, float myy,
                                  float dx, float dy) {
  Quad q;
  const float dx2 = dx * dx, dxy = dx * dy, dy2 = dy * dy;
  q.b = fmaf(gx, dx, gy * dy);
  q.c = fmaf(cxx, dx2, fmaf(cxy2, dxy, cyy * dy2));
  q.den = fmaf(2.f, q.b, 1.f) + q.c;
  q.num = fmaf(mxx, dx2, fmaf(mxy2, dxy, myy * dy2));
  return q;
}

// Candidate test in two predicated stages (no early returns: divergent branches cost scalar
// exec-mask instructions per list entry).  Stage 1 (cheap): the quadric terms, the
// conservative alpha pre-cut and the near-plane test of the peak.  Stage 2: alpha =
// min(0.99, o G*) >= 1/255 and the key (view z of the peak; the pixel's ray distance t* is
// key |d|, so the per-pixel order is the order of t*).  Callers skip stage 2 with a
// wave-uniform branch when no lane passed stage 1.
struct Cand1 {
  Quad q;
  float sn;
  bool pre;
};

__device__ inline Cand1 candidate_stage1(const StageEntry& e, int lx, int ly, float near_plane) {
  Cand1 c;
  const float dx = (float)(e.ix + lx) + e.hx, dy = (float)(e.iy + ly) + e.hy;
  c.q = quad_terms(e.gx, e.gy, e.cxx, e.cxy2, e.cyy, e.mxx, e.mxy2, e.myy, dx, dy);
  c.sn = e.mz * (1.f + c.q.b);
  c.pre = (c.q.den > 0.f) && !(c.q.num > 1.0001f * e.thr * c.q.den) && (c.sn > near_plane * c.q.den);
  return c;
}

__device__ inline bool candidate_stage2(const StageEntry& e, const Cand1& c, float& key, float& alpha) {
  const float r = __builtin_amdgcn_rcpf(c.q.den);
  const float x = fmaxf(c.q.num * r, 0.f);
  alpha = fminf(kAlphaMax, e.o * __builtin_amdgcn_exp2f(-x));
  key = c.sn * r;
  return c.pre && alpha >= kAlphaMin;
}

// Wave-uniform copy of a staged rectangle (every lane reads the same LDS word).
__device__ inline uint2 uniform_rect(uint2 r) {
  return make_uint2(__builtin_amdgcn_readfirstlane(r.x), __builtin_amdgcn_readfirstlane(r.y));
}

template <int W>
struct Window {
  float k[W > 0 ? W : 1];
  float a[W > 0 ? W : 1];
  uint32_t t[W > 0 ? W : 1];
  int count;
  __device__ inline void init() {
    count = 0;
#pragma unroll
    for (int i = 0; i < (W > 0 ? W : 1); ++i) {
      k[i] = __builtin_huge_valf();
      a[i] = 0.f;
      t[i] = 0u;
    }
  }
  // Remove the smallest entry (the head) at the end of the list.
  __device__ inline void pop_front(float& ea, uint32_t& et) {
    float ek;
    pop_front(ea, et, ek);
  }
  __device__ inline void pop_front(float& ea, uint32_t& et, float& ek) {
    ea = a[0];
    et = t[0];
    ek = k[0];
    if constexpr (W > 1) {
#pragma unroll
      for (int i = 0; i < W - 1; ++i) {
        k[i] = k[i + 1];
        a[i] = a[i + 1];
        t[i] = t[i + 1];
      }
    }
    k[W > 0 ? W - 1 : 0] = __builtin_huge_valf();
    --count;
  }
  // Feed one candidate.  Returns true with (ea, et) set when an entry leaves the window
  // (ek: its key).
  __device__ inline bool push(float key, float al, uint32_t tag, float& ea, uint32_t& et) {
    float ek;
    return push(key, al, tag, ea, et, ek);
  }
  __device__ inline bool push(float key, float al, uint32_t tag, float& ea, uint32_t& et, float& ek) {
    if constexpr (W == 0) {
      ea = al;
      et = tag;
      ek = key;
      return true;
    } else {
      if (count < W) {
        // sorted insert; empty slots hold +inf and shift right
#pragma unroll
        for (int i = W - 1; i >= 0; --i) {
          const bool gt = k[i] > key;
          const bool gtp = (i > 0) ? (k[i - 1] > key) : false;
          const float nk = gtp ? k[i > 0 ? i - 1 : 0] : key;
          const float na = gtp ? a[i > 0 ? i - 1 : 0] : al;
          const uint32_t nt = gtp ? t[i > 0 ? i - 1 : 0] : tag;
          k[i] = gt ? nk : k[i];
          a[i] = gt ? na : a[i];
          t[i] = gt ? nt : t[i];
        }
        ++count;
        return false;
      }
      if (key < k[0]) {
        ea = al;
        et = tag;
        ek = key;
        return true;
      }
      ea = a[0];
      et = t[0];
      ek = k[0];
      // drop the head, insert the newcomer after every entry with key <= its key
#pragma unroll
      for (int i = 0; i < W; ++i) {
        const bool take_next = (i < W - 1) ? (k[i < W - 1 ? i + 1 : i] <= key) : false;
        const bool prev_le = (i > 0) ? (k[i] <= key) : true;
        const float nk = take_next ? k[i < W - 1 ? i + 1 : i] : (prev_le ? key : k[i]);
        const float na = take_next ? a[i < W - 1 ? i + 1 : i] : (prev_le ? al : a[i]);
        const uint32_t nt = take_next ? t[i < W - 1 ? i + 1 : i] : (prev_le ? tag : t[i]);
        k[i] = nk;
        a[i] = na;
        t[i] = nt;
      }
      return true;
    }
  }
};

__device__ inline int find_cam(const CamInfo* ci, int n_cams, int tile) {
  int lo = 0, hi = n_cams - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ci[mid].tile_off <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

}  // namespace sof
