// Internal layouts of the caller-owned buffers and helpers shared by the HIP kernels and
// the C-ABI host code.  Nothing here is part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sof.h"

namespace sof {

constexpr int kMaxShCoeffs = 16;
constexpr float kAlphaMin = 1.0f / 255.0f;   // a contribution below this is skipped
constexpr float kAlphaMax = 0.99f;           // alpha clamp
constexpr float kTMin = 1e-4f;               // blending stops before T would drop below
constexpr float kHalfLog2e = 0.72134752044448170368f;   // 0.5 * log2(e): exp(-q/2) = exp2(-K q)
constexpr float kLn2 = 0.69314718055994530942f;
constexpr int kGradFields = 16;              // per-instance gradient partials
constexpr int kAuxChannels = 6;              // per-pixel replay state and work counters
constexpr size_t kAlign = 256;

inline __host__ __device__ size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }

// ------------------------------------------------------------------------------------
// proj buffer: per (camera, Gaussian) records, index vg = cam * n + gaussian.
//
// geom (16 floats, 64 B) -- everything the per-pixel loop reads, in pixel units:
//   [0] u_int (int bits)  [1] u_frac   [2] v_int (int bits)  [3] v_frac
//       projected centre u = fx mu_x/mu_z + cx split into integer and fraction so that a
//       pixel offset is formed without cancellation
//   [4] gx  [5] gy                  b' = gx dx + gy dy
//   [6] cxx [7] 2 cxy [8] cyy       c' = cxx dx^2 + 2cxy dx dy + cyy dy^2
//   [9] mxx [10] 2 mxy [11] myy     n' = mxx dx^2 + ...           (includes 0.5 log2 e)
//   [12] mu_z  [13] opacity  [14] log2(255 o)  [15] a = dm^T P dm
// with (dx, dy) the pixel-centre offset from (u, v), P the camera-space precision,
// dm = (mu_x/mu_z, mu_y/mu_z, 1).  Along the pixel ray d = dm + (dx/fx, dy/fy, 0):
//   den' = 1 + 2 b' + c' = d^T P d / a,   z-depth of the peak s* = mu_z (1 + b') / den',
//   G* = exp2(-n'/den'),   q* = n' / (den' 0.5 log2 e).
// app (8 floats): r g b (linear, clamped >= 0), opacity, nx ny nz (world normal), pad
// bwdr (8 floats): P00 P01 P02 P11 P12 P22 dm_x dm_y   (camera-space precision)
// rect (4 x int16): x0 y0 x1 y1 inclusive pixel rectangle; x0 > x1 when not live
// zmin (float): mu_z - E sqrt(Sigma_zz), the smallest view z on the E-ellipsoid
// ------------------------------------------------------------------------------------
// Query layout (sof_opacity_query): no app / bwdr records; instead one view-independent
// world record per Gaussian (16 floats): rows of S^-1 R^T (9), mean (3), pad (4), used to
// evaluate a Gaussian at a point in front of its peak without cancellation.
struct ProjLayout {
  size_t geom, app, bwdr, rect, zmin, world, total;
  static __host__ __device__ ProjLayout make(int64_t vn, bool query = false, int64_t n = 0) {
    ProjLayout L;
    size_t o = 0;
    L.geom = o; o = align_up(o + (size_t)vn * 64);
    L.app = o;  o = align_up(o + (query ? 0 : (size_t)vn * 32));
    L.bwdr = o; o = align_up(o + (query ? 0 : (size_t)vn * 32));
    L.rect = o; o = align_up(o + (size_t)vn * 8);
    L.zmin = o; o = align_up(o + (size_t)vn * 4);
    L.world = o; o = align_up(o + (query ? (size_t)n * 64 : 0));
    L.total = o;
    return L;
  }
};

// Per-camera table written on the device by sof_bin_sort (read by render kernels).
struct CamInfo {
  int32_t tile_off;   // first global tile id of this camera
  int32_t tiles_x, tiles_y;
  int32_t pad;
  int64_t pix_off;    // first pixel of this camera in concatenated images
  int64_t pad2;
};

// Device status block at offset 0 of `bins` (and of the query schedule buffer).
struct StatusBlock {
  int64_t count;      // instances requested
  int32_t flags;      // bit 0: capacity exceeded
  int32_t pad;
  int64_t aux[30];
};

constexpr int kSortItems = 8;                    // keys per thread in a radix sort tile
constexpr int kSortThreads = 256;
constexpr int kSortTile = kSortItems * kSortThreads;
constexpr int kScanItems = 16;
constexpr int kScanThreads = 256;
constexpr int kScanChunk = kScanItems * kScanThreads;

inline __host__ __device__ int64_t div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }

// bins buffer layout.  The render lists (launch_bin_sort) use keys0 for the tile buckets
// (uint64 depth key << 32 | emission index), keys1 for the per-instance (tile, depth key) and
// then as merge scratch, vals0 for the sorted emission indices, vals1 for the ranks inside the
// tiles and ranges first as the tile counters; the query's 32-bit lists use the four key /
// value regions and hist / hist_tmp for their radix sort.
struct BinsLayout {
  size_t status, cams, counts, offsets, scan_tmp, keys0, keys1, vals0, vals1, gid, hist, hist_tmp,
      ranges, total;
  int64_t vn, cap, n_tiles, sort_blocks;
  static __host__ __device__ BinsLayout make(int64_t vn, int32_t n_cams, int64_t cap, int64_t n_tiles) {
    BinsLayout L;
    L.vn = vn; L.cap = cap; L.n_tiles = n_tiles;
    L.sort_blocks = div_up(cap > 0 ? cap : 1, kSortTile);
    size_t o = 0;
    L.status = o;   o = align_up(o + sizeof(StatusBlock));
    L.cams = o;     o = align_up(o + (size_t)(n_cams + 1) * sizeof(CamInfo));
    L.counts = o;   o = align_up(o + (size_t)vn * 4);
    L.offsets = o;  o = align_up(o + (size_t)vn * 8);
    L.scan_tmp = o; o = align_up(o + (size_t)(div_up(vn > 0 ? vn : 1, kScanChunk) + 1) * 8);
    L.keys0 = o;    o = align_up(o + (size_t)cap * 8);
    L.keys1 = o;    o = align_up(o + (size_t)cap * 8);
    L.vals0 = o;    o = align_up(o + (size_t)cap * 4);
    L.vals1 = o;    o = align_up(o + (size_t)cap * 4);
    L.gid = o;      o = align_up(o + (size_t)cap * 4);
    const int64_t hn = 256 * L.sort_blocks;
    L.hist = o;     o = align_up(o + (size_t)hn * 4);
    L.hist_tmp = o; o = align_up(o + (size_t)(div_up(hn, kScanChunk) + 1) * 8);
    L.ranges = o;   o = align_up(o + (size_t)(n_tiles > 0 ? n_tiles : 1) * 8);
    L.total = o;
    return L;
  }
};

// Recorded blend order (sof_render_fwd writes it, sof_render_bwd reads it): one int32 flag
// per tile, then for each tile and 64-lane wave `slots` rows of 64 uint16 list positions
// (row e holds each lane's e-th blended Gaussian), so that a wave's reads and writes of one
// row are one contiguous 128-byte segment.
constexpr int64_t kMaxOrderSlots = 4096;
constexpr int64_t kMaxOrderListLength = 65536;  // positions are stored in 16 bits
struct OrderLayout {
  size_t flags, rec, total;
  static __host__ __device__ OrderLayout make(int64_t n_tiles, int tile, int64_t slots) {
    OrderLayout L;
    L.flags = 0;
    L.rec = align_up((size_t)(n_tiles > 0 ? n_tiles : 1) * 4);
    L.total = L.rec + (size_t)n_tiles * tile * tile * slots * 2;
    return L;
  }
};

// Number of bits needed to hold values 0..v-1 (at least 1).
inline __host__ __device__ int bits_for(int64_t v) {
  int b = 1;
  while ((int64_t(1) << b) < v) ++b;
  return b;
}

inline __host__ __device__ uint32_t fbits(float f) {
  union { float f; uint32_t u; } x;
  x.f = f;
  return x.u;
}

// Order-preserving map from float to uint32 (for keys that may be negative).
inline __host__ __device__ uint32_t float_order_bits(float f) {
  uint32_t u = fbits(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// NDC mapping of the distortion and extent losses (near 0.2, far 100 on the ray distance)
constexpr float kNdcNear = 0.2f, kNdcFar = 100.f;
constexpr int kLossChannels = 6;   // distortion, extent, mean, moment, opacity tail, position of k

// Depth key of the query's tile lists.  shift < 0: the exact order of the float.  Otherwise
// a monotone integer quantisation of it: offset of the float's order bits above those of
// 2^-10, clamped to 28 bits (32 octaves), shifted right by `shift`.  Monotone (z1 <= z2 gives
// key(z1) <= key(z2)) and computed with integer operations only, so every kernel that
// evaluates it on the same float gets the same key.
constexpr float kQueryKeyBase = 0.0009765625f;
inline __host__ __device__ int query_key_shift(int dbits) { return dbits <= 0 ? -1 : (dbits >= 28 ? 0 : 28 - dbits); }
inline __host__ __device__ uint32_t query_depth_key(float z, int shift) {
  const uint32_t b = float_order_bits(z);
  if (shift < 0) return b;
  const uint32_t base = float_order_bits(kQueryKeyBase);
  const uint32_t lim = (1u << 28) - 1u;
  const uint32_t d = b > base ? b - base : 0u;
  return (d < lim ? d : lim) >> shift;
}

}  // namespace sof
