// Opacity-field queries (Eq. (12)-(13)) at arbitrary points over many views, with the
// paper's ray/tile scheduling of points (Sec. 3.4, Eq. (14)) and z_min early stopping
// (Eq. (15)).
//
// Pipeline (all on the device, one persistent evaluation launch for every view):
//   1. project all (view, Gaussian) pairs; per-Gaussian world record S^-1 R^T, mean;
//   2. per (view, tile) Gaussian lists sorted by z_min (the same stable radix sort);
//   3. every (point, view) pair that sees the point gets the key [view tile, depth]
//      (depth log-quantised: the order only balances work) and is radix-sorted;
//   4. per tile ceil(N_P / 256) blocks of 256 points, an inclusive scan and a block -> tile
//      lookup table;
//   5. a persistent kernel pulls blocks from an atomic counter; the 256 lanes share the
//      tile's Gaussian list staged through LDS and each lane accumulates
//      T = prod (1 - alpha_i(t_eval)) for its point, stopping at z_min > z(x) or once
//      1 - T reaches the point's running minimum over views (the min cannot drop then);
//      the result enters the output through an atomic min on the float bits (values are
//      non-negative, so their bit patterns order like the floats).
// Order independence of O_N (App. A.2) is what allows walking lists in z_min order.
#include "render_common.h"

namespace sof {

constexpr int kQueryBlock = 256;
constexpr int kQueryStage = 128;          // Gaussians staged per batch (LDS bounds the occupancy:
                                          // 16.6 KB admits the eight workgroups per CU that the
                                          // 64-VGPR bound of k_query_eval allows)

// sched buffer layout.
struct SchedLayout {
  size_t status, cnt, off, scan_tmp, keys0, keys1, vals0, vals1, hist, hist_tmp, pranges, nblk, blk_off, blk_tmp, lut,
      total;
  int64_t pvcap, max_blocks;
  static __host__ __device__ SchedLayout make(int64_t n_points, int64_t pvcap, int64_t n_tiles) {
    SchedLayout L;
    L.pvcap = pvcap;
    L.max_blocks = div_up(pvcap, kQueryBlock) + n_tiles + 1;
    const int64_t nb = div_up(pvcap > 0 ? pvcap : 1, kSortTile);
    size_t o = 0;
    L.status = o;   o = align_up(o + sizeof(StatusBlock));
    L.cnt = o;      o = align_up(o + (size_t)n_points * 4);
    L.off = o;      o = align_up(o + (size_t)n_points * 8);
    L.scan_tmp = o; o = align_up(o + (size_t)(div_up(n_points > 0 ? n_points : 1, kScanChunk) + 1) * 8);
    L.keys0 = o;    o = align_up(o + (size_t)pvcap * 4);
    L.keys1 = o;    o = align_up(o + (size_t)pvcap * 4);
    L.vals0 = o;    o = align_up(o + (size_t)pvcap * 4);
    L.vals1 = o;    o = align_up(o + (size_t)pvcap * 4);
    L.hist = o;     o = align_up(o + (size_t)256 * nb * 4);
    L.hist_tmp = o; o = align_up(o + (size_t)(div_up(256 * nb, kScanChunk) + 1) * 8);
    L.pranges = o;  o = align_up(o + (size_t)(n_tiles > 0 ? n_tiles : 1) * 8);
    L.nblk = o;     o = align_up(o + (size_t)(n_tiles > 0 ? n_tiles : 1) * 4);
    L.blk_off = o;  o = align_up(o + (size_t)(n_tiles > 0 ? n_tiles : 1) * 4);
    L.blk_tmp = o;  o = align_up(o + (size_t)(div_up(n_tiles > 0 ? n_tiles : 1, kScanChunk) + 1) * 8);
    L.lut = o;      o = align_up(o + (size_t)L.max_blocks * 4);
    L.total = o;
    return L;
  }
};

// Projection of a point into a view in float64; true when the view sees it.
__device__ inline bool view_point(const sof_camera& cam, float near_plane, float x, float y, float z, double& u,
                                  double& v, double& zc) {
  const double xc = (double)cam.R[0] * x + (double)cam.R[1] * y + (double)cam.R[2] * z + cam.t[0];
  const double yc = (double)cam.R[3] * x + (double)cam.R[4] * y + (double)cam.R[5] * z + cam.t[1];
  zc = (double)cam.R[6] * x + (double)cam.R[7] * y + (double)cam.R[8] * z + cam.t[2];
  if (!(zc > (double)near_plane)) return false;
  u = cam.fx * xc / zc + cam.cx;
  v = cam.fy * yc / zc + cam.cy;
  return u >= 0.0 && u < (double)cam.width && v >= 0.0 && v < (double)cam.height;
}

__global__ __launch_bounds__(256) void k_pv_count(const float* pts, int64_t np, const sof_camera* cams, int n_cams,
                                                  float near_plane, int32_t* cnt) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const float x = pts[3 * p], y = pts[3 * p + 1], z = pts[3 * p + 2];
  int c = 0;
  for (int v = 0; v < n_cams; ++v) {
    double u, w, zc;
    c += view_point(cams[v], near_plane, x, y, z, u, w, zc) ? 1 : 0;
  }
  cnt[p] = c;
}

// Depth part of a pair key: the lists' depth key of the point's view depth (float bits, so no
// logarithm), cut to the bits left beside the tile id.  It only orders the points of a tile
// (the evaluation recomputes each point's own key), so any monotone map would do.
__device__ inline uint32_t pair_depth_bits(double z, int bits) {
  return bits > 0 ? query_depth_key((float)z, query_key_shift(bits)) : 0u;
}

// The pairs of a wave's 64 points fill one contiguous range (the scan's offset of its first
// point, of length the sum of their counts); inside it they are laid out view by view, each
// view's visible lanes in lane order, so every store instruction writes consecutive words.
// The order of pairs with equal keys only changes which points share a block, not a result.
__global__ __launch_bounds__(256) void k_pv_emit(const float* pts, int64_t np, const sof_camera* cams,
                                                 const CamInfo* ci, int n_cams, float near_plane, int tile,
                                                 const int64_t* off, int64_t pvcap, int dbits, uint32_t* keys,
                                                 uint32_t* vals, StatusBlock* status) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = p < np;
  if (!__any(live)) return;                           // wave-uniform: lane 0 holds the smallest p
  const int64_t e0 = live ? off[p] : 0;
  const int64_t base = ((int64_t)__builtin_amdgcn_readfirstlane((int)(e0 >> 32)) << 32) |
                       (uint32_t)__builtin_amdgcn_readfirstlane((int)(e0 & 0xFFFFFFFF));
  const int lane = (int)(threadIdx.x & 63);
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  float x = 0.f, y = 0.f, z = 0.f;
  if (live) { x = pts[3 * p]; y = pts[3 * p + 1]; z = pts[3 * p + 2]; }
  int64_t run = 0;
  bool over = false;
  for (int v = 0; v < n_cams; ++v) {
    double u = 0.0, w = 0.0, zc = 0.0;
    const bool vis = live && view_point(cams[v], near_plane, x, y, z, u, w, zc);
    const uint64_t m = __ballot(vis);
    if (vis) {
      const int64_t e = base + run + __popcll(m & below);
      if (e < pvcap) {
        const uint32_t t = (uint32_t)(ci[v].tile_off + ((int)w / tile) * ci[v].tiles_x + ((int)u / tile));
        keys[e] = (t << dbits) | pair_depth_bits(zc, dbits);
        vals[e] = (uint32_t)p;
      } else {
        over = true;
      }
    }
    run += __popcll(m);
  }
  if (__any(over) && lane == 0) atomicOr(&status->flags, 1);
}

__global__ __launch_bounds__(256) void k_zero_i32(int32_t* a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

__global__ __launch_bounds__(256) void k_fill_f32(float* a, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ __launch_bounds__(256) void k_pv_ranges(const uint32_t* keys, const int64_t* count, int64_t cap, int dbits,
                                                   int2* ranges) {
  const int64_t k = *count;
  const int64_t n = k < cap ? k : cap;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t t = keys[i] >> dbits;
  if (i == 0 || (keys[i - 1] >> dbits) != t) ranges[t].x = (int)i;
  if (i == n - 1 || (keys[i + 1] >> dbits) != t) ranges[t].y = (int)(i + 1);
}

__global__ __launch_bounds__(256) void k_nblk(const int2* ranges, int64_t n_tiles, int32_t* nblk) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  const int2 r = ranges[t];
  nblk[t] = (r.y - r.x + kQueryBlock - 1) / kQueryBlock;
}

__global__ __launch_bounds__(256) void k_lut(const int32_t* nblk, const int32_t* blk_off, int64_t n_tiles,
                                             int64_t max_blocks, int32_t* lut) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  const int b0 = blk_off[t];
  for (int k = 0; k < nblk[t]; ++k)
    if (b0 + k < max_blocks) lut[b0 + k] = (int32_t)t;
}

struct __align__(16) StageQ {
  float zmin;           // the walk's skip test reads these four words in one 16-byte load
  uint32_t qz;          // depth key of the list order (query_depth_key of zmin)
  uint32_t rx, ry;      // pixel rectangle x0 | x1 << 16, y0 | y1 << 16
  int ui, vi;
  float uf, vf;
  float gx, gy, cxx, cxy2;
  float cyy, mxx, mxy2, myy;
  float mz, o, thr, pad0;
  float m[9];
  float mu[3];
  float pad1[4];        // 144-byte stride: the 16-byte stores of consecutive lanes when a batch is
                        // staged start on 16 different LDS bank groups (128 bytes: only two)
};

struct QueryArgs {
  const float* pts;
  const sof_camera* cams;
  const CamInfo* cam_info;
  int n_cams;
  float near_plane;
  int64_t n;
  const float4* geom;
  const float* zmin;
  const float4* world;
  const short4* rect;
  const int2* granges;          // Gaussian tile lists
  const uint32_t* gvals;        // Gaussian ids (compact lists) or emission indices
  const int32_t* ggid;          // emission index -> Gaussian id (64-bit lists only)
  int key_shift;                // depth key of the lists (query_depth_key)
  int compact;
  int levelset;                 // only O > 0.5 or not is needed
  int cap;                      // instance capacity of the lists
  const int2* pranges;          // point lists per tile
  const uint32_t* pvals;
  const int32_t* blk_off;
  const int32_t* lut;
  const int64_t* total_blocks;
  int32_t* counter;
  float* out;
};

__global__ __launch_bounds__(kQueryBlock, 8) void k_query_eval(QueryArgs a) {
  __shared__ StageQ stage[kQueryStage];
  __shared__ int s_blk;
  const int64_t total = *a.total_blocks;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_blk = atomicAdd(a.counter, 1);
    __syncthreads();
    const int b = s_blk;
    if (b >= total) break;
    const int t = a.lut[b];
    const int2 pr = a.pranges[t];
    const int i = pr.x + (b - a.blk_off[t]) * kQueryBlock + (int)threadIdx.x;
    const bool active = i < pr.y;
    const int c = find_cam(a.cam_info, a.n_cams, t);
    const sof_camera& cam = a.cams[c];
    const int64_t cam_base = (int64_t)c * a.n;

    uint32_t p = 0;
    float px = 0.f, py = 0.f, pz = 0.f, zx = 0.f, uxf = 0.f, vyf = 0.f, cur = 1.f;
    int uxi = 0, vyi = 0;
    bool done = !active;
    if (active) {
      p = a.pvals[i];
      px = a.pts[3 * p]; py = a.pts[3 * p + 1]; pz = a.pts[3 * p + 2];
      double u, v, zc;
      view_point(cam, a.near_plane, px, py, pz, u, v, zc);
      const double fu = floor(u), fv = floor(v);
      uxi = (int)fu; vyi = (int)fv;
      uxf = (float)(u - fu); vyf = (float)(v - fv);
      zx = (float)zc;
      cur = a.out[p];
    }
    const uint32_t qx = query_depth_key(zx, a.key_shift);
    // level set: some view already gave O_N <= 1/2, so the minimum stays there
    bool pruned = a.levelset && active && cur <= 0.5f;
    done = done || pruned;
    float T = 1.f;
    int2 gr = a.granges[t];
    gr.x = max(0, min(gr.x, a.cap));                   // lists are read in bounds whatever bins holds
    gr.y = max(gr.x, min(gr.y, a.cap));
    for (int gs = gr.x; gs < gr.y; gs += kQueryStage) {
      if (__syncthreads_count(!done) == 0) break;
      const int gi = gs + (int)threadIdx.x;
      if (threadIdx.x < kQueryStage && gi < gr.y) {
        int32_t g = a.compact ? (int32_t)a.gvals[gi] : a.ggid[min(a.gvals[gi], (uint32_t)(a.cap - 1))];
        g = max(0, min(g, (int32_t)a.n - 1));
        const int64_t vg = cam_base + g;
        const float4 r0 = a.geom[4 * vg], r1 = a.geom[4 * vg + 1], r2 = a.geom[4 * vg + 2], r3 = a.geom[4 * vg + 3];
        const float4 w0 = a.world[4 * g], w1 = a.world[4 * g + 1], w2 = a.world[4 * g + 2];
        StageQ e;
        e.ui = __float_as_int(r0.x); e.uf = r0.y; e.vi = __float_as_int(r0.z); e.vf = r0.w;
        e.gx = r1.x; e.gy = r1.y; e.cxx = r1.z; e.cxy2 = r1.w;
        e.cyy = r2.x; e.mxx = r2.y; e.mxy2 = r2.z; e.myy = r2.w;
        e.mz = r3.x; e.o = r3.y; e.thr = r3.z; e.pad0 = 0.f; e.zmin = a.zmin[vg];
        e.m[0] = w0.x; e.m[1] = w0.y; e.m[2] = w0.z; e.m[3] = w0.w;
        e.m[4] = w1.x; e.m[5] = w1.y; e.m[6] = w1.z; e.m[7] = w1.w;
        e.m[8] = w2.x; e.mu[0] = w2.y; e.mu[1] = w2.z; e.mu[2] = w2.w;
        const short4 rc = a.rect[vg];
        e.rx = (uint32_t)(uint16_t)rc.x | ((uint32_t)(uint16_t)rc.z << 16);
        e.ry = (uint32_t)(uint16_t)rc.y | ((uint32_t)(uint16_t)rc.w << 16);
        e.qz = query_depth_key(e.zmin, a.key_shift);
        stage[threadIdx.x] = e;
      }
      __syncthreads();
      const int nb = min(kQueryStage, gr.y - gs);
      // Branch-light walk: lanes keep per-entry decisions as predicates and only wave-uniform
      // branches skip work (divergent branches cost scalar exec-mask instructions per entry,
      // which bound this loop otherwise).
      for (int j = 0; j < nb; ++j) {
        if (!__any(!done)) break;
        const StageQ& e = stage[j];
        const uint4 head = *reinterpret_cast<const uint4*>(&stage[j]);
        const float zmin = __uint_as_float(head.x);
        const uint32_t qz = head.y, rx = head.z, ry = head.w;
        // lists are sorted by a monotone key of z_min: past the point's key every later entry
        // lies beyond the point; inside its bucket the exact z_min decides
        done = done || (qz > qx);
        const bool in = !done && zmin <= zx && uxi >= (int)(rx & 0xFFFFu) && uxi <= (int)(rx >> 16) &&
                        vyi >= (int)(ry & 0xFFFFu) && vyi <= (int)(ry >> 16);
        if (!__any(in)) continue;
        const float dx = (float)(uxi - e.ui) + (uxf - e.uf);
        const float dy = (float)(vyi - e.vi) + (vyf - e.vf);
        const Quad q = quad_terms(e.gx, e.gy, e.cxx, e.cxy2, e.cyy, e.mxx, e.mxy2, e.myy, dx, dy);
        const float sn = e.mz * (1.f + q.b);
        bool ok = in && (q.den > 0.f) && !(q.num > 1.0001f * e.thr * q.den);
        const bool before = sn < zx * q.den;                       // peak in front of the point
        ok = ok && (!before || sn > a.near_plane * q.den);
        float xk = fmaxf(q.num * __builtin_amdgcn_rcpf(q.den), 0.f);
        const bool atx = ok && !before;                            // evaluate at the point itself
        if (__any(atx)) {
          const float wx = px - e.mu[0], wy = py - e.mu[1], wz = pz - e.mu[2];
          const float g0 = fmaf(e.m[0], wx, fmaf(e.m[1], wy, e.m[2] * wz));
          const float g1 = fmaf(e.m[3], wx, fmaf(e.m[4], wy, e.m[5] * wz));
          const float g2 = fmaf(e.m[6], wx, fmaf(e.m[7], wy, e.m[8] * wz));
          const float xa = kHalfLog2e * fmaf(g0, g0, fmaf(g1, g1, g2 * g2));
          xk = atx ? xa : xk;
        }
        const float al = fminf(kAlphaMax, e.o * __builtin_amdgcn_exp2f(-xk));
        ok = ok && al >= kAlphaMin;
        T = ok ? T * (1.f - al) : T;
        const bool prune = ok && (1.f - T >= cur);
        const bool half = a.levelset && ok && (1.f - T > 0.5f);   // this view's O_N exceeds 1/2
        pruned = pruned || prune;
        done = done || prune || half;
      }
    }
    if (active && !pruned) atomicMin((unsigned int*)(a.out + p), __float_as_uint(1.f - T));
  }
}

__global__ __launch_bounds__(256) void k_bisect_step(float* a, float* b, float* mid, const float* opacity,
                                                     int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float ax = a[3 * i], ay = a[3 * i + 1], az = a[3 * i + 2];
  float bx = b[3 * i], by = b[3 * i + 1], bz = b[3 * i + 2];
  if (opacity) {
    const float mx = mid[3 * i], my = mid[3 * i + 1], mz = mid[3 * i + 2];
    if (opacity[i] > 0.5f) {
      ax = mx; ay = my; az = mz;
      a[3 * i] = ax; a[3 * i + 1] = ay; a[3 * i + 2] = az;
    } else {
      bx = mx; by = my; bz = mz;
      b[3 * i] = bx; b[3 * i + 1] = by; b[3 * i + 2] = bz;
    }
  }
  mid[3 * i] = 0.5f * (ax + bx);
  mid[3 * i + 1] = 0.5f * (ay + by);
  mid[3 * i + 2] = 0.5f * (az + bz);
}

}  // namespace sof

using namespace sof;

extern "C" {

int sof_bisect_step(float* a, float* b, float* mid, const float* opacity, int64_t n_edges, hipStream_t stream) {
  if (n_edges < 0) return SOF_E_ARG;
  if (n_edges == 0) return SOF_OK;
  if (!a || !b || !mid) return SOF_E_ARG;
  hipLaunchKernelGGL(k_bisect_step, dim3((unsigned)div_up(n_edges, 256)), dim3(256), 0, stream, a, b, mid, opacity,
                     n_edges);
  return hipGetLastError() == hipSuccess ? SOF_OK : SOF_E_HIP;
}

int sof_query_workspace_size(int64_t n, const sof_camera* h_cams, int32_t n_cams, const sof_options* opts,
                             int64_t n_points, int64_t pv_capacity, size_t* proj_bytes, size_t* bins_bytes,
                             size_t* sched_bytes) {
  if (!opts || !h_cams || n_cams < 1 || n < 0 || n >= (int64_t(1) << 31)) return SOF_E_ARG;
  if (opts->tile != 8 && opts->tile != 16 && opts->tile != 32) return SOF_E_ARG;
  if (opts->capacity < 0 || opts->capacity >= (int64_t(1) << 31)) return SOF_E_ARG;
  if (n_points < 0 || n_points >= (int64_t(1) << 31) || pv_capacity < 0 || pv_capacity >= (int64_t(1) << 31))
    return SOF_E_ARG;
  int64_t n_tiles = 0;
  for (int c = 0; c < n_cams; ++c) {
    if (h_cams[c].width < 1 || h_cams[c].height < 1 || h_cams[c].width > 32767 || h_cams[c].height > 32767)
      return SOF_E_ARG;
    n_tiles += (int64_t)((h_cams[c].width + opts->tile - 1) / opts->tile) * ((h_cams[c].height + opts->tile - 1) / opts->tile);
  }
  if (bits_for(n_tiles) > 24) return SOF_E_UNSUPPORTED;
  const int64_t vn = n * n_cams;
  if (proj_bytes) *proj_bytes = ProjLayout::make(vn, true, n).total;
  if (bins_bytes) *bins_bytes = BinsLayout::make(vn, n_cams, opts->capacity, n_tiles).total;
  if (sched_bytes) *sched_bytes = SchedLayout::make(n_points, pv_capacity, n_tiles).total;
  return SOF_OK;
}

int sof_opacity_query(const sof_gaussians* g, const sof_camera* h_cams, const sof_camera* d_cams, int32_t n_cams,
                      const sof_options* opts, const float* points, int64_t n_points, int64_t pv_capacity,
                      float* opacity, void* proj, size_t proj_bytes, void* bins, size_t bins_bytes, void* sched,
                      size_t sched_bytes, hipStream_t s) {
  size_t pb = 0, bb = 0, sb = 0;
  int st = sof_query_workspace_size(g ? g->n : -1, h_cams, n_cams, opts, n_points, pv_capacity, &pb, &bb, &sb);
  if (st) return st;
  if (g->sh_degree < 0 || g->sh_degree > 3) return SOF_E_ARG;
  if (g->n > 0 && (!g->means || !g->scales || !g->quats || !g->opacities || !g->sh)) return SOF_E_ARG;
  if (!d_cams || !bins || !sched || (n_points > 0 && (!points || !opacity)) || (!proj && g->n > 0)) return SOF_E_ARG;
  if (proj_bytes < pb || bins_bytes < bb || sched_bytes < sb) return SOF_E_WORKSPACE;
  if (!(opts->near_plane > 0.f)) return SOF_E_ARG;
  int64_t n_tiles = 0;
  for (int c = 0; c < n_cams; ++c)
    n_tiles += (int64_t)((h_cams[c].width + opts->tile - 1) / opts->tile) * ((h_cams[c].height + opts->tile - 1) / opts->tile);
  const int tile = opts->tile;
  const float near_plane = opts->near_plane;
  const int64_t n = g->n, vn = n * n_cams;
  const int th = 256;
  hipError_t e = hipSuccess;

  // 1-2: Gaussians -> per (view, tile) lists sorted by z_min (or those of the previous call)
  int gpar = 0, gdbits = 0;
  if ((opts->flags & SOF_QUERY_REUSE) && n > 0) {
    gdbits = query_key_bits(n_tiles);
    gpar = gdbits ? ((32 + 7) / 8) & 1 : 0;           // where the previous call's sort left the lists
  } else {
    if ((e = launch_project(g, d_cams, n_cams, near_plane, proj, s, true)) != hipSuccess) return SOF_E_HIP;
    if ((e = launch_query_bin_sort(n, d_cams, n_cams, n_tiles, tile, opts->capacity, proj, bins, s, &gpar,
                                   &gdbits)) != hipSuccess)
      return SOF_E_HIP;
  }
  const ProjLayout P = ProjLayout::make(vn, true, n);
  const BinsLayout B = BinsLayout::make(vn, n_cams, opts->capacity, n_tiles);
  char* pbase = (char*)proj;
  char* bbase = (char*)bins;
  char* sbase = (char*)sched;
  const SchedLayout S = SchedLayout::make(n_points, pv_capacity, n_tiles);
  StatusBlock* sst = (StatusBlock*)(sbase + S.status);
  const CamInfo* ci = (const CamInfo*)(bbase + B.cams);

  // 3: (point, view) pairs keyed by [view tile, depth]
  // reset the schedule's status block (count, flags, block total, work counter)
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(th), 0, s, (int32_t*)sst, (int64_t)(sizeof(StatusBlock) / 4));
  int32_t* cnt = (int32_t*)(sbase + S.cnt);
  int64_t* off = (int64_t*)(sbase + S.off);
  if (n_points > 0)
    hipLaunchKernelGGL(k_pv_count, dim3((unsigned)div_up(n_points, th)), dim3(th), 0, s, points, n_points, d_cams,
                       n_cams, near_plane, cnt);
  if ((e = exclusive_scan<int32_t, int64_t>(cnt, n_points, off, (int64_t*)(sbase + S.scan_tmp), &sst->count, s)) !=
      hipSuccess)
    return SOF_E_HIP;
  const int tbits = bits_for(n_tiles);
  const int dbits = 32 - tbits;
  uint32_t* k0 = (uint32_t*)(sbase + S.keys0);
  uint32_t* k1 = (uint32_t*)(sbase + S.keys1);
  uint32_t* v0 = (uint32_t*)(sbase + S.vals0);
  uint32_t* v1 = (uint32_t*)(sbase + S.vals1);
  if (n_points > 0)
    hipLaunchKernelGGL(k_pv_emit, dim3((unsigned)div_up(n_points, th)), dim3(th), 0, s, points, n_points, d_cams, ci,
                       n_cams, near_plane, tile, off, pv_capacity, dbits, k0, v0, sst);
  int ppar = 0;
  if ((e = radix_sort<uint32_t>(k0, v0, k1, v1, &sst->count, pv_capacity, 32, (int32_t*)(sbase + S.hist),
                                (int32_t*)(sbase + S.hist_tmp), &ppar, s)) != hipSuccess)
    return SOF_E_HIP;
  const uint32_t* pk = ppar ? k1 : k0;
  const uint32_t* pv = ppar ? v1 : v0;

  // 4: blocks of 256 points per tile, scan, block -> tile table
  int2* pranges = (int2*)(sbase + S.pranges);
  int32_t* nblk = (int32_t*)(sbase + S.nblk);
  int32_t* blk_off = (int32_t*)(sbase + S.blk_off);
  int32_t* lut = (int32_t*)(sbase + S.lut);
  hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)div_up(2 * n_tiles, th)), dim3(th), 0, s, (int32_t*)pranges,
                     2 * n_tiles);
  if (pv_capacity > 0)
    hipLaunchKernelGGL(k_pv_ranges, dim3((unsigned)div_up(pv_capacity, th)), dim3(th), 0, s, pk, &sst->count,
                       pv_capacity, dbits, pranges);
  hipLaunchKernelGGL(k_nblk, dim3((unsigned)div_up(n_tiles, th)), dim3(th), 0, s, pranges, n_tiles, nblk);
  if ((e = exclusive_scan<int32_t, int32_t>(nblk, n_tiles, blk_off, (int32_t*)(sbase + S.blk_tmp), &sst->aux[0], s)) !=
      hipSuccess)
    return SOF_E_HIP;
  hipLaunchKernelGGL(k_lut, dim3((unsigned)div_up(n_tiles, th)), dim3(th), 0, s, nblk, blk_off, n_tiles, S.max_blocks,
                     lut);
  if (n_points > 0)
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)div_up(n_points, th)), dim3(th), 0, s, opacity, n_points, 1.0f);

  // 5: persistent evaluation over every (view, tile, block)
  QueryArgs qa;
  qa.pts = points; qa.cams = d_cams; qa.cam_info = ci; qa.n_cams = n_cams; qa.near_plane = near_plane; qa.n = n;
  qa.geom = (const float4*)(pbase + P.geom);
  qa.zmin = (const float*)(pbase + P.zmin);
  qa.rect = (const short4*)(pbase + P.rect);
  qa.world = (const float4*)(pbase + P.world);
  qa.granges = (const int2*)(bbase + B.ranges);
  qa.gvals = (const uint32_t*)(bbase + (gpar ? B.vals1 : B.vals0));
  qa.key_shift = query_key_shift(gdbits);
  qa.compact = gdbits > 0 ? 1 : 0;
  qa.levelset = (opts->flags & SOF_QUERY_LEVELSET) ? 1 : 0;
  qa.cap = (int)opts->capacity;
  qa.ggid = (const int32_t*)(bbase + B.gid);
  qa.pranges = pranges;
  qa.pvals = pv;
  qa.blk_off = blk_off;
  qa.lut = lut;
  qa.total_blocks = &sst->aux[0];
  qa.counter = (int32_t*)&sst->aux[1];
  qa.out = opacity;
  // persistent grid: every CU filled to the kernel's occupancy (256 CUs x 1 if a query fails;
  // the work counter makes any grid size correct, only the speed depends on it)
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_query_eval, kQueryBlock, 0) != hipSuccess) per_cu = 0;
  (void)hipGetLastError();                            // the launch check below sees only the launch
  const int64_t grid = (int64_t)(cus > 0 ? cus : 256) * (per_cu > 0 ? per_cu : 1);
  const int64_t maxb = S.max_blocks;
  timing_mark(kTimeQuery, 0, s);
  hipLaunchKernelGGL(k_query_eval, dim3((unsigned)(grid < maxb ? grid : maxb)), dim3(kQueryBlock), 0, s, qa);
  const hipError_t le = hipGetLastError();
  timing_mark(kTimeQuery, 1, s);
  return le == hipSuccess ? SOF_OK : SOF_E_HIP;
}

}  // extern "C"
