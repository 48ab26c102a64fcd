// Duplication of Gaussians into tiles and the per-tile key sort (level 0 of the
// hierarchical resort, Sec. 3.1), plus the device-wide scan and the stable LSD radix sort
// used by the query's 32-bit lists.  Instance counts stay on the device: every grid is sized
// from static capacities and reads the live count from the status block, so the sequence can
// be captured in a graph.
//
// Render lists (and the query's lists when tile ids need more than 20 bits) are built by
// bucketing, not by a global sort: each instance takes its rank inside its tile with an
// atomic increment of the tile's counter, one workgroup scans the counters into the tile
// ranges, instances are scattered into their tile's range, and one wave per tile sorts its
// range in registers by (depth key, emission index).  Emission indices grow with the Gaussian
// index inside a camera, and a tile holds one camera's instances, so this is the order
// (tile, depth key, Gaussian index) whatever order the atomics handed out.
//
// Radix sort: 8-bit digits, 4096 32-bit keys (2048 64-bit keys) per workgroup of 256 lanes
// (4 wave64s).  Per pass a histogram kernel writes per-(digit, block) counts digit-major, an
// exclusive scan turns them into global offsets, and a scatter kernel ranks keys stably
// inside the workgroup: each wave owns a run of consecutive keys, walks them in input order,
// groups equal digits with 8 ballots and keeps running per-digit counts in LDS.
#include "launch.h"

namespace sof {

// ------------------------------------------------------------------------- scan

template <typename Tin, typename Tacc>
__device__ inline Tacc block_exclusive_scan(Tacc v, Tacc* lds_wave, Tacc& total) {
  // 256 threads = 4 waves of 64
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  Tacc x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    Tacc y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) lds_wave[w] = x;
  __syncthreads();
  Tacc base = 0;
  total = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    Tacc t = lds_wave[k];
    if (k < w) base += t;
    total += t;
  }
  __syncthreads();
  return base + x - v;
}

// Both scan passes load all of a thread's items before using them, every index clamped into
// [0, n) (n > 0 whenever they run): a load inside each predicated step was waited for on its
// own.  The chunk sums need no particular assignment of items to lanes, so that pass reads
// them coalesced.
template <typename Tin, typename Tacc>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const Tin* in, int64_t n, Tacc* sums) {
  __shared__ Tacc lw[4];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + threadIdx.x;
  Tin raw[kScanItems];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + (int64_t)k * kScanThreads;
    raw[k] = in[i < n ? i : n - 1];
  }
  Tacc s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + (int64_t)k * kScanThreads < n) s += (Tacc)raw[k];
  Tacc total;
  block_exclusive_scan<Tin, Tacc>(s, lw, total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Exclusive scan of the chunk sums in one workgroup; writes the grand total.
template <typename Tacc>
__global__ __launch_bounds__(kScanThreads) void k_scan_chunks(Tacc* sums, int64_t nchunks, int64_t* total_out) {
  __shared__ Tacc lw[4];
  Tacc carry = 0;
  for (int64_t b = 0; b < nchunks; b += kScanThreads) {
    const int64_t i = b + threadIdx.x;
    Tacc v = i < nchunks ? sums[i] : 0;
    Tacc tot;
    Tacc ex = block_exclusive_scan<Tacc, Tacc>(v, lw, tot);
    if (i < nchunks) sums[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && total_out) *total_out = (int64_t)carry;
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const Tin* in, int64_t n, const Tout* sums, Tout* out) {
  __shared__ Tout lw[4];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
  Tin raw[kScanItems];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) raw[k] = in[base + k < n ? base + k : n - 1];
  Tout v[kScanItems];
  Tout s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = base + k < n ? (Tout)raw[k] : 0;
    s += v[k];
  }
  Tout total;
  Tout run = sums[blockIdx.x] + block_exclusive_scan<Tout, Tout>(s, lw, total);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
}

template <typename Tin, typename Tout>
hipError_t exclusive_scan(const Tin* in, int64_t n, Tout* out, Tout* tmp, int64_t* total, hipStream_t s) {
  if (n <= 0) {
    if (total) hipLaunchKernelGGL((k_scan_chunks<Tout>), dim3(1), dim3(kScanThreads), 0, s, tmp, (int64_t)0, total);
    return hipGetLastError();
  }
  const int64_t nch = div_up(n, kScanChunk);
  hipLaunchKernelGGL((k_scan_reduce<Tin, Tout>), dim3((unsigned)nch), dim3(kScanThreads), 0, s, in, n, tmp);
  hipLaunchKernelGGL((k_scan_chunks<Tout>), dim3(1), dim3(kScanThreads), 0, s, tmp, nch, total);
  hipLaunchKernelGGL((k_scan_apply<Tin, Tout>), dim3((unsigned)nch), dim3(kScanThreads), 0, s, in, n, tmp, out);
  return hipGetLastError();
}

template hipError_t exclusive_scan<int32_t, int64_t>(const int32_t*, int64_t, int64_t*, int64_t*, int64_t*, hipStream_t);
template hipError_t exclusive_scan<int32_t, int32_t>(const int32_t*, int64_t, int32_t*, int32_t*, int64_t*, hipStream_t);

// ------------------------------------------------------------------------- radix sort

__device__ inline int64_t live_count(const int64_t* count, int64_t cap) {
  const int64_t k = *count;
  return k < cap ? k : cap;
}

// Keys per thread of a radix sort tile: 32-bit keys (the query's lists and point schedule, up
// to a billion entries) use tiles of 4096, whose longer digit runs coalesce the scatter's
// writes better; 64-bit keys keep 2048, which leaves the scatter at four waves per SIMD.
// Workspace sizes use kSortTile, the smaller tile, so both fit.
template <typename K>
constexpr int sort_items() { return sizeof(K) == 4 ? 2 * kSortItems : kSortItems; }
template <typename K>
constexpr int sort_tile() { return sort_items<K>() * kSortThreads; }

// A thread's keys i0, i0 + 64, ... with every index clamped into [0, n) (zeros when n is 0), so
// that the loads are unconditional and in flight together.
template <typename K, typename T, int N>
__device__ __attribute__((always_inline)) inline void load_clamped(const T* src, int64_t i0, int64_t n, T (&out)[N]) {
  if (n > 0) {
#pragma unroll
    for (int it = 0; it < N; ++it) {
      const int64_t i = i0 + it * 64;
      out[it] = src[i < n ? i : n - 1];
    }
  } else {
#pragma unroll
    for (int it = 0; it < N; ++it) out[it] = T(0);
  }
}
template <typename K, int N>
__device__ __attribute__((always_inline)) inline void load_keys_clamped(const K* keys, int64_t i0, int64_t n, K (&out)[N]) {
  load_clamped<K, K, N>(keys, i0, n, out);
}

template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const K* keys, const int64_t* count, int64_t cap,
                                                             int shift, int32_t* hist, int64_t nblocks) {
  __shared__ int32_t cnt[4][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int t = threadIdx.x; t < 4 * 256; t += kSortThreads) (&cnt[0][0])[t] = 0;
  __syncthreads();
  const int64_t n = live_count(count, cap);
  const int64_t start = (int64_t)blockIdx.x * sort_tile<K>() + (int64_t)w * (sort_items<K>() * 64);
  // all keys first (indices clamped into the live range), then the counts: a load inside
  // each predicated step was waited for on its own
  K kv[sort_items<K>()];
  load_keys_clamped<K>(keys, start + lane, n, kv);
#pragma unroll
  for (int it = 0; it < sort_items<K>(); ++it) {
    if (start + it * 64 + lane < n) atomicAdd(&cnt[w][(int)((kv[it] >> shift) & 0xFF)], 1);
  }
  __syncthreads();
  const int t = threadIdx.x;
  hist[(int64_t)t * nblocks + blockIdx.x] = cnt[0][t] + cnt[1][t] + cnt[2][t] + cnt[3][t];
}

template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const K* keys_in, const uint32_t* vals_in, K* keys_out,
                                                                uint32_t* vals_out, const int64_t* count, int64_t cap,
                                                                int shift, const int32_t* hist, int64_t nblocks) {
  __shared__ int32_t wc[4][256];       // per-wave digit counts, then per-wave block-local offsets
  __shared__ int32_t lstart[256];      // block-local start of each digit
  __shared__ int32_t gbase[256];       // global start of this block's run of each digit
  __shared__ int32_t lw[4];
  __shared__ K skey[sort_tile<K>()];
  __shared__ uint32_t sval[sort_tile<K>()];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int t = threadIdx.x; t < 4 * 256; t += kSortThreads) (&wc[0][0])[t] = 0;
  __syncthreads();
  const int64_t n = live_count(count, cap);
  const int64_t bstart = (int64_t)blockIdx.x * sort_tile<K>();
  const int64_t start = bstart + (int64_t)w * (sort_items<K>() * 64);
  K key[sort_items<K>()];
  uint32_t val[sort_items<K>()];
  int rank[sort_items<K>()];
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  // (loading all keys and values first, as the histogram does, measured slower here: 8.0
  // against 7.8 ms a pass at 1.1G keys; four waves per SIMD already hide these loads)
#pragma unroll
  for (int it = 0; it < sort_items<K>(); ++it) {
    const int64_t idx = start + it * 64 + lane;
    const bool valid = idx < n;
    key[it] = valid ? keys_in[idx] : K(0);
    val[it] = valid ? vals_in[idx] : 0u;
    const int d = (int)((key[it] >> shift) & 0xFF);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    int prior = 0;
    if (valid) prior = wc[w][d];
    const int below = __popcll(peers & lt);
    rank[it] = prior + below;
    // the lowest lane of each digit group advances the running count
    if (valid && below == 0) wc[w][d] = prior + __popcll(peers);
  }
  __syncthreads();
  {
    // block-local digit starts (scan over digits) and per-wave offsets inside each digit
    const int t = threadIdx.x;
    const int c0 = wc[0][t], c1 = wc[1][t], c2 = wc[2][t], c3 = wc[3][t];
    int total;
    const int ls = block_exclusive_scan<int, int>(c0 + c1 + c2 + c3, lw, total);
    lstart[t] = ls;
    gbase[t] = hist[(int64_t)t * nblocks + blockIdx.x];
    wc[0][t] = ls;
    wc[1][t] = ls + c0;
    wc[2][t] = ls + c0 + c1;
    wc[3][t] = ls + c0 + c1 + c2;
  }
  __syncthreads();
  // block-local stable sort in LDS
#pragma unroll
  for (int it = 0; it < sort_items<K>(); ++it) {
    const int64_t idx = start + it * 64 + lane;
    if (idx < n) {
      const int d = (int)((key[it] >> shift) & 0xFF);
      const int lp = wc[w][d] + rank[it];
      skey[lp] = key[it];
      sval[lp] = val[it];
    }
  }
  __syncthreads();
  // write out: consecutive local positions of one digit go to consecutive global slots
  const int nloc = (int)((n - bstart) < sort_tile<K>() ? (n - bstart > 0 ? n - bstart : 0) : sort_tile<K>());
  for (int sidx = threadIdx.x; sidx < nloc; sidx += kSortThreads) {
    const K k = skey[sidx];
    const int d = (int)((k >> shift) & 0xFF);
    const int64_t dst = (int64_t)gbase[d] + (sidx - lstart[d]);
    keys_out[dst] = k;
    vals_out[dst] = sval[sidx];
  }
}

template <typename K>
hipError_t radix_sort(K* k0, uint32_t* v0, K* k1, uint32_t* v1, const int64_t* count, int64_t cap, int bits,
                      int32_t* hist, int32_t* hist_tmp, int* out_parity, hipStream_t s) {
  const int64_t nb = div_up(cap > 0 ? cap : 1, sort_tile<K>());
  const int passes = (bits + 7) / 8;
  K* ki = k0; uint32_t* vi = v0; K* ko = k1; uint32_t* vo = v1;
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    hipLaunchKernelGGL((k_radix_hist<K>), dim3((unsigned)nb), dim3(kSortThreads), 0, s, ki, count, cap, shift, hist, nb);
    hipError_t e = exclusive_scan<int32_t, int32_t>(hist, 256 * nb, hist, hist_tmp, nullptr, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_radix_scatter<K>), dim3((unsigned)nb), dim3(kSortThreads), 0, s, ki, vi, ko, vo, count, cap,
                       shift, hist, nb);
    K* tk = ki; ki = ko; ko = tk;
    uint32_t* tv = vi; vi = vo; vo = tv;
  }
  *out_parity = passes & 1;
  return hipGetLastError();
}

template hipError_t radix_sort<uint64_t>(uint64_t*, uint32_t*, uint64_t*, uint32_t*, const int64_t*, int64_t, int,
                                         int32_t*, int32_t*, int*, hipStream_t);
template hipError_t radix_sort<uint32_t>(uint32_t*, uint32_t*, uint32_t*, uint32_t*, const int64_t*, int64_t, int,
                                         int32_t*, int32_t*, int*, hipStream_t);

// ------------------------------------------------------------------------- tiles

__global__ void k_cam_table(const sof_camera* cams, int n_cams, int tile, CamInfo* out, StatusBlock* status) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int32_t toff = 0;
  int64_t poff = 0;
  for (int c = 0; c < n_cams; ++c) {
    CamInfo ci;
    ci.tiles_x = (cams[c].width + tile - 1) / tile;
    ci.tiles_y = (cams[c].height + tile - 1) / tile;
    ci.tile_off = toff;
    ci.pix_off = poff;
    ci.pad = 0; ci.pad2 = 0;
    out[c] = ci;
    toff += ci.tiles_x * ci.tiles_y;
    poff += (int64_t)cams[c].width * cams[c].height;
  }
  CamInfo end;
  end.tile_off = toff; end.pix_off = poff; end.tiles_x = end.tiles_y = 0; end.pad = 0; end.pad2 = 0;
  out[n_cams] = end;
  status->count = 0;
  status->flags = 0;
}

__global__ __launch_bounds__(256) void k_count(const short4* rect, int64_t vn, int tile, int32_t* counts) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= vn) return;
  const short4 r = rect[idx];
  int c = 0;
  if (r.x <= r.z && r.y <= r.w) c = (r.z / tile - r.x / tile + 1) * (r.w / tile - r.y / tile + 1);
  counts[idx] = c;
}

// One instance per (camera, Gaussian, touched tile), in emission order e (the scan of the
// per-Gaussian counts): its tile, depth key and Gaussian, and its rank inside the tile from
// an atomic increment of the tile's counter (ranges[t].y, zeroed by k_bin_count).  Instances
// with e >= cap are dropped and flagged.  Each wave owns 64 consecutive (camera, Gaussian)
// pairs and hands out their instances one per lane (an owner search over the wave's
// inclusive prefix of counts), so a wave's 64 atomics and stores issue together and the
// stores are coalesced whatever the size of each Gaussian's rectangle.
struct EmitOwner {
  int32_t tx0, ty0, nx, toff, tiles_x, g;
  uint32_t key;
  int32_t pad;
};

__global__ __launch_bounds__(256) void k_emit(const short4* rect, const float4* geom, const float* zmin, int64_t n,
                                              int64_t vn, int tile, const CamInfo* cams, const int32_t* counts,
                                              const int64_t* offsets, int64_t cap, int query_keys, uint2* inst,
                                              uint32_t* rank, int32_t* gid, int2* ranges, StatusBlock* status) {
  __shared__ EmitOwner own[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t base = ((int64_t)blockIdx.x * 4 + w) * 64;
  if (base >= vn) return;                                 // wave-uniform
  const int64_t vg = base + lane;
  int cnt = 0;
  if (vg < vn) {
    cnt = counts[vg];
    if (cnt > 0) {
      const short4 r = rect[vg];
      const int c = (int)(vg / n);
      const CamInfo ci = cams[c];
      EmitOwner o;
      o.tx0 = r.x / tile;
      o.ty0 = r.y / tile;
      o.nx = r.z / tile - o.tx0 + 1;
      o.toff = ci.tile_off;
      o.tiles_x = ci.tiles_x;
      o.g = (int32_t)(vg - (int64_t)c * n);
      o.key = query_keys ? float_order_bits(zmin[vg]) : float_order_bits(geom[4 * vg + 3].x);
      o.pad = 0;
      own[w][lane] = o;
    }
  }
  int incl = cnt;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  const int total = __shfl(incl, 63, 64);
  const int64_t e0 = offsets[base];                       // emission index of the wave's first instance
  if (lane == 0 && e0 + total > cap && total > 0) atomicOr(&status->flags, 1);
  __builtin_amdgcn_wave_barrier();                        // own[w] written by this wave only
  // the loop and the shuffles run on all 64 lanes (total is wave-uniform); only the stores
  // are predicated
  const int excl = incl - cnt;
  // kEmitUnroll instances per lane and step: their tile-counter atomics are all in flight
  // before the first returned rank is stored
  constexpr int kEmitUnroll = 4;
  for (int j0 = 0; j0 < total; j0 += 64 * kEmitUnroll) {
    uint32_t rk[kEmitUnroll];
    int64_t ee[kEmitUnroll];
    bool ok[kEmitUnroll];
#pragma unroll
    for (int u = 0; u < kEmitUnroll; ++u) {
      const int j = j0 + 64 * u + lane;
      // owner: the first lane whose inclusive prefix exceeds j (it has a non-zero count)
      int lo = 0, hi = 63;
#pragma unroll
      for (int it = 0; it < 6; ++it) {
        const int mid = (lo + hi) >> 1;
        const bool right = __shfl(incl, mid, 64) <= j;
        lo = right ? mid + 1 : lo;
        hi = right ? hi : mid;
      }
      const int before = __shfl(excl, lo, 64);
      ee[u] = e0 + j;
      ok[u] = j < total && ee[u] < cap;
      rk[u] = 0u;
      if (ok[u]) {
        const EmitOwner o = own[w][lo];
        const int local = j - before;
        const int ty = o.ty0 + local / o.nx, tx = o.tx0 + local % o.nx;
        const uint32_t t = (uint32_t)(o.toff + ty * o.tiles_x + tx);
        rk[u] = (uint32_t)atomicAdd(&ranges[t].y, 1);
        inst[ee[u]] = make_uint2(t, o.key);
        gid[ee[u]] = o.g;
      }
    }
#pragma unroll
    for (int u = 0; u < kEmitUnroll; ++u)
      if (ok[u]) rank[ee[u]] = rk[u];
  }
}

// The first dispatch of the render lists: camera table and status reset (thread 0), zeroed
// tile counters, each (camera, Gaussian)'s count of touched tiles, and the per-chunk sums of
// those counts (the first step of the exclusive scan that gives the emission offsets).
// One dispatch instead of three: each of these light kernels cost 4-6 us at 1M Gaussians.
__device__ inline int32_t rect_tile_count(short4 r, int tile) {
  return (r.x <= r.z && r.y <= r.w) ? (r.z / tile - r.x / tile + 1) * (r.w / tile - r.y / tile + 1) : 0;
}

__global__ __launch_bounds__(kScanThreads) void k_bin_count(const sof_camera* cams, int n_cams, int tile,
                                                            CamInfo* out, StatusBlock* status, int2* ranges,
                                                            int64_t n_tiles, const short4* rect, int64_t vn,
                                                            int32_t* counts, int64_t* sums) {
  __shared__ int64_t lw[4];
  const int64_t gid = (int64_t)blockIdx.x * kScanThreads + threadIdx.x;
  for (int64_t t = gid; t < n_tiles; t += (int64_t)gridDim.x * kScanThreads) ranges[t] = make_int2(0, 0);
  if (gid == 0) {
    int32_t toff = 0;
    int64_t poff = 0;
    for (int c = 0; c < n_cams; ++c) {
      CamInfo ci;
      ci.tiles_x = (cams[c].width + tile - 1) / tile;
      ci.tiles_y = (cams[c].height + tile - 1) / tile;
      ci.tile_off = toff;
      ci.pix_off = poff;
      ci.pad = 0; ci.pad2 = 0;
      out[c] = ci;
      toff += ci.tiles_x * ci.tiles_y;
      poff += (int64_t)cams[c].width * cams[c].height;
    }
    CamInfo end;
    end.tile_off = toff; end.pix_off = poff; end.tiles_x = end.tiles_y = 0; end.pad = 0; end.pad2 = 0;
    out[n_cams] = end;
    status->count = 0;
    status->flags = 0;
  }
  // only the chunk's total is needed here, so the lanes read consecutive records (the
  // offsets kernel then gives each thread its own run of kScanItems)
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + threadIdx.x;
  // all records first (indices clamped into [0, vn)), so the loads are in flight together
  short4 rr[kScanItems];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + (int64_t)k * kScanThreads;
    rr[k] = vn > 0 ? rect[i < vn ? i : vn - 1] : make_short4(0, 0, -1, -1);
  }
  int64_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + (int64_t)k * kScanThreads;
    if (i < vn) {
      const int32_t c = rect_tile_count(rr[k], tile);
      counts[i] = c;
      sum += c;
    }
  }
  int64_t total;
  block_exclusive_scan<int64_t, int64_t>(sum, lw, total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Tile counters -> ranges [start, start + count) in one workgroup (an exclusive scan over
// the tiles, 1024 lanes x 8 tiles per round, carried across rounds).
constexpr int kTileScanThreads = 1024, kTileScanItems = 8;
__global__ __launch_bounds__(kTileScanThreads) void k_tile_scan(int2* ranges, int64_t n_tiles) {
  __shared__ int32_t wsum[kTileScanThreads / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int32_t carry = 0;
  for (int64_t b = 0; b < n_tiles; b += (int64_t)kTileScanThreads * kTileScanItems) {
    const int64_t base = b + (int64_t)threadIdx.x * kTileScanItems;
    int32_t v[kTileScanItems];
    int32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kTileScanItems; ++k) {
      v[k] = base + k < n_tiles ? ranges[base + k].y : 0;
      sum += v[k];
    }
    int32_t x = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int32_t y = __shfl_up(x, d, 64);
      if (lane >= d) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int32_t before = 0, total = 0;
#pragma unroll
    for (int k = 0; k < kTileScanThreads / 64; ++k) {
      const int32_t t = wsum[k];
      before += k < w ? t : 0;
      total += t;
    }
    __syncthreads();
    int32_t run = carry + before + x - sum;
#pragma unroll
    for (int k = 0; k < kTileScanItems; ++k) {
      if (base + k < n_tiles) ranges[base + k] = make_int2(run, run + v[k]);
      run += v[k];
    }
    carry += total;
  }
}

// Instances into their tile's range, keyed (depth key << 32 | emission index).
__global__ __launch_bounds__(256) void k_tile_scatter(const uint2* inst, const uint32_t* rank, const int2* ranges,
                                                      const int64_t* count, int64_t cap, uint64_t* bucket) {
  const int64_t n = live_count(count, cap);
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const uint2 it = inst[e];
  bucket[ranges[it.x].x + rank[e]] = ((uint64_t)it.y << 32) | (uint64_t)e;
}

// Per-tile sort: one wave per tile, the keys in registers.  A list of L <= kTileSortCap entries
// is padded to P = 64 E entries (E a power of two, the smallest with P >= L; the padding holds
// the largest key) and lane l holds entries i = l E + k, k < E.  A bitonic network then sorts
// them: a compare-exchange of entries i and i ^ J (ascending where i & K is clear, K the size
// of the merged block) joins two registers of one lane when J < E, else the same register of
// lanes l and l ^ (J / E), whose values a DPP move (lane distance 1, 2, 4, 8) or a row or
// half-wave swap (16, 32) brings over.  No LDS and no barrier: at the benchmark's sizes
// (lists of about 400 entries, E = 8) 24 of the 45 stages stay inside a lane and 18 of the
// others use DPP.
constexpr int kTileSortThreads = 64, kTileSortCap = 2048;

constexpr int kDppQuadXor1 = 0xB1;       // quad permutation (1, 0, 3, 2): lane i ^ 1
constexpr int kDppQuadXor2 = 0x4E;       // quad permutation (2, 3, 0, 1): lane i ^ 2
constexpr int kDppQuadRev = 0x1B;        // quad permutation (3, 2, 1, 0): lane i ^ 3
constexpr int kDppRowHalfMirror = 0x141; // lane i of a half-row reads lane 7 - i: i ^ 7
constexpr int kDppRowRor8 = 0x128;       // rotate a row of 16 lanes by 8: i ^ 8

template <int CTRL>
__device__ inline uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, true);
}

// The value of lane l ^ D (D a power of two below 64).
template <int D>
__device__ inline uint32_t lane_xor_u32(uint32_t v, bool lower) {
  if constexpr (D == 1) return dpp_u32<kDppQuadXor1>(v);
  else if constexpr (D == 2) return dpp_u32<kDppQuadXor2>(v);
  else if constexpr (D == 4) return dpp_u32<kDppQuadRev>(dpp_u32<kDppRowHalfMirror>(v));   // (i ^ 7) ^ 3
  else if constexpr (D == 8) return dpp_u32<kDppRowRor8>(v);
  else if constexpr (D == 16) {
    // odd rows of the first operand swap with even rows of the second: with both the same,
    // the first result holds rows (0, 0, 2, 2) and the second rows (1, 1, 3, 3)
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return lower ? r[1] : r[0];
  } else {
    // upper half of the first operand swaps with the lower half of the second
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return lower ? r[1] : r[0];
  }
}

template <int D>
__device__ inline uint64_t lane_xor_u64(uint64_t v, bool lower) {
  const uint32_t lo = lane_xor_u32<D>((uint32_t)v, lower);
  const uint32_t hi = lane_xor_u32<D>((uint32_t)(v >> 32), lower);
  return ((uint64_t)hi << 32) | lo;
}

// Compare-exchange of two entries of one lane (the smaller to x when up).
__device__ inline void ce_pair(uint64_t& x, uint64_t& y, bool up) {
  const uint64_t a = x, b = y;
  const bool sw = (a > b) == up;
  x = sw ? b : a;
  y = sw ? a : b;
}

// Blocks of K <= E entries lie inside one lane: the first phases of the network.
template <int E, int K = 2>
__device__ inline void wave_bitonic_in_lane(uint64_t (&v)[E], int lane) {
  if constexpr (K <= E) {
#pragma unroll
    for (int J = K / 2; J >= 1; J >>= 1)
#pragma unroll
      for (int k = 0; k < E; ++k)
        if ((k & J) == 0) ce_pair(v[k], v[k | J], (((lane * E) + k) & K) == 0);
    wave_bitonic_in_lane<E, 2 * K>(v, lane);
  }
}

// Stage J = D E of a phase K > J: lane l keeps the smaller of its entry and lane l ^ D's
// when keep_min.
template <int E, int D>
__device__ inline void wave_bitonic_lanes(uint64_t (&v)[E], bool lower, bool keep_min) {
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const uint64_t o = lane_xor_u64<D>(v[k], lower);
    v[k] = ((o < v[k]) == keep_min) ? o : v[k];
  }
}

// Phases K = 2 E .. 64 E run as a loop (the stages between lanes picked by their distance),
// so that the code of one E stays small; each phase ends with its stages inside the lane,
// whose direction is the lane's for the whole phase.
template <int E>
__device__ inline void wave_bitonic_sort(uint64_t (&v)[E], int lane) {
  wave_bitonic_in_lane<E>(v, lane);
  for (int K = 2 * E; K <= 64 * E; K <<= 1) {
    const bool up = ((lane * E) & K) == 0;
    for (int D = K / (2 * E); D >= 1; D >>= 1) {
      const bool lower = (lane & D) == 0;
      const bool keep_min = up == lower;
      switch (D) {
        case 1: wave_bitonic_lanes<E, 1>(v, lower, keep_min); break;
        case 2: wave_bitonic_lanes<E, 2>(v, lower, keep_min); break;
        case 4: wave_bitonic_lanes<E, 4>(v, lower, keep_min); break;
        case 8: wave_bitonic_lanes<E, 8>(v, lower, keep_min); break;
        case 16: wave_bitonic_lanes<E, 16>(v, lower, keep_min); break;
        default: wave_bitonic_lanes<E, 32>(v, lower, keep_min); break;
      }
    }
#pragma unroll
    for (int J = E / 2; J >= 1; J >>= 1)
#pragma unroll
      for (int k = 0; k < E; ++k)
        if ((k & J) == 0) ce_pair(v[k], v[k | J], up);
  }
}

// Sort src[0, m) (m <= 64 E) by the wave; the sorted keys go to dst, or their low words
// (emission indices) to vals when dst is null.
template <int E>
__device__ __attribute__((always_inline)) inline void wave_sort_chunk(const uint64_t* src, int m, uint64_t* dst,
                                                                      uint32_t* vals) {
  const int lane = (int)(threadIdx.x & 63);
  uint64_t v[E];
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const int i = lane * E + k;
    v[k] = i < m ? src[i] : ~0ull;
  }
  wave_bitonic_sort<E>(v, lane);
  if (dst) {
#pragma unroll
    for (int k = 0; k < E; ++k)
      if (lane * E + k < m) dst[lane * E + k] = v[k];
  } else {
#pragma unroll
    for (int k = 0; k < E; ++k)
      if (lane * E + k < m) vals[lane * E + k] = (uint32_t)v[k];
  }
}

__device__ __attribute__((always_inline)) inline void wave_sort_any(const uint64_t* src, int m, uint64_t* dst,
                                                                    uint32_t* vals) {
  if (m <= 64) wave_sort_chunk<1>(src, m, dst, vals);
  else if (m <= 128) wave_sort_chunk<2>(src, m, dst, vals);
  else if (m <= 256) wave_sort_chunk<4>(src, m, dst, vals);
  else if (m <= 512) wave_sort_chunk<8>(src, m, dst, vals);
  else if (m <= 1024) wave_sort_chunk<16>(src, m, dst, vals);
  else wave_sort_chunk<32>(src, m, dst, vals);
}

// One wave per tile: its range sorted by (depth key, emission index); the emission indices are
// written to vals.  Ranges above kTileSortCap (not met at the benchmark's sizes, where the
// longest list is about a thousand) are sorted in chunks of kTileSortCap and then merged
// pairwise in global memory, each element placed by its rank in the other run (keys are
// unique), ping-ponging between bucket and tmp.
// Four waves per SIMD (128 VGPRs): 0.224 against 0.239 ms for the whole bin sort without a
// bound (208 VGPRs); only the 2048-entry variant, for lists above 1024, spills.
__global__ __launch_bounds__(kTileSortThreads, 4) void k_tile_sort(const int2* ranges, uint64_t* bucket, uint64_t* tmp,
                                                                uint32_t* vals) {
  const int2 rg = ranges[blockIdx.x];
  const int L = rg.y - rg.x;
  if (L <= 0) return;
  uint64_t* src = bucket + rg.x;
  uint64_t* dst = tmp + rg.x;
  const bool small = L <= kTileSortCap;
  for (int c0 = 0; c0 < L; c0 += kTileSortCap)
    wave_sort_any(src + c0, min(kTileSortCap, L - c0), small ? nullptr : src + c0, vals + rg.x);
  if (small) return;
  __syncthreads();
  for (int width = kTileSortCap; width < L; width <<= 1) {
    for (int i = threadIdx.x; i < L; i += kTileSortThreads) {
      const int lo = (i / (2 * width)) * (2 * width);
      const int mid = min(lo + width, L), hi = min(lo + 2 * width, L);
      const uint64_t x = src[i];
      // rank of x in the other run of its pair (binary search; keys are unique)
      const bool in_a = i < mid;
      int a = in_a ? mid : lo, b = in_a ? hi : mid;
      while (a < b) {
        const int h = (a + b) >> 1;
        if (src[h] < x) a = h + 1; else b = h;
      }
      const int other = a - (in_a ? mid : lo);
      const int self = i - (in_a ? lo : mid);
      dst[lo + self + other] = x;
    }
    __syncthreads();
    uint64_t* t = src; src = dst; dst = t;
  }
  for (int i = threadIdx.x; i < L; i += kTileSortThreads) vals[rg.x + i] = (uint32_t)src[i];
}

// Query tile lists with 32-bit keys: (tile << dbits) | quantised z_min, value = Gaussian id.
// Wave-cooperative like k_emit: each wave owns 64 consecutive (camera, Gaussian) pairs and
// writes their instances one per lane, so the stores are coalesced and no wave waits for the
// largest rectangle among its lanes.
__global__ __launch_bounds__(256) void k_emit_query32(const short4* rect, const float* zmin, int64_t n, int64_t vn,
                                                      int tile, const CamInfo* cams, const int32_t* counts,
                                                      const int64_t* offsets, int64_t cap, int dbits, uint32_t* keys,
                                                      uint32_t* vals, StatusBlock* status) {
  __shared__ EmitOwner own[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t base = ((int64_t)blockIdx.x * 4 + w) * 64;
  if (base >= vn) return;                                 // wave-uniform
  const int64_t vg = base + lane;
  int cnt = 0;
  if (vg < vn) {
    cnt = counts[vg];
    if (cnt > 0) {
      const short4 r = rect[vg];
      const int c = (int)(vg / n);
      const CamInfo ci = cams[c];
      EmitOwner o;
      o.tx0 = r.x / tile;
      o.ty0 = r.y / tile;
      o.nx = r.z / tile - o.tx0 + 1;
      o.toff = ci.tile_off;
      o.tiles_x = ci.tiles_x;
      o.g = (int32_t)(vg - (int64_t)c * n);
      o.key = query_depth_key(zmin[vg], query_key_shift(dbits));
      o.pad = 0;
      own[w][lane] = o;
    }
  }
  int incl = cnt;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  const int total = __shfl(incl, 63, 64);
  const int64_t e0 = offsets[base];
  if (lane == 0 && e0 + total > cap && total > 0) atomicOr(&status->flags, 1);
  __builtin_amdgcn_wave_barrier();
  const int excl = incl - cnt;
  for (int j0 = 0; j0 < total; j0 += 64) {
    const int j = j0 + lane;
    int lo = 0, hi = 63;
#pragma unroll
    for (int it = 0; it < 6; ++it) {
      const int mid = (lo + hi) >> 1;
      const bool right = __shfl(incl, mid, 64) <= j;
      lo = right ? mid + 1 : lo;
      hi = right ? hi : mid;
    }
    const int before = __shfl(excl, lo, 64);
    const int64_t e = e0 + j;
    if (j < total && e < cap) {
      const EmitOwner o = own[w][lo];
      const int local = j - before;
      const uint32_t t = (uint32_t)(o.toff + (o.ty0 + local / o.nx) * o.tiles_x + (o.tx0 + local % o.nx));
      keys[e] = (t << dbits) | o.key;
      vals[e] = (uint32_t)o.g;
    }
  }
}

__global__ __launch_bounds__(256) void k_ranges32(const uint32_t* keys, const int64_t* count, int64_t cap, int dbits,
                                                  int2* ranges) {
  const int64_t n = live_count(count, cap);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t t = keys[i] >> dbits;
  if (i == 0 || (keys[i - 1] >> dbits) != t) ranges[t].x = (int)i;
  if (i == n - 1 || (keys[i + 1] >> dbits) != t) ranges[t].y = (int)(i + 1);
}

__global__ __launch_bounds__(256) void k_fill_ranges(int2* ranges, int64_t n_tiles) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_tiles) ranges[i] = make_int2(0, 0);
}

hipError_t launch_cam_table(const sof_camera* d_cams, int n_cams, int tile, CamInfo* out, StatusBlock* status,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_cam_table, dim3(1), dim3(64), 0, s, d_cams, n_cams, tile, out, status);
  return hipGetLastError();
}

hipError_t launch_bin_sort(int64_t n, const sof_camera* d_cams, int n_cams, int64_t n_tiles, int tile, int64_t cap,
                           int query_keys, const void* proj, void* bins, hipStream_t s, int* parity) {
  const int64_t vn = n * (int64_t)n_cams;
  const ProjLayout P = ProjLayout::make(vn, query_keys != 0, n);
  const BinsLayout B = BinsLayout::make(vn, n_cams, cap, n_tiles);
  const char* pb = (const char*)proj;
  char* bb = (char*)bins;
  StatusBlock* status = (StatusBlock*)(bb + B.status);
  CamInfo* cams = (CamInfo*)(bb + B.cams);
  int32_t* counts = (int32_t*)(bb + B.counts);
  int64_t* offsets = (int64_t*)(bb + B.offsets);
  int64_t* scan_tmp = (int64_t*)(bb + B.scan_tmp);
  // render-list roles of the shared regions (see BinsLayout)
  uint64_t* bucket = (uint64_t*)(bb + B.keys0);
  uint2* inst = (uint2*)(bb + B.keys1);            // consumed by the scatter, then merge scratch
  uint64_t* tmp = (uint64_t*)(bb + B.keys1);
  uint32_t* vals = (uint32_t*)(bb + B.vals0);
  uint32_t* rank = (uint32_t*)(bb + B.vals1);
  int32_t* gid = (int32_t*)(bb + B.gid);
  int2* ranges = (int2*)(bb + B.ranges);
  const short4* rect = (const short4*)(pb + P.rect);
  const float4* geom = (const float4*)(pb + P.geom);
  const float* zmin = (const float*)(pb + P.zmin);

  const int th = 256;
  // init, counts and chunk sums; the chunk scan (writes the instance total); the offsets
  const int64_t nch = div_up(vn > 0 ? vn : 1, kScanChunk);
  hipLaunchKernelGGL(k_bin_count, dim3((unsigned)nch), dim3(kScanThreads), 0, s, d_cams, n_cams, tile, cams, status,
                     ranges, n_tiles, rect, vn, counts, scan_tmp);
  hipLaunchKernelGGL((k_scan_chunks<int64_t>), dim3(1), dim3(kScanThreads), 0, s, scan_tmp, nch, &status->count);
  if (vn > 0) {
    hipLaunchKernelGGL((k_scan_apply<int32_t, int64_t>), dim3((unsigned)nch), dim3(kScanThreads), 0, s, counts, vn,
                       scan_tmp, offsets);
    hipLaunchKernelGGL(k_emit, dim3((unsigned)div_up(vn, 256)), dim3(256), 0, s, rect, geom, zmin, n, vn, tile, cams,
                       counts, offsets, cap, query_keys, inst, rank, gid, ranges, status);
  }
  hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(kTileScanThreads), 0, s, ranges, n_tiles);
  if (cap > 0) {
    hipLaunchKernelGGL(k_tile_scatter, dim3((unsigned)div_up(cap, th)), dim3(th), 0, s, inst, rank, ranges,
                       &status->count, cap, bucket);
  }
  hipLaunchKernelGGL(k_tile_sort, dim3((unsigned)n_tiles), dim3(kTileSortThreads), 0, s, ranges, bucket, tmp, vals);
  *parity = 0;
  return hipGetLastError();
}

int query_key_bits(int64_t n_tiles) {
  const int tb = bits_for(n_tiles);
  return tb <= 20 ? 32 - tb : 0;          // 0: tile ids too wide for 32-bit keys
}

hipError_t launch_query_bin_sort(int64_t n, const sof_camera* d_cams, int n_cams, int64_t n_tiles, int tile,
                                 int64_t cap, const void* proj, void* bins, hipStream_t s, int* parity,
                                 int* dbits_out) {
  const int dbits = query_key_bits(n_tiles);
  *dbits_out = dbits;
  if (dbits == 0) return launch_bin_sort(n, d_cams, n_cams, n_tiles, tile, cap, 1, proj, bins, s, parity);
  const int64_t vn = n * (int64_t)n_cams;
  const ProjLayout P = ProjLayout::make(vn, true, n);
  const BinsLayout B = BinsLayout::make(vn, n_cams, cap, n_tiles);
  const char* pb = (const char*)proj;
  char* bb = (char*)bins;
  StatusBlock* status = (StatusBlock*)(bb + B.status);
  CamInfo* cams = (CamInfo*)(bb + B.cams);
  int32_t* counts = (int32_t*)(bb + B.counts);
  int64_t* offsets = (int64_t*)(bb + B.offsets);
  int64_t* scan_tmp = (int64_t*)(bb + B.scan_tmp);
  uint32_t* k0 = (uint32_t*)(bb + B.keys0);
  uint32_t* k1 = (uint32_t*)(bb + B.keys1);
  uint32_t* v0 = (uint32_t*)(bb + B.vals0);
  uint32_t* v1 = (uint32_t*)(bb + B.vals1);
  int32_t* hist = (int32_t*)(bb + B.hist);
  int32_t* hist_tmp = (int32_t*)(bb + B.hist_tmp);
  int2* ranges = (int2*)(bb + B.ranges);
  const short4* rect = (const short4*)(pb + P.rect);
  const float* zmin = (const float*)(pb + P.zmin);

  hipLaunchKernelGGL(k_cam_table, dim3(1), dim3(64), 0, s, d_cams, n_cams, tile, cams, status);
  const int th = 256;
  if (vn > 0) hipLaunchKernelGGL(k_count, dim3((unsigned)div_up(vn, th)), dim3(th), 0, s, rect, vn, tile, counts);
  hipError_t e = exclusive_scan<int32_t, int64_t>(counts, vn, offsets, scan_tmp, &status->count, s);
  if (e != hipSuccess) return e;
  if (vn > 0)
    hipLaunchKernelGGL(k_emit_query32, dim3((unsigned)div_up(vn, 256)), dim3(256), 0, s, rect, zmin, n, vn, tile, cams,
                       counts, offsets, cap, dbits, k0, v0, status);
  e = radix_sort<uint32_t>(k0, v0, k1, v1, &status->count, cap, 32, hist, hist_tmp, parity, s);
  if (e != hipSuccess) return e;
  const uint32_t* ks = *parity ? k1 : k0;
  hipLaunchKernelGGL(k_fill_ranges, dim3((unsigned)div_up(n_tiles > 0 ? n_tiles : 1, th)), dim3(th), 0, s, ranges, n_tiles);
  if (cap > 0)
    hipLaunchKernelGGL(k_ranges32, dim3((unsigned)div_up(cap, th)), dim3(th), 0, s, ks, &status->count, cap, dbits,
                       ranges);
  return hipGetLastError();
}

}  // namespace sof
