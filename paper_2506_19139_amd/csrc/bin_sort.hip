// Duplication of Gaussians into tiles and the per-tile key sort (level 0 of the
// hierarchical resort, Sec. 3.1), plus the device-wide scan and the stable LSD radix sort
// used by the query's 32-bit lists.  Instance counts stay on the device: every grid is sized
// from static capacities and reads the live count from the status block, so the sequence can
// be captured in a graph.
//
// Render lists (and the query's lists when tile ids need more than 20 bits) are built by
// bucketing, not by a global sort: each instance takes its rank inside its tile with an
// atomic increment of the tile's counter, one workgroup scans the counters into the tile
// ranges, instances are scattered into their tile's range, and one workgroup per tile sorts
// its range in LDS by (depth key, emission index).  Emission indices grow with the Gaussian
// index inside a camera, and a tile holds one camera's instances, so this is the order
// (tile, depth key, Gaussian index) whatever order the atomics handed out.
//
// Radix sort: 8-bit digits, 2048 keys per workgroup of 256 lanes (4 wave64s).  Per pass a
// histogram kernel writes per-(digit, block) counts digit-major, an exclusive scan turns
// them into global offsets, and a scatter kernel ranks keys stably inside the workgroup:
// each wave owns 512 consecutive keys, walks them in input order, groups equal digits with
// 8 ballots and keeps running per-digit counts in LDS.
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

template <typename Tin, typename Tacc>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const Tin* in, int64_t n, Tacc* sums) {
  __shared__ Tacc lw[4];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
  Tacc s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) s += (Tacc)in[base + k];
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
  Tout v[kScanItems];
  Tout s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = base + k < n ? (Tout)in[base + k] : 0;
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

template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const K* keys, const int64_t* count, int64_t cap,
                                                             int shift, int32_t* hist, int64_t nblocks) {
  __shared__ int32_t cnt[4][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int t = threadIdx.x; t < 4 * 256; t += kSortThreads) (&cnt[0][0])[t] = 0;
  __syncthreads();
  const int64_t n = live_count(count, cap);
  const int64_t start = (int64_t)blockIdx.x * sort_tile<K>() + (int64_t)w * (sort_items<K>() * 64);
#pragma unroll
  for (int it = 0; it < sort_items<K>(); ++it) {
    const int64_t idx = start + it * 64 + lane;
    if (idx < n) {
      const int d = (int)((keys[idx] >> shift) & 0xFF);
      atomicAdd(&cnt[w][d], 1);
    }
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
// an atomic increment of the tile's counter (ranges[t].y, zeroed by k_bin_init).  Instances
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

// Camera table, status reset and zeroed tile counters.
__global__ __launch_bounds__(256) void k_bin_init(const sof_camera* cams, int n_cams, int tile, CamInfo* out,
                                                  StatusBlock* status, int2* ranges, int64_t n_tiles) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_tiles) ranges[i] = make_int2(0, 0);
  if (i != 0) return;
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

// Bitonic sort of P (a power of two, <= kTileSortCap) keys in LDS by the whole workgroup,
// with the network unrolled at compile time (no scalar loop or branch work per stage).  Lane
// t takes the compare-exchange pairs t, t + 256, ...; pair p of a stage with distance j joins
// entries i = 2 j (p / j) + p mod j and i + j.  For j < 64 both entries lie in one 64-entry
// block whose 32 pairs belong to 32 consecutive lanes of one wave, so those stages need only
// the wave's own ordering of its LDS accesses; a workgroup barrier is taken only around
// stages whose pairs span waves (j >= 64).
constexpr int kTileSortThreads = 256, kTileSortCap = 2048;

__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int P, int K, int J>
__device__ inline void bitonic_stage(uint64_t* s) {
  constexpr int kPairs = P / 2;
#pragma unroll
  for (int p0 = 0; p0 < kPairs; p0 += kTileSortThreads) {
    const int p = p0 + (int)threadIdx.x;
    if (kPairs % kTileSortThreads == 0 || p < kPairs) {
      const int i = ((p & ~(J - 1)) << 1) | (p & (J - 1));
      const int l = i | J;
      const uint64_t a = s[i], b = s[l];
      const bool sw = (a > b) == ((i & K) == 0);
      s[i] = sw ? b : a;
      s[l] = sw ? a : b;
    }
  }
  constexpr bool next_crosses = (J > 1) ? ((J >> 1) >= 64) : (2 * K <= P && K >= 64);
  if constexpr (J >= 64 || next_crosses) {
    __syncthreads();
  } else {
    wave_lds_sync();
  }
}

template <int P, int K, int J>
__device__ inline void bitonic_merge(uint64_t* s) {
  bitonic_stage<P, K, J>(s);
  if constexpr (J > 1) bitonic_merge<P, K, J / 2>(s);
}

template <int P, int K = 2>
__device__ inline void bitonic_sort(uint64_t* s) {
  bitonic_merge<P, K, K / 2>(s);
  if constexpr (K < P) bitonic_sort<P, 2 * K>(s);
}

// Sort s[0, P) for the smallest power of two P >= L (entries L..P-1 hold the largest key).
__device__ __attribute__((always_inline)) inline void lds_bitonic(uint64_t* s, int P) {
  switch (P) {
    case 2: bitonic_sort<2>(s); break;
    case 4: bitonic_sort<4>(s); break;
    case 8: bitonic_sort<8>(s); break;
    case 16: bitonic_sort<16>(s); break;
    case 32: bitonic_sort<32>(s); break;
    case 64: bitonic_sort<64>(s); break;
    case 128: bitonic_sort<128>(s); break;
    case 256: bitonic_sort<256>(s); break;
    case 512: bitonic_sort<512>(s); break;
    case 1024: bitonic_sort<1024>(s); break;
    default: bitonic_sort<kTileSortCap>(s); break;
  }
  __syncthreads();
}

// One workgroup per tile: its range sorted by (depth key, emission index); the emission
// indices are written to vals.  Ranges above kTileSortCap (not met at the benchmark's
// sizes, where the longest list is about a thousand) are sorted in chunks of kTileSortCap
// in LDS and then merged pairwise in global memory, each element placed by its rank in the
// other run (keys are unique), ping-ponging between bucket and tmp.
__global__ __launch_bounds__(kTileSortThreads) void k_tile_sort(const int2* ranges, uint64_t* bucket, uint64_t* tmp,
                                                                uint32_t* vals) {
  __shared__ uint64_t s[kTileSortCap];
  const int2 rg = ranges[blockIdx.x];
  const int L = rg.y - rg.x;
  if (L <= 0) return;
  const bool small = L <= kTileSortCap;
  int P = 2;
  while (P < L && P < kTileSortCap) P <<= 1;
  uint64_t* src = bucket + rg.x;
  uint64_t* dst = tmp + rg.x;
  // one LDS sort per chunk of kTileSortCap entries (a single chunk for a short list, whose
  // sorted emission indices go straight to vals)
  for (int c0 = 0; c0 < L; c0 += kTileSortCap) {
    const int m = min(kTileSortCap, L - c0);
    for (int i = threadIdx.x; i < P; i += kTileSortThreads) s[i] = i < m ? src[c0 + i] : ~0ull;
    __syncthreads();
    lds_bitonic(s, P);
    if (small) {
      for (int i = threadIdx.x; i < m; i += kTileSortThreads) vals[rg.x + i] = (uint32_t)s[i];
    } else {
      for (int i = threadIdx.x; i < m; i += kTileSortThreads) src[c0 + i] = s[i];
    }
    __syncthreads();
  }
  if (small) return;
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
  hipLaunchKernelGGL(k_bin_init, dim3((unsigned)div_up(n_tiles > 0 ? n_tiles : 1, th)), dim3(th), 0, s, d_cams, n_cams,
                     tile, cams, status, ranges, n_tiles);
  if (vn > 0) {
    hipLaunchKernelGGL(k_count, dim3((unsigned)div_up(vn, th)), dim3(th), 0, s, rect, vn, tile, counts);
  }
  hipError_t e = exclusive_scan<int32_t, int64_t>(counts, vn, offsets, scan_tmp, &status->count, s);
  if (e != hipSuccess) return e;
  if (vn > 0) {
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
