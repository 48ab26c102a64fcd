// C ABI entry points: argument checks, buffer layouts and kernel launches.  No allocation,
// no synchronisation, no device-to-host reads.
#include <stdlib.h>
#include <string.h>
#include <stdio.h>

#include <mutex>

#include "launch.h"

using namespace sof;

namespace {

bool trace_enabled() {
  static const int on = [] {
    const char* e = getenv("SOF_TRACE");
    return (e && e[0] == '1') ? 1 : 0;
  }();
  return on != 0;
}

int check_opts(const sof_options* o) {
  if (!o) return SOF_E_ARG;
  if (o->tile != 8 && o->tile != 16 && o->tile != 32) return SOF_E_ARG;
  if (o->window < 0) return SOF_E_ARG;
  if (!render_supported(o->tile, o->window)) return SOF_E_UNSUPPORTED;
  if (!(o->near_plane > 0.f)) return SOF_E_ARG;
  if (o->capacity < 0 || o->capacity >= (int64_t(1) << 31)) return SOF_E_ARG;
  if (o->order_slots < 0 || o->order_slots > kMaxOrderSlots) return SOF_E_ARG;
  return SOF_OK;
}

int check_cams(const sof_camera* h, int n_cams, int64_t* n_tiles, int tile) {
  if (!h || n_cams < 1) return SOF_E_ARG;
  int64_t t = 0;
  for (int c = 0; c < n_cams; ++c) {
    if (h[c].width < 1 || h[c].height < 1 || h[c].width > 32767 || h[c].height > 32767) return SOF_E_ARG;
    if (!(h[c].fx > 0.f) || !(h[c].fy > 0.f)) return SOF_E_ARG;
    t += (int64_t)((h[c].width + tile - 1) / tile) * ((h[c].height + tile - 1) / tile);
  }
  if (t >= (int64_t(1) << 31)) return SOF_E_ARG;
  *n_tiles = t;
  return SOF_OK;
}

int check_gauss(const sof_gaussians* g, bool need_params) {
  if (!g || g->n < 0 || g->n >= (int64_t(1) << 31)) return SOF_E_ARG;
  if (g->sh_degree < 0 || g->sh_degree > 3) return SOF_E_ARG;
  if (need_params && g->n > 0 && (!g->means || !g->scales || !g->quats || !g->opacities || !g->sh)) return SOF_E_ARG;
  return SOF_OK;
}

int hip_status(hipError_t e) { return e == hipSuccess ? SOF_OK : SOF_E_HIP; }


hipEvent_t g_timing[2 * kTimedKernels] = {};

// Scratch of sof_render_bwd_static: the per-instance gradient partials (16 floats per tile
// instance) of up to kStaticInstances instances, 64 MiB on every device the library runs on,
// held until the process ends.  Host code never passes `scratch` itself to a kernel (on the
// host it names a stand-in, not device memory): its device address, looked up once per device
// with that device current, is kept in g_scratch_ptr.
constexpr int64_t kStaticInstances = int64_t(1) << 20;
static __device__ __align__(256) float scratch[kStaticInstances * kGradFields];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int static_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SOF_E_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SOF_E_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SOF_OK;
}

}  // namespace

namespace sof {
void timing_mark(TimedKernel k, int end, hipStream_t s) {
  hipEvent_t ev = g_timing[2 * (int)k + end];
  if (ev) (void)hipEventRecord(ev, s);                // instrumentation only: a failed mark is not an error
}
}  // namespace sof

extern "C" {

size_t sof_read_status_offset(void) { return 0; }

int sof_set_timing_events(void* const* events) {
  for (int k = 0; k < 2 * kTimedKernels; ++k) g_timing[k] = events ? (hipEvent_t)events[k] : nullptr;
  return SOF_OK;
}

const char* sof_strerror(int code) {
  switch (code) {
    case SOF_OK: return "ok";
    case SOF_E_ARG: return "invalid argument";
    case SOF_E_WORKSPACE: return "workspace buffer too small";
    case SOF_E_CAPACITY: return "tile-instance capacity exceeded";
    case SOF_E_HIP: return "HIP launch failed";
    case SOF_E_UNSUPPORTED: return "unsupported tile/window combination";
    case SOF_E_SCRATCH: return "capacity exceeds the static scratch of sof_render_bwd_static (2^20 instances)";
    default: return "unknown sof status";
  }
}

int sof_workspace_size(int64_t n, const sof_camera* h_cams, int32_t n_cams, const sof_options* opts,
                       size_t* proj_bytes, size_t* bins_bytes, size_t* grad_bytes, size_t* order_bytes) {
  int st = check_opts(opts);
  if (st) return st;
  if (n < 0 || n >= (int64_t(1) << 31)) return SOF_E_ARG;
  int64_t n_tiles = 0;
  if ((st = check_cams(h_cams, n_cams, &n_tiles, opts->tile))) return st;
  const int64_t vn = n * n_cams;
  if (proj_bytes) *proj_bytes = ProjLayout::make(vn).total;
  if (bins_bytes) *bins_bytes = BinsLayout::make(vn, n_cams, opts->capacity, n_tiles).total;
  if (grad_bytes) *grad_bytes = (size_t)opts->capacity * kGradFields * sizeof(float);
  if (order_bytes) *order_bytes = opts->order_slots > 0 ? OrderLayout::make(n_tiles, opts->tile, opts->order_slots).total : 0;
  return SOF_OK;
}

int sof_project(const sof_gaussians* g, const sof_camera* h_cams, const sof_camera* d_cams, int32_t n_cams,
                const sof_options* opts, void* proj, size_t proj_bytes, hipStream_t stream) {
  int st = check_opts(opts);
  if (st) return st;
  if ((st = check_gauss(g, true))) return st;
  int64_t n_tiles = 0;
  if ((st = check_cams(h_cams, n_cams, &n_tiles, opts->tile))) return st;
  if (!d_cams || (!proj && g->n > 0)) return SOF_E_ARG;
  if (proj_bytes < ProjLayout::make(g->n * n_cams).total) return SOF_E_WORKSPACE;
  if (trace_enabled()) fprintf(stderr, "[sof] project n=%lld cams=%d\n", (long long)g->n, n_cams);
  return hip_status(launch_project(g, d_cams, n_cams, opts->near_plane, proj, stream));
}

int sof_bin_sort(int64_t n, const sof_camera* h_cams, const sof_camera* d_cams, int32_t n_cams,
                 const sof_options* opts, const void* proj, size_t proj_bytes, void* bins, size_t bins_bytes,
                 hipStream_t stream) {
  int st = check_opts(opts);
  if (st) return st;
  if (n < 0 || n >= (int64_t(1) << 31)) return SOF_E_ARG;
  int64_t n_tiles = 0;
  if ((st = check_cams(h_cams, n_cams, &n_tiles, opts->tile))) return st;
  if (!d_cams || !bins || (!proj && n > 0)) return SOF_E_ARG;
  const int64_t vn = n * n_cams;
  if (proj_bytes < ProjLayout::make(vn).total) return SOF_E_WORKSPACE;
  if (bins_bytes < BinsLayout::make(vn, n_cams, opts->capacity, n_tiles).total) return SOF_E_WORKSPACE;
  if (trace_enabled())
    fprintf(stderr, "[sof] bin_sort n=%lld cams=%d tiles=%lld cap=%lld\n", (long long)n, n_cams, (long long)n_tiles,
            (long long)opts->capacity);
  int parity = 0;
  return hip_status(launch_bin_sort(n, d_cams, n_cams, n_tiles, opts->tile, opts->capacity,
                                    (opts->flags & SOF_QUERY_KEYS) ? 1 : 0, proj, bins, stream, &parity));
}

static int fill_fwd_args(int64_t n, const sof_camera* h_cams, const sof_camera* d_cams, int32_t n_cams,
                         const sof_options* opts, const void* proj, size_t proj_bytes, const void* bins,
                         size_t bins_bytes, RenderFwdArgs* a, int64_t* n_tiles_out) {
  int st = check_opts(opts);
  if (st) return st;
  if (n < 0 || n >= (int64_t(1) << 31)) return SOF_E_ARG;
  int64_t n_tiles = 0;
  if ((st = check_cams(h_cams, n_cams, &n_tiles, opts->tile))) return st;
  if (!d_cams || !bins || (!proj && n > 0)) return SOF_E_ARG;
  const int64_t vn = n * n_cams;
  const ProjLayout P = ProjLayout::make(vn);
  const BinsLayout B = BinsLayout::make(vn, n_cams, opts->capacity, n_tiles);
  if (proj_bytes < P.total) return SOF_E_WORKSPACE;
  if (bins_bytes < B.total) return SOF_E_WORKSPACE;
  const char* pb = (const char*)proj;
  const char* bb = (const char*)bins;
  memset(a, 0, sizeof(*a));
  a->n = n;
  a->cams = d_cams;
  a->cam_info = (const CamInfo*)(bb + B.cams);
  a->n_cams = n_cams;
  a->near_plane = opts->near_plane;
  a->bg[0] = opts->bg[0]; a->bg[1] = opts->bg[1]; a->bg[2] = opts->bg[2];
  a->flags = opts->flags;
  a->geom = (const float4*)(pb + P.geom);
  a->app = (const float4*)(pb + P.app);
  a->rect = (const short4*)(pb + P.rect);
  a->ranges = (const int2*)(bb + B.ranges);
  a->vals = (const uint32_t*)(bb + B.vals0);                  // sorted tile lists (emission indices)
  a->gid = (const int32_t*)(bb + B.gid);
  *n_tiles_out = n_tiles;
  return SOF_OK;
}

// The recorded blend order (null: none).  Needs opts->order_slots > 0 and a buffer of the
// size sof_workspace_size gives.
static int set_order(const sof_options* opts, int64_t n_tiles, const void* order, size_t order_bytes,
                     RenderFwdArgs* a) {
  a->order = nullptr;
  a->order_flags = nullptr;
  a->order_slots = 0;
  if (!order) return SOF_OK;
  if (opts->order_slots <= 0) return SOF_E_ARG;
  const OrderLayout L = OrderLayout::make(n_tiles, opts->tile, opts->order_slots);
  if (order_bytes < L.total) return SOF_E_WORKSPACE;
  char* ob = (char*)order;
  a->order_flags = (int32_t*)(ob + L.flags);
  a->order = (uint16_t*)(ob + L.rec);
  a->order_slots = opts->order_slots;
  return SOF_OK;
}

int sof_render_fwd(int64_t n, const sof_camera* h_cams, const sof_camera* d_cams, int32_t n_cams,
                   const sof_options* opts, const void* proj, size_t proj_bytes, const void* bins, size_t bins_bytes,
                   float* rgb, float* acc, float* depth, float* normal, float* aux, float* losses,
                   void* order, size_t order_bytes, hipStream_t stream) {
  RenderFwdArgs a;
  int64_t n_tiles = 0;
  int st = fill_fwd_args(n, h_cams, d_cams, n_cams, opts, proj, proj_bytes, bins, bins_bytes, &a, &n_tiles);
  if (st) return st;
  if ((st = set_order(opts, n_tiles, order, order_bytes, &a))) return st;
  if (a.order && !aux) return SOF_E_ARG;                // the backward reads both
  a.rgb = rgb; a.acc = acc; a.depth = depth; a.normal = normal; a.aux = aux; a.losses = losses;
  if (trace_enabled())
    fprintf(stderr, "[sof] render_fwd tiles=%lld tile=%d window=%d\n", (long long)n_tiles, opts->tile, opts->window);
  timing_mark(kTimeRenderFwd, 0, stream);
  const hipError_t e = launch_render_fwd(a, opts->tile, opts->window, n_tiles, stream);
  timing_mark(kTimeRenderFwd, 1, stream);
  return hip_status(e);
}

int sof_render_order(int64_t n, const sof_camera* h_cams, const sof_camera* d_cams, int32_t n_cams,
                     const sof_options* opts, const void* proj, size_t proj_bytes, const void* bins, size_t bins_bytes,
                     const int32_t* slot, int64_t n_slots, int32_t max_entries, int32_t* stream_ids,
                     float* stream_keys, int32_t* emit_ids, int32_t* counts, hipStream_t stream) {
  RenderFwdArgs a;
  int64_t n_tiles = 0;
  int st = fill_fwd_args(n, h_cams, d_cams, n_cams, opts, proj, proj_bytes, bins, bins_bytes, &a, &n_tiles);
  if (st) return st;
  if (!slot || n_slots < 0 || max_entries < 0) return SOF_E_ARG;
  if (n_slots > 0 && (!counts || (max_entries > 0 && (!stream_ids || !stream_keys || !emit_ids)))) return SOF_E_ARG;
  if (n_slots > 0 && max_entries > 0 && n_slots > INT64_MAX / max_entries) return SOF_E_ARG;
  a.dump.slot = slot;
  a.dump.n_slots = n_slots;
  a.dump.max_entries = max_entries;
  a.dump.stream_ids = stream_ids;
  a.dump.stream_keys = stream_keys;
  a.dump.emit_ids = emit_ids;
  a.dump.counts = counts;
  if (trace_enabled())
    fprintf(stderr, "[sof] render_order tiles=%lld slots=%lld max=%d\n", (long long)n_tiles, (long long)n_slots,
            max_entries);
  return hip_status(launch_render_fwd(a, opts->tile, opts->window, n_tiles, stream));
}

int sof_filter3d(const sof_gaussians* g, const sof_camera* h_cams, const sof_camera* d_cams, int32_t n_cams,
                 float near_plane, float k, float* var, float* scales_out, float* opacities_out, hipStream_t stream) {
  if (!g || g->n < 0 || g->n >= (int64_t(1) << 31) || n_cams < 0 || !(near_plane > 0.f) || !(k >= 0.f))
    return SOF_E_ARG;
  if (g->n > 0 && (!g->means || !g->scales || !g->opacities || !var || !scales_out || !opacities_out))
    return SOF_E_ARG;
  if (n_cams > 0 && (!h_cams || !d_cams)) return SOF_E_ARG;
  return hip_status(launch_filter3d(g->means, g->scales, g->opacities, g->n, d_cams, n_cams, near_plane, k, var,
                                    scales_out, opacities_out, stream));
}

int sof_filter3d_bwd(const sof_gaussians* g, const float* var, const float* d_scales_out,
                     const float* d_opacities_out, float* d_scales, float* d_opacities, hipStream_t stream) {
  if (!g || g->n < 0 || g->n >= (int64_t(1) << 31)) return SOF_E_ARG;
  if (g->n > 0 && (!g->scales || !g->opacities || !var || !d_scales || !d_opacities)) return SOF_E_ARG;
  return hip_status(launch_filter3d_bwd(g->scales, g->opacities, var, g->n, d_scales_out, d_opacities_out, d_scales,
                                        d_opacities, stream));
}

int sof_render_opacity(int64_t n, const sof_camera* h_cams, const sof_camera* d_cams, int32_t n_cams,
                       const sof_options* opts, const void* proj, size_t proj_bytes, const void* bins,
                       size_t bins_bytes, const float* depth, const float* aux, const float* losses,
                       const void* order, size_t order_bytes, float* opacity, hipStream_t stream) {
  RenderOpaArgs a;
  int64_t n_tiles = 0;
  int st = fill_fwd_args(n, h_cams, d_cams, n_cams, opts, proj, proj_bytes, bins, bins_bytes, &a.f, &n_tiles);
  if (st) return st;
  if ((st = set_order(opts, n_tiles, order, order_bytes, &a.f))) return st;
  if (!depth || !aux || !opacity) return SOF_E_ARG;
  a.f.depth = (float*)depth;
  a.f.aux = (float*)aux;
  a.tail = losses;
  a.opa = opacity;
  if (trace_enabled())
    fprintf(stderr, "[sof] render_opacity tiles=%lld tile=%d window=%d\n", (long long)n_tiles, opts->tile, opts->window);
  return hip_status(launch_render_opa(a, opts->tile, opts->window, n_tiles, stream));
}

static int render_bwd_impl(const sof_gaussians* g, const sof_camera* h_cams, const sof_camera* d_cams,
                           int32_t n_cams, const sof_options* opts, const void* proj, size_t proj_bytes,
                           const void* bins, size_t bins_bytes, const float* rgb, const float* normal,
                           const float* aux, const void* order, size_t order_bytes, const float* d_rgb,
                           const float* d_acc, const float* d_depth, const float* d_normal, const float* depth,
                           const float* opacity, const float* d_opacity, const float* losses, const float* d_losses,
                           void* grads, size_t grad_bytes, float* d_means, float* d_scales, float* d_quats,
                           float* d_opacities, float* d_sh, hipStream_t stream) {
  int st = check_gauss(g, true);
  if (st) return st;
  RenderBwdArgs b;
  int64_t n_tiles = 0;
  st = fill_fwd_args(g->n, h_cams, d_cams, n_cams, opts, proj, proj_bytes, bins, bins_bytes, &b.f, &n_tiles);
  if (st) return st;
  if ((st = set_order(opts, n_tiles, order, order_bytes, &b.f))) return st;
  if (!rgb || !aux) return SOF_E_ARG;
  if (d_normal && !normal) return SOF_E_ARG;            // its suffix sums need the forward's normal
  if (g->n > 0 && (!d_means || !d_scales || !d_quats || !d_opacities || !d_sh)) return SOF_E_ARG;
  if (!grads && opts->capacity > 0) return SOF_E_ARG;
  if (grad_bytes < (size_t)opts->capacity * kGradFields * sizeof(float)) return SOF_E_WORKSPACE;
  const int64_t vn = g->n * n_cams;
  const ProjLayout P = ProjLayout::make(vn);
  const BinsLayout B = BinsLayout::make(vn, n_cams, opts->capacity, n_tiles);
  const char* pb = (const char*)proj;
  const char* bb = (const char*)bins;
  b.bwdr = (const float4*)(pb + P.bwdr);
  b.out_rgb = rgb; b.out_normal = normal;
  b.d_rgb = d_rgb; b.d_acc = d_acc; b.d_depth = d_depth; b.d_normal = d_normal;
  b.grads = (float*)grads;
  b.f.aux = (float*)aux;
  if (d_opacity && (!depth || !opacity)) return SOF_E_ARG;
  b.out_depth = d_opacity ? depth : nullptr;
  b.opa = d_opacity ? opacity : nullptr;
  b.d_opa = d_opacity;
  if (d_losses && !losses) return SOF_E_ARG;
  b.losses = d_losses ? losses : nullptr;
  b.d_losses = d_losses;
  if (trace_enabled())
    fprintf(stderr, "[sof] render_bwd tiles=%lld tile=%d window=%d\n", (long long)n_tiles, opts->tile, opts->window);
  timing_mark(kTimeRenderBwd, 0, stream);
  hipError_t e = launch_render_bwd(b, opts->tile, opts->window, n_tiles, stream);
  timing_mark(kTimeRenderBwd, 1, stream);
  if (e != hipSuccess) return SOF_E_HIP;
  ProjectBwdArgs pa;
  pa.means = g->means; pa.scales = g->scales; pa.quats = g->quats; pa.opac = g->opacities; pa.sh = g->sh;
  pa.sh_degree = g->sh_degree; pa.n = g->n; pa.cams = d_cams; pa.n_cams = n_cams;
  pa.counts = (const int32_t*)(bb + B.counts);
  pa.offsets = (const int64_t*)(bb + B.offsets);
  pa.count_total = (const int64_t*)(bb + B.status);
  pa.cap = opts->capacity;
  pa.grads = (float*)grads;
  pa.d_means = d_means; pa.d_scales = d_scales; pa.d_quats = d_quats; pa.d_opac = d_opacities; pa.d_sh = d_sh;
  return hip_status(launch_project_bwd(pa, stream));
}

int sof_render_bwd(const sof_gaussians* g, const sof_camera* h_cams, const sof_camera* d_cams, int32_t n_cams,
                   const sof_options* opts, const void* proj, size_t proj_bytes, const void* bins, size_t bins_bytes,
                   const float* rgb, const float* normal, const float* aux, const void* order, size_t order_bytes,
                   const float* d_rgb, const float* d_acc,
                   const float* d_depth, const float* d_normal, const float* depth, const float* opacity,
                   const float* d_opacity, const float* losses, const float* d_losses, void* grads,
                   size_t grad_bytes, float* d_means, float* d_scales, float* d_quats, float* d_opacities,
                   float* d_sh, hipStream_t stream) {
  return render_bwd_impl(g, h_cams, d_cams, n_cams, opts, proj, proj_bytes, bins, bins_bytes, rgb, normal, aux,
                         order, order_bytes, d_rgb, d_acc, d_depth, d_normal, depth, opacity, d_opacity, losses,
                         d_losses, grads, grad_bytes, d_means, d_scales, d_quats, d_opacities, d_sh, stream);
}

int sof_render_bwd_static(const sof_gaussians* g, const sof_camera* h_cams, const sof_camera* d_cams,
                          int32_t n_cams, const sof_options* opts, const void* proj, size_t proj_bytes,
                          const void* bins, size_t bins_bytes, const float* rgb, const float* normal,
                          const float* aux, const void* order, size_t order_bytes, const float* d_rgb,
                          const float* d_acc, const float* d_depth, const float* d_normal, const float* depth,
                          const float* opacity, const float* d_opacity, const float* losses, const float* d_losses,
                          float* d_means, float* d_scales, float* d_quats, float* d_opacities, float* d_sh,
                          hipStream_t stream) {
  if (!opts) return SOF_E_ARG;
  if (opts->capacity > kStaticInstances) return SOF_E_SCRATCH;   // before any device call
  void* ptr = nullptr;
  const int st = static_scratch(&ptr);
  if (st) return st;
  return render_bwd_impl(g, h_cams, d_cams, n_cams, opts, proj, proj_bytes, bins, bins_bytes, rgb, normal, aux,
                         order, order_bytes, d_rgb, d_acc, d_depth, d_normal, depth, opacity, d_opacity, losses,
                         d_losses, ptr, sizeof(scratch), d_means, d_scales, d_quats, d_opacities, d_sh, stream);
}

}  // extern "C"
