// Host-side launch helpers implemented in the individual kernel files.
#pragma once

#include "sof_internal.h"

namespace sof {

template <typename Tin, typename Tout>
hipError_t exclusive_scan(const Tin* in, int64_t n, Tout* out, Tout* tmp, int64_t* total, hipStream_t s);

template <typename K>
hipError_t radix_sort(K* k0, uint32_t* v0, K* k1, uint32_t* v1, const int64_t* count, int64_t cap, int bits,
                      int32_t* hist, int32_t* hist_tmp, int* out_parity, hipStream_t s);

hipError_t launch_project(const sof_gaussians* g, const sof_camera* d_cams, int n_cams, float near_plane,
                          void* proj, hipStream_t stream, bool query = false);

// parity: which of the two key/value buffers holds the sorted instances (0 or 1).
hipError_t launch_bin_sort(int64_t n, const sof_camera* d_cams, int n_cams, int64_t n_tiles, int tile, int64_t cap,
                           int query_keys, const void* proj, void* bins, hipStream_t s, int* parity);
// Per-camera tile / pixel offsets on the device (also resets the status block).
// Tile lists for the opacity query: 32-bit keys (tile, quantised z_min) and Gaussian ids as
// values when the tile ids fit in 20 bits (*dbits = depth-key bits), otherwise the 64-bit
// lists of launch_bin_sort with exact z_min keys and emission indices (*dbits = 0).
int query_key_bits(int64_t n_tiles);
hipError_t launch_query_bin_sort(int64_t n, const sof_camera* d_cams, int n_cams, int64_t n_tiles, int tile,
                                 int64_t cap, const void* proj, void* bins, hipStream_t s, int* parity, int* dbits);
hipError_t launch_cam_table(const sof_camera* d_cams, int n_cams, int tile, CamInfo* out, StatusBlock* status,
                            hipStream_t s);

// Per-pixel order output of sof_render_order (all null: off).
struct OrderDump {
  const int32_t* slot;      // [P] output slot of each pixel; outside [0, n_slots): none
  int64_t n_slots;
  int32_t max_entries;      // M: entries kept per slot and list
  int32_t* stream_ids;      // [n_slots, M] candidates in the order the window received them
  float* stream_keys;       // [n_slots, M] their keys (view z of the peak)
  int32_t* emit_ids;        // [n_slots, M] entries in the order they left the window
  int32_t* counts;          // [n_slots, 2] candidates fed, entries out (may exceed M)
};

struct RenderFwdArgs {
  int64_t n;
  const sof_camera* cams;
  const CamInfo* cam_info;
  int n_cams;
  float near_plane;
  float bg[3];
  uint32_t flags;
  const float4* geom;
  const float4* app;
  const short4* rect;
  const int2* ranges;
  const uint32_t* vals;     // sorted instance -> emission index
  const int32_t* gid;       // emission index -> Gaussian
  float* rgb;
  float* acc;
  float* depth;
  float* normal;
  float* aux;
  float* losses;            // [6, P]: the loss outputs (null: off)
  OrderDump dump;
  // Recorded blend order (null: not recorded).  The forward writes, for each pixel, the tile
  // list position of every Gaussian it blends, in blend order, and one flag per tile; the
  // backward then reads the order instead of replaying the candidate test and the window.
  uint16_t* order;          // [tile][wave][slot][lane] (order_slots slots per pixel)
  int32_t* order_flags;     // [tile] 1: not recorded (a pixel blends more than order_slots
                            // Gaussians, or the tile list is longer than 2^16): replay it
  int32_t order_slots;
};

struct RenderBwdArgs {
  RenderFwdArgs f;
  const float4* bwdr;
  const float* out_rgb;
  const float* out_normal;
  const float* d_rgb;
  const float* d_acc;
  const float* d_depth;
  const float* d_normal;
  float* grads;             // [cap, 16] per emission index
  // opacity at the rendered depth (all null when it has no upstream gradient)
  const float* out_depth;
  const float* opa;
  const float* d_opa;
  // distortion and extent losses: the forward's [4, P] output and upstream [2, P] (null: off)
  const float* losses;
  const float* d_losses;
};

struct RenderOpaArgs {
  RenderFwdArgs f;          // f.depth and f.aux are the forward's outputs (read)
  const float* tail;        // the forward's loss outputs (opacity tail, position of k), or null
  float* opa;
};

hipError_t launch_render_fwd(const RenderFwdArgs& a, int tile, int window, int64_t n_tiles, hipStream_t s);
hipError_t launch_render_bwd(const RenderBwdArgs& a, int tile, int window, int64_t n_tiles, hipStream_t s);
hipError_t launch_render_opa(const RenderOpaArgs& a, int tile, int window, int64_t n_tiles, hipStream_t s);
bool render_supported(int tile, int window);

struct ProjectBwdArgs {
  const float* means;
  const float* scales;
  const float* quats;
  const float* opac;
  const float* sh;
  int sh_degree;
  int64_t n;
  const sof_camera* cams;
  int n_cams;
  const int32_t* counts;
  const int64_t* offsets;
  const int64_t* count_total;
  int64_t cap;
  float* grads;             // per-instance partials; reduced in place per (camera, Gaussian)
  float* d_means;
  float* d_scales;
  float* d_quats;
  float* d_opac;
  float* d_sh;
};
hipError_t launch_project_bwd(const ProjectBwdArgs& a, hipStream_t s);

hipError_t launch_filter3d(const float* means, const float* scales, const float* opac, int64_t n,
                           const sof_camera* cams, int n_cams, float near_plane, float k, float* var,
                           float* scales_out, float* opac_out, hipStream_t s);
hipError_t launch_filter3d_bwd(const float* scales, const float* opac, const float* var, int64_t n,
                               const float* d_scales_out, const float* d_opac_out, float* d_scales, float* d_opac,
                               hipStream_t s);

// Optional timing events recorded around single kernels (see sof_set_timing_events).
enum TimedKernel { kTimeRenderFwd = 0, kTimeRenderBwd = 1, kTimeQuery = 2, kTimedKernels = 3 };
void timing_mark(TimedKernel k, int end, hipStream_t s);

}  // namespace sof
