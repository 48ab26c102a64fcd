/*
 * sof.h -- C ABI of the MI355X (gfx950) Sorted Opacity Fields hot path.
 *
 * The library computes, for 3D Gaussians (mean mu, scale s, rotation quaternion q,
 * opacity o, spherical-harmonic colour f; Sec. 3.1 of the SOF paper):
 *
 *   sof_project        per (camera, Gaussian) preprocessing: culling, the per-ray
 *                      quadric constants of the ray-Gaussian evaluation (Sec. 3.1,
 *                      Eq. (7)-(10); App. A.1), the opacity-aware bound E = sqrt(2 ln 255 o)
 *                      (Eq. (3)), SH colour, normal, screen rectangle, depth keys.
 *   sof_bin_sort       duplication of every Gaussian into the screen tiles it touches and
 *                      the per-tile key sort (level 0 of the hierarchical resort; Sec. 3.1).
 *   sof_render_fwd     per-pixel hierarchical resort by the ray depth of maximum response
 *                      (Eq. (2)/(9)) with a bounded window, front-to-back alpha blending
 *                      (Eq. (1)) of colour, normal and opacity, and the exact 0.5-level-set
 *                      depth (Sec. 3.2 "Exact Depth", App. A.3).
 *   sof_render_opacity opacity field at each pixel's rendered depth (Sec. 3.3, the L_opa term).
 *   sof_render_bwd     adjoint of render + project: walks each pixel's order front to back
 *                      (recorded by the forward, or replayed), recomputing transmittance, and
 *                      writes gradients for mu, s, q, o, f.
 *   sof_filter3d       the 3D filter's opacity and covariance adjustment (App. "Dead Gaussians").
 *   sof_opacity_query  opacity field O(x) = min over views of O_N(x) (Eq. (12)-(13)) at
 *                      arbitrary points, with tile scheduling of points (Sec. 3.4, Eq. (14))
 *                      and z_min early stopping (Eq. (15)); all views in one persistent launch.
 *
 * Conventions shared by every entry point
 *   - All array arguments are DEVICE pointers unless named h_*, row-major, contiguous,
 *     float32 unless stated.  The caller owns every buffer; the library never allocates,
 *     frees or synchronises.  Work is enqueued on `stream` in order; no entry point reads
 *     a device value back to the host, so a sequence of calls can be captured in a graph.
 *   - Cameras are passed twice: h_cams (host copy, used for launch sizes) and d_cams
 *     (identical device copy, read by kernels).  World -> camera is x_c = R x + t with
 *     OpenCV axes (x right, y down, z forward); pixel (px, py) has its centre at
 *     (px + 1/2, py + 1/2); intrinsics fx, fy, cx, cy in pixels.
 *   - Images of several cameras are concatenated in camera order.  Per camera, a C-channel
 *     image is planar [C, H, W]; camera c's block starts at C * sum_{c'<c} W_c' H_c'.
 *   - Return value: SOF_OK (0) or a negative sof_status.  Argument checks happen before
 *     anything is enqueued.  A device-side condition (instance capacity exceeded) cannot be
 *     returned from an asynchronous call; it is recorded in the status word inside the
 *     `bins` buffer (see sof_read_status_offset) and the affected work is clipped so that
 *     nothing is written out of bounds.
 *   - State and thread safety: the library keeps nothing between calls except two
 *     process-wide items, the timing-event table of sof_set_timing_events (instrumentation,
 *     not thread-safe) and the per-device static scratch of sof_render_bwd_static (calls of
 *     it that overlap on one device race).  Every other call works only on the caller's
 *     buffers: calls on different streams with different buffers may run concurrently.
 */
#ifndef SOF_H
#define SOF_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sof_status {
  SOF_OK = 0,
  SOF_E_ARG = -1,          /* null pointer, negative size, sh_degree > 3, bad tile/window   */
  SOF_E_WORKSPACE = -2,    /* a workspace buffer is smaller than sof_workspace_size asks   */
  SOF_E_CAPACITY = -3,     /* (device status bit) more tile instances than `capacity`       */
  SOF_E_HIP = -4,          /* a HIP launch failed (hipGetLastError after enqueue)          */
  SOF_E_UNSUPPORTED = -5,  /* window or tile size without a compiled kernel               */
  SOF_E_SCRATCH = -6       /* sof_render_bwd_static: capacity above its fixed scratch       */
} sof_status;

/* Option flags */
enum {
  SOF_DEPTH_MEDIAN = 1u << 0,    /* depth output = t*_k of the crossing Gaussian (GOF median
                                    depth) instead of the exact 0.5-level-set depth           */
  SOF_DEPTH_GRAD_FULL = 1u << 1, /* render_bwd: differentiate the exact-depth correction
                                    (App. A.3) too; default treats it as a constant, as the
                                    paper does, so d depth = d t*_k                           */
  SOF_QUERY_KEYS = 1u << 2,      /* set internally by sof_opacity_query: tile lists sorted by
                                    z_min (Eq. (15)) instead of the mean's view depth          */
  SOF_QUERY_LEVELSET = 1u << 3,  /* sof_opacity_query: only O(x) > 0.5 or not is needed
                                    (Sec. 3.4): stop a view once its O_N exceeds 0.5 and skip
                                    a point once some view gave O_N <= 0.5                    */
  SOF_QUERY_REUSE = 1u << 4      /* sof_opacity_query: proj and bins still hold the Gaussian
                                    side (projection, per-tile lists) of the previous call with
                                    the same Gaussians, cameras, tile and capacity; only the
                                    points are processed (the binary search's later steps)    */
};

/* Gaussians, Sec. 3.1: n primitives, activated parameters. */
typedef struct sof_gaussians {
  int64_t n;                 /* number of Gaussians, 0 <= n < 2^31                            */
  int32_t sh_degree;         /* 0..3; K = (sh_degree + 1)^2 coefficients per channel          */
  int32_t reserved;
  const float* means;        /* [n,3] world-space centres                                      */
  const float* scales;       /* [n,3] standard deviations along the rotated axes (> 0)         */
  const float* quats;        /* [n,4] rotation quaternion (w,x,y,z); normalised internally     */
  const float* opacities;    /* [n]   in [0,1]                                                  */
  const float* sh;           /* [n,K,3] real SH coefficients, coefficient l^2 + l + m          */
} sof_gaussians;

/* Pinhole camera (72 bytes). */
typedef struct sof_camera {
  float R[9];                /* world -> camera rotation, row-major                            */
  float t[3];                /* world -> camera translation                                    */
  float fx, fy, cx, cy;      /* intrinsics in pixels                                           */
  int32_t width, height;     /* image size in pixels (>= 1)                                    */
} sof_camera;

typedef struct sof_options {
  int32_t tile;              /* screen tile side: 8, 16 or 32                                  */
  int32_t window;            /* per-pixel resort window W: 0 (no resort), 1, 2, 4, 8, 16, 32 */
  float near_plane;          /* tau_n; the paper's near plane is 0.2                           */
  float bg[3];               /* background colour added with weight T_end (default 0)          */
  uint32_t flags;            /* SOF_* flags                                                    */
  int32_t order_slots;       /* 0..4096: Gaussians per pixel the recorded blend order holds
                                (the `order` buffer of sof_render_fwd / sof_render_bwd); 0:
                                no recorded order                                             */
  int64_t capacity;          /* maximum number of tile instances (all cameras), < 2^31         */
} sof_options;

/*
 * Sizes of the caller-owned device buffers for a render of n Gaussians over the given
 * cameras:
 *   proj   per (camera, Gaussian) records written by sof_project          ~ 160 B x cams x n
 *   bins   tile instances, sort buffers, tile ranges, status word          ~ 24 B x capacity
 *   grads  per-instance gradient partials used only by sof_render_bwd      64 B x capacity
 *   order  the recorded blend order (optional; 0 when opts->order_slots is 0): written by
 *          sof_render_fwd, read by sof_render_bwd    2 B x order_slots x pixels (tile-padded)
 * Any output pointer may be NULL.  Returns SOF_E_ARG on invalid arguments.
 */
int sof_workspace_size(int64_t n, const sof_camera* h_cams, int32_t n_cams, const sof_options* opts,
                       size_t* proj_bytes, size_t* bins_bytes, size_t* grad_bytes, size_t* order_bytes);

/* Byte offset, inside `bins`, of the device status block:
 *   int64 [0] instance count K requested by the last sof_bin_sort (may exceed capacity)
 *   int32 [2] status bits: 1 = capacity exceeded (K > capacity; lists were clipped)       */
size_t sof_read_status_offset(void);

/*
 * sof_project -- Sec. 3.1 (Eq. (3), (7)-(10)), App. A.1.
 * For every camera c and Gaussian i writes into `proj` the record the rasteriser needs:
 * liveness (o >= 1/255 and view z of the mean > near_plane; a Gaussian with a non-finite
 * mean, scale, quaternion, opacity or colour, a scale <= 0 or a zero quaternion is culled
 * as well, so it touches no tile and contributes nothing), the quadric constants of the
 * pixel-ray evaluation (computed in float64, stored in float32 in a cancellation-free form
 * relative to the projected centre), opacity, colour max(0, SH(dir) + 1/2) with dir from
 * the camera centre to the mean, the normal (shortest axis, facing the camera), the
 * inclusive pixel rectangle covering the E-ellipsoid and the depth keys.  Overwrites proj.
 */
int sof_project(const sof_gaussians* g, const sof_camera* h_cams, const sof_camera* d_cams,
                int32_t n_cams, const sof_options* opts, void* proj, size_t proj_bytes,
                hipStream_t stream);

/*
 * sof_bin_sort -- the per-tile key sort (level 0 of the hierarchical resort, Sec. 3.1).
 * Emits one instance per (camera, Gaussian, touched tile), sorts instances by
 * (global tile, float32 view depth of the mean, Gaussian index) with a stable LSD radix
 * sort and writes per-tile [start, end) ranges.  With SOF_QUERY_KEYS the depth key is
 * z_min = mu_z - E sqrt(Sigma_zz) instead (Eq. (15)).  Reads proj, overwrites bins.
 * Instances beyond opts->capacity are dropped and status bit 1 is set.
 */
int sof_bin_sort(int64_t n, const sof_camera* h_cams, const sof_camera* d_cams, int32_t n_cams,
                 const sof_options* opts, const void* proj, size_t proj_bytes, void* bins,
                 size_t bins_bytes, hipStream_t stream);

/*
 * sof_render_fwd -- Eq. (1), (2), Sec. 3.2.
 * For every pixel: walks its tile's list, keeps Gaussians with alpha = min(0.99, o G*) >=
 * 1/255 whose peak lies beyond the near plane, re-sorts them by the ray distance t* of
 * maximum response with a window of opts->window entries, and blends front to back,
 * stopping before a Gaussian that would drop T below 1e-4.  Outputs (any may be NULL):
 *   rgb    [3,H,W] per camera   sum w c + bg T_end
 *   acc    [H,W]                1 - T_end
 *   depth  [H,W]                exact depth t_k - sqrt(2 ln(G*_k / g) / A_k) on the ray,
 *                               g = (T_k - 1/2) / (T_k o_k), k = first Gaussian with
 *                               T_k > 1/2 >= T_k (1 - alpha_k); 0 without a crossing
 *                               (t*_k with SOF_DEPTH_MEDIAN)
 *   normal [3,H,W]              sum w n (not normalised)
 *   aux    [6,H,W] float32 bits T_end, n_emitted (int32), k (int32 Gaussian index or -1),
 *                               T_k -- needed by sof_render_bwd -- then two int32 work
 *                               counters: list entries tested and candidates found.
 *   losses [6,H,W]              the per-pixel distortion and extent losses of Sec. 3.3
 *                               (App. C.1, C.2), then two moments sof_render_bwd needs, then
 *                               two channels sof_render_opacity reads (below).  With
 *                               d = NDC(t*) = f (t* - n) / ((f - n) t*), n = 0.2, f = 100,
 *                               over the blended Gaussians: distortion = sum_ij w_i w_j
 *                               (d_i - d_j)^2 = 2 A M with A = sum w, mean mu = sum w d / A
 *                               and M = sum w (d - mu)^2 (channels 2, 3, accumulated one
 *                               Gaussian at a time); extent = f n / (f - n) sum w 2 A_i
 *                               sqrt(B_i^2 - 4 A_i (C_i - E_i^2)) / B_i^2.  Channel 4 is
 *                               prod_{i >= k} (1 - alpha_i(x)) over the blended Gaussians from
 *                               the crossing Gaussian k on, each at x = o + t_r d (t_r the depth
 *                               output; alpha as in sof_render_opacity), channel 5 the position
 *                               of k in the blend order (int32, -1 without a crossing).  NULL:
 *                               not computed (a kernel without this work runs).
 *   order  (optional, with aux; order_bytes from sof_workspace_size, opts->order_slots > 0)
 *          the blend order of every pixel, for sof_render_bwd: per tile an int32 flag, then
 *          per tile and 64-pixel wave (8x8 sub-tile) order_slots rows of 64 uint16 tile-list
 *          positions, row e holding each pixel's e-th blended Gaussian.  A tile whose list is
 *          longer than 2^16 or with a pixel that blends more than order_slots Gaussians is
 *          flagged and its order is not used (the backward replays it).  Contents beyond
 *          that are unspecified.  NULL: not recorded.
 */
int sof_render_fwd(int64_t n, const sof_camera* h_cams, const sof_camera* d_cams, int32_t n_cams,
                   const sof_options* opts, const void* proj, size_t proj_bytes, const void* bins,
                   size_t bins_bytes, float* rgb, float* acc, float* depth, float* normal, float* aux,
                   float* losses, void* order, size_t order_bytes, hipStream_t stream);

/*
 * sof_render_order -- the per-pixel order of Sec. 3.1 (level-0 tile list, then the per-pixel
 * resort window), as a debug output for checking it entry by entry.
 * Runs the forward rasteriser with the same n, cameras, options, proj and bins as
 * sof_render_fwd (its decisions are those of sof_render_fwd: the same kernel code with stores
 * added) and writes no image.  slot [sum of W H] int32 (device) names, for each pixel, a row
 * of the output arrays; pixels whose slot lies outside [0, n_slots) are not written.  Each
 * row holds up to max_entries (M) entries:
 *   stream_ids  [n_slots, M] int32  Gaussian index of each candidate (alpha >= 1/255, peak
 *                                   beyond the near plane) in the order the window received
 *                                   them, up to where the pixel stopped
 *   stream_keys [n_slots, M] float  its key: the view z of the peak (the ray distance t* is
 *                                   the key times |(x_n, y_n, 1)|, so both order alike)
 *   emit_ids    [n_slots, M] int32  Gaussian index of each entry in the order it left the
 *                                   window; the first n_emitted were blended, one more means
 *                                   that entry stopped the pixel (T would drop below 1e-4)
 *   counts      [n_slots, 2] int32  number of candidates fed and of entries out (may exceed
 *                                   M; only the first M of each list are written)
 * Two pixels must not share a slot.  Caller-owned device buffers; entries beyond the counts
 * are left as they were.  SOF_E_ARG for a null slot or counts, or null lists with
 * max_entries > 0.
 */
int sof_render_order(int64_t n, const sof_camera* h_cams, const sof_camera* d_cams, int32_t n_cams,
                     const sof_options* opts, const void* proj, size_t proj_bytes, const void* bins,
                     size_t bins_bytes, const int32_t* slot, int64_t n_slots, int32_t max_entries,
                     int32_t* stream_ids, float* stream_keys, int32_t* emit_ids, int32_t* counts,
                     hipStream_t stream);

/*
 * sof_render_opacity -- Sec. 3.3 (direct opacity-field supervision).
 * A second pass after sof_render_fwd (same n, cameras, options, proj and bins; its depth
 * and aux outputs as inputs): for each pixel with a 0.5 crossing, opacity = O_N(x) at
 * x = o + t_r d, t_r the depth the forward wrote, over the Gaussians the pixel blended, each
 * with alpha = min(0.99, o_i G_i(min(t*_i, t_r))) and counted when alpha >= 1/255 and the
 * evaluated point lies beyond the near plane (Eq. (12)); 0 where there is no crossing.
 * The pass walks the forward's per-pixel order: read from `order` (NULL, or the forward's
 * recorded order with the same opts->order_slots; the tiles it flagged are replayed) or
 * replayed.  With `losses` (the forward's [6,H,W] losses output, or NULL) it uses the paper's
 * split O_N = O_k + T_k sum_{i >= k} alpha_i prod_{k <= j < i} (1 - alpha_j): the forward
 * accumulated the part from the crossing Gaussian k on, and the walk stops in front of k; with
 * NULL it walks every blended Gaussian.  All give O_N up to float rounding.  Overwrites
 * opacity [sum of W H].  The L_opa loss |O_N - 0.5|^2 is the caller's to form.
 */
int sof_render_opacity(int64_t n, const sof_camera* h_cams, const sof_camera* d_cams, int32_t n_cams,
                       const sof_options* opts, const void* proj, size_t proj_bytes, const void* bins,
                       size_t bins_bytes, const float* depth, const float* aux, const float* losses,
                       const void* order, size_t order_bytes, float* opacity, hipStream_t stream);

/*
 * sof_render_bwd -- adjoint of sof_render_fwd, sof_render_opacity and sof_project.
 * Inputs: the same g, cameras, options, proj and bins as the forward call, its rgb,
 * normal and aux outputs, and upstream gradients d_rgb, d_acc, d_depth, d_normal (NULL =
 * zero; d_normal requires normal, else SOF_E_ARG).  d_opacity (NULL = zero) is the upstream gradient of sof_render_opacity's output;
 * with it, depth and opacity must be the forward's depth and that output.  The depth t_r
 * at which the opacity is evaluated is held constant (like the exact-depth correction).
 * d_losses [2,H,W] (NULL = zero) is the upstream gradient of the forward's distortion and
 * extent losses; with it, losses is the forward's [4,H,W] losses output.  Their gradients
 * follow App. C.1 (dL/dalpha front to back from the stored totals) and C.2.
 * Each pixel's forward order is walked front to back; suffix sums come from the stored
 * totals.  `order` (NULL or the forward's recorded order, with the same opts->order_slots)
 * gives that order directly; without it, and for the tiles the forward flagged, the order is
 * replayed (the same candidate test and window as the forward).  Writes (overwrites) d_means [n,3], d_scales [n,3], d_quats [n,4], d_opacities
 * [n], d_sh [n,K,3].  `grads` is scratch.  Reproducible to float rounding, not bitwise: a
 * tile's pixels add into each instance's partials with LDS float atomics, whose order follows
 * the scheduling of the tile's waves; the per-instance partials of a Gaussian are then summed
 * in a fixed order.
 */
int sof_render_bwd(const sof_gaussians* g, const sof_camera* h_cams, const sof_camera* d_cams,
                   int32_t n_cams, const sof_options* opts, const void* proj, size_t proj_bytes,
                   const void* bins, size_t bins_bytes, const float* rgb, const float* normal,
                   const float* aux, const void* order, size_t order_bytes, const float* d_rgb,
                   const float* d_acc, const float* d_depth, const float* d_normal, const float* depth,
                   const float* opacity, const float* d_opacity, const float* losses,
                   const float* d_losses, void* grads,
                   size_t grad_bytes, float* d_means, float* d_scales, float* d_quats,
                   float* d_opacities, float* d_sh, hipStream_t stream);

/*
 * sof_render_bwd_static -- sof_render_bwd without the `grads` workspace, for callers that
 * cannot allocate device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  It allocates nothing: the per-instance gradient partials live in a
 * static device array inside the library, 64 MiB per device (opts->capacity up to 2^20 tile
 * instances; larger capacities return SOF_E_SCRATCH before anything is enqueued), held by
 * every device the library runs on until the process ends.  The array's device address is
 * looked up on the first call on each device (that device must be current).  Every other
 * argument, and the results, are those of sof_render_bwd.  All calls on one device share its
 * array: calls that overlap in time on one device (other streams, other threads) race and
 * must be serialised by the caller.  Nothing in the array needs clearing between calls (each
 * call writes every partial it reads).
 */
int sof_render_bwd_static(const sof_gaussians* g, const sof_camera* h_cams, const sof_camera* d_cams,
                          int32_t n_cams, const sof_options* opts, const void* proj, size_t proj_bytes,
                          const void* bins, size_t bins_bytes, const float* rgb, const float* normal,
                          const float* aux, const void* order, size_t order_bytes, const float* d_rgb,
                          const float* d_acc, const float* d_depth, const float* d_normal,
                          const float* depth, const float* opacity, const float* d_opacity,
                          const float* losses, const float* d_losses,
                          float* d_means, float* d_scales, float* d_quats, float* d_opacities, float* d_sh,
                          hipStream_t stream);

/*
 * Workspace for sof_opacity_query: like sof_workspace_size with the per-view tile lists
 * sorted by z_min plus the (view, point) schedule.  `pv_capacity` bounds the number of
 * (point, view) pairs that project inside a view (<= n_points * n_cams).
 */
int sof_query_workspace_size(int64_t n, const sof_camera* h_cams, int32_t n_cams,
                             const sof_options* opts, int64_t n_points, int64_t pv_capacity,
                             size_t* proj_bytes, size_t* bins_bytes, size_t* sched_bytes);

/*
 * sof_opacity_query -- Eq. (12)-(13), App. A.2, Sec. 3.4.
 * opacity[p] = min over cameras v that see points[p] (view z > near_plane and projection
 * inside the image) of O_N = 1 - prod_i (1 - alpha_i), alpha_i = min(0.99, o_i G_i(t_eval)),
 * t_eval = min(t*_i, |x - c_v|), counting Gaussians with alpha_i >= 1/255 whose evaluated
 * point lies beyond the near plane; 1 where no camera sees the point.  Points are scheduled
 * per (view, tile) in blocks of 256 sorted by depth (Eq. (14)); each tile's Gaussians are
 * sorted by a monotone key of z_min (32-bit keys quantise it to 1/128 octave when the tile
 * ids fit in 20 bits, 64-bit keys keep it exact otherwise) and the walk stops once the key
 * passes the point's own (Eq. (15); inside the point's bucket the exact z_min decides) or
 * once the partial O_N already reaches the point's running minimum.  With
 * SOF_QUERY_LEVELSET in opts->flags the result is exact only up to the classification the
 * binary search needs: opacity[p] <= 0.5 exactly when O(x) <= 0.5, and then it is the O_N of
 * one view, in [O(x), 0.5] (a view whose work starts after another view of the point has
 * reported O_N <= 0.5 is skipped, so which view depends on scheduling); otherwise it is a value
 * in (0.5, O(x)].  All (view, tile, block) work items run in one persistent launch.
 * Overwrites opacity [n_points].
 */
int sof_opacity_query(const sof_gaussians* g, const sof_camera* h_cams, const sof_camera* d_cams,
                      int32_t n_cams, const sof_options* opts, const float* points, int64_t n_points,
                      int64_t pv_capacity, float* opacity, void* proj, size_t proj_bytes, void* bins,
                      size_t bins_bytes, void* sched, size_t sched_bytes, hipStream_t stream);

/*
 * sof_filter3d -- the 3D filter of App. "Dead Gaussians": Sigma + s I for a per-Gaussian
 * filter size s, and o_hat = o sqrt(|Sigma| / |Sigma + s I|).  s follows the filter the paper
 * adopts: s = (k z / f_x)^2 for the camera with the largest f_x / z whose image contains the
 * projected centre beyond near_plane (k = 0.2 there), s = 0 when no camera does.  Writes
 * var [n] = s, scales_out [n,3] = sqrt(scales^2 + s) (the rotation is unchanged) and
 * opacities_out [n] = o prod_j scales_j / scales_out_j.  Only means, scales and opacities
 * of g are read.  n_cams may be 0 (no filtering).
 */
int sof_filter3d(const sof_gaussians* g, const sof_camera* h_cams, const sof_camera* d_cams, int32_t n_cams,
                 float near_plane, float k, float* var, float* scales_out, float* opacities_out,
                 hipStream_t stream);

/*
 * sof_filter3d_bwd -- adjoint of sof_filter3d with var held constant: from the upstream
 * gradients of scales_out and opacities_out (NULL = zero) writes (overwrites) d_scales [n,3]
 * and d_opacities [n] with respect to the unfiltered scales and opacities.
 */
int sof_filter3d_bwd(const sof_gaussians* g, const float* var, const float* d_scales_out,
                     const float* d_opacities_out, float* d_scales, float* d_opacities,
                     hipStream_t stream);

/*
 * Instrumentation, not part of the method: per-kernel timing for benchmarks.  `events`
 * points to 6 hipEvent_t handles created by the caller (or is NULL to switch timing off);
 * while set, every later call records, on its own stream, events[0]/[1] immediately before
 * and after the sof_render_fwd kernel, events[2]/[3] around the rasteriser adjoint kernel
 * of sof_render_bwd (the per-Gaussian reduction that follows it is excluded) and
 * events[4]/[5] around the evaluation kernel of sof_opacity_query.  A NULL handle skips
 * that record.  The handles are borrowed, not owned; the setting is process-wide and not
 * thread-safe.  Always returns SOF_OK.
 */
int sof_set_timing_events(void* const* events);

/*
 * Instrumentation, not part of the method: machine-peak probes for benchmarks.
 *   sof_bench_copy  copies n_vec4 16-byte elements from src to dst (device, non-overlapping)
 *                   with a grid-stride streaming kernel: reachable HBM bandwidth.
 *   sof_bench_fma   runs n_blocks workgroups of 256 lanes, each lane 16 independent chains of
 *                   `iters` float32 fused multiply-adds (2 x 16 x iters flops per lane), and
 *                   writes one float per lane to out [n_blocks * 256]: reachable vector rate.
 * Both return SOF_E_ARG for negative sizes or null buffers.
 */
int sof_bench_copy(const void* src, void* dst, int64_t n_vec4, hipStream_t stream);
int sof_bench_fma(float* out, int64_t n_blocks, int32_t iters, hipStream_t stream);

/*
 * sof_bisect_step -- one step of the binary search towards the 0.5 level set of the opacity
 * field (Sec. 3.4: eight steps on the edges of the tetrahedral grid).  a, b and mid are
 * device [n_edges, 3] float32 arrays: a[i] an endpoint inside (O > 0.5), b[i] one outside.
 * With opacity == NULL the call only writes mid = (a + b) / 2.  Otherwise opacity[i] is the
 * opacity at mid[i] (e.g. from sof_opacity_query with SOF_QUERY_LEVELSET): mid replaces a
 * when opacity > 0.5 and b otherwise, then mid is set to the new (a + b) / 2.  Arrays are
 * caller-owned and updated in place; after k steps mid is the centre of a bracket 2^-k the
 * initial length.  Returns SOF_E_ARG for null arrays (with n_edges > 0) or n_edges < 0.
 */
int sof_bisect_step(float* a, float* b, float* mid, const float* opacity, int64_t n_edges, hipStream_t stream);

/* Human-readable text for a sof_status value (static storage). */
const char* sof_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* SOF_H */
