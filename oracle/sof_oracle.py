"""Plain, slow FP64 CPU oracle for the Sorted Opacity Fields (SOF) hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only tests, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code, constants generator or helper with
the HIP library.

Everything here works on float64 copies of the float32 inputs and evaluates
every pixel by brute force over *all* Gaussians (no tiles), following the
paper's definitions:

* scene representation and alpha blending          -- Sec. 3.1, Eq. (1)
* ray depth of maximum response                     -- Sec. 3.1, Eq. (2), Eq. (9)
* opacity-aware cutoff E_i = sqrt(2 ln(255 o_i))    -- Sec. 3.1, Eq. (3)
* 1D Gaussian along a ray, A/B/C, peak value        -- Sec. 3.1, Eq. (7)-(10)
* opacity field O_N and its minimum over views      -- Sec. 3.1, Eq. (12)-(13)
* order independence of O_N                         -- App. A.2 (Proposition)
* exact 0.5-level-set depth                         -- Sec. 3.2 "Exact Depth", App. A.3
* hierarchical per-pixel resorting                   -- Sec. 3.1 "StopThePop" (the paper
  cites StopThePop for it and does not restate it; the two-level reading used here is
  documented at `hierarchical_order`)
* opacity-sorted early stop for queries (z_min)     -- Sec. 3.4 "Early Stopping", Eq. (15)
* level-set classification and binary search         -- Sec. 3.4 (8 binary-search steps
  towards the 0.5 level set; only O > 0.5 or not matters there)
* opacity field at the rendered depth (L_opa)         -- Sec. 3.3 "Direct Opacity Field
  Supervision"
* distortion and extent losses                       -- Sec. 3.3 "Distortion Loss", "Extent
  Loss"; App. C.1, C.2
* 3D filter: opacity and covariance adjustment       -- App. "Dead Gaussians" (o_hat =
  o sqrt(|Sigma| / |Sigma + s I|))

Readings of passages the paper leaves open (all listed in the design notes):
  R1  A, B, C are written with Sigma^{-1} directly (A = d^T S^-1 d, B = 2 d^T S^-1 (o-mu),
      C = (o-mu)^T S^-1 (o-mu)); the Gaussian-space transform of Sec. 3.1 is the same thing.
  R2  rays use unit directions, so every depth is a Euclidean ray distance.
  R3  3DGS blending conventions: alpha = min(0.99, o G); a Gaussian with alpha < 1/255 is
      skipped; blending stops before the Gaussian that would push T below 1e-4.
  R4  exact depth: T_k (1 - o_k G(t)) = 0.5 is solved with the *unclamped* o_k, i.e.
      G(t) = (T_k - 0.5) / (T_k o_k).  (App. A.3 drops T_k when isolating G; keeping it is
      what makes the result the 0.5 level set claimed in Sec. 3.2.)
  R5  the crossing Gaussian k is the first with T_k > 0.5 >= T_k (1 - alpha_k); with no
      crossing the depth output is 0.
  R6  near plane tau_n = 0.2 (the NDC near plane of Sec. 3.3): a Gaussian whose mean has
      view z <= tau_n is culled for that camera; a contribution counts only if the view z
      of the evaluated point is > tau_n.
  R7  level-0 stream order is the per-tile key sort of 3DGS: view-space z of the mean,
      stored as a float32, ties broken by Gaussian index.
  R8  Gaussian normal: the rotation column of the smallest scale (lowest index on ties),
      flipped to face the camera (the paper defers to GOF; parity unpinned vs. GOF).
  R9  colour: real spherical harmonics (Condon-Shortley phase), + 0.5, clamped at 0,
      evaluated at the unit direction from the camera centre to the mean.
  R10 an unobserved query point (no valid view) has opacity 1 (identity of min on [0,1]).
  R16 binary search: a point is inside when O(x) > 0.5; an edge joins an inside endpoint a
      and an outside endpoint b; each step evaluates the midpoint and replaces the endpoint
      of the same class; the result after the last step is the midpoint of the final
      bracket (the paper gives the step count, 8, not the final pick).
  R17 opacity at the rendered depth: x = o + t_r d with t_r the exact depth of the pixel;
      O_N(x) over the Gaussians the pixel blends (the paper's first pass accumulates over
      them), each with alpha at t_eval = min(t*_j, t_r) as in Eq. (12); undefined without a
      crossing.  Gradients treat t_r as a constant (as the exact-depth correction).
  R18 distortion and extent losses: NDC(t) = f (t - n) / ((f - n) t) with n = 0.2, f = 100 on
      the ray distance (its derivative is the f n / ((f - n) t^2) of App. C.2); the depth of a
      Gaussian is its t*; sums run over the Gaussians the pixel blends with w = alpha T.
  R19 3D filter size (the paper takes it from Mip-Splatting): s_i = (k z_i / f)^2 for the
      camera that samples the centre most finely (largest f / z among cameras whose image
      contains the projected centre beyond the near plane), k = 0.2; no camera: s_i = 0.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.special import lpmv

NEAR = 0.2            # R6
ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99      # R3
T_MIN = 1e-4          # R3


# ----------------------------------------------------------------------------------------
# Scene representation (Sec. 3.1: mu, s, R, o, f in R^48; Sigma = R S S^T R^T)
# ----------------------------------------------------------------------------------------

def _hamilton(p, q):
    """Hamilton product of quaternions stored (w, x, y, z)."""
    pw, px, py, pz = p
    qw, qx, qy, qz = q
    return np.array([
        pw * qw - px * qx - py * qy - pz * qz,
        pw * qx + px * qw + py * qz - pz * qy,
        pw * qy - px * qz + py * qw + pz * qx,
        pw * qz + px * qy - py * qx + pz * qw,
    ])


def quat_to_rot(quat):
    """Rotation matrix of the normalised quaternion (w, x, y, z).

    Built from its definition v -> q v q*: column j is the image of the j-th unit vector.
    """
    q = np.asarray(quat, np.float64)
    q = q / np.linalg.norm(q)
    qc = q * np.array([1.0, -1.0, -1.0, -1.0])
    R = np.zeros((3, 3))
    for j in range(3):
        e = np.zeros(4)
        e[1 + j] = 1.0
        R[:, j] = _hamilton(_hamilton(q, e), qc)[1:]
    return R


@dataclass
class Scene:
    """float64 copies of the float32 inputs (the arrays both sides receive)."""
    means: np.ndarray      # [N,3]
    scales: np.ndarray     # [N,3] activated (> 0)
    quats: np.ndarray      # [N,4] (w,x,y,z), raw
    opac: np.ndarray       # [N]   activated, in [0,1]
    sh: np.ndarray         # [N,(d+1)^2,3]
    sh_degree: int

    @staticmethod
    def from_arrays(means, scales, quats, opac, sh, sh_degree):
        f = lambda a: np.array(a, dtype=np.float64)
        return Scene(f(means), f(scales), f(quats), f(opac).reshape(-1), f(sh), int(sh_degree))

    @property
    def n(self):
        return self.means.shape[0]

    def rotations(self):
        return np.stack([quat_to_rot(q) for q in self.quats]) if self.n else np.zeros((0, 3, 3))

    def covariances(self):
        R = self.rotations()
        return np.einsum("nij,nj,nkj->nik", R, self.scales ** 2, R)

    def precisions(self):
        R = self.rotations()
        return np.einsum("nij,nj,nkj->nik", R, self.scales ** -2.0, R)


@dataclass
class Camera:
    """Pinhole camera, world -> camera x_c = R x + t, OpenCV axes; pixel centres at +1/2."""
    R: np.ndarray
    t: np.ndarray
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    @staticmethod
    def from_arrays(R, t, fx, fy, cx, cy, width, height):
        return Camera(np.array(R, np.float64).reshape(3, 3), np.array(t, np.float64).reshape(3),
                      float(fx), float(fy), float(cx), float(cy), int(width), int(height))

    @property
    def center(self):
        return -self.R.T @ self.t

    def pixel_ray(self, px, py):
        """Unit world direction through the centre of pixel (px, py) and its camera-space
        direction with unit z (the z-depth along the ray is t / |d_c|)."""
        dc = np.array([(px + 0.5 - self.cx) / self.fx, (py + 0.5 - self.cy) / self.fy, 1.0])
        d = self.R.T @ dc
        return d / np.linalg.norm(d), dc


def opacity_cutoff(opac):
    """E_i = sqrt(2 ln(255 o_i)), Eq. (3); the Mahalanobis radius where o G = 1/255."""
    return np.sqrt(2.0 * np.log(255.0 * np.asarray(opac, np.float64)))


# ----------------------------------------------------------------------------------------
# Colour and normal (R8, R9)
# ----------------------------------------------------------------------------------------

def sh_basis(degree, dirs):
    """Real orthonormal spherical harmonics up to `degree` at unit `dirs` [M,3].

    Y_l^0 = K_l^0 P_l^0(cos th), Y_l^m = sqrt2 K_l^m cos(m ph) P_l^m, Y_l^-m = sqrt2 K_l^m
    sin(m ph) P_l^m, with K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) and P_l^m the associated
    Legendre functions including the Condon-Shortley phase.  Column l^2 + l + m.
    """
    dirs = np.atleast_2d(np.asarray(dirs, np.float64))
    ct = np.clip(dirs[:, 2], -1.0, 1.0)
    ph = np.arctan2(dirs[:, 1], dirs[:, 0])
    out = np.zeros((dirs.shape[0], (degree + 1) ** 2))
    for l in range(degree + 1):
        for m in range(0, l + 1):
            K = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))
            P = lpmv(m, l, ct)
            if m == 0:
                out[:, l * l + l] = K * P
            else:
                out[:, l * l + l + m] = math.sqrt(2.0) * K * np.cos(m * ph) * P
                out[:, l * l + l - m] = math.sqrt(2.0) * K * np.sin(m * ph) * P
    return out


def gaussian_colors(scene: Scene, cam_center):
    """c = max(0, sum_lm f_lm Y_lm(dir) + 1/2), dir = unit(mu - camera centre)."""
    d = scene.means - np.asarray(cam_center)[None, :]
    d = d / np.linalg.norm(d, axis=1, keepdims=True)
    Y = sh_basis(scene.sh_degree, d)                       # [N,K]
    K = (scene.sh_degree + 1) ** 2
    c = np.einsum("nk,nkc->nc", Y, scene.sh[:, :K, :]) + 0.5
    return np.maximum(c, 0.0)


def gaussian_normals(scene: Scene, cam_center):
    """Shortest-axis rotation column, flipped so that n . (camera - mu) >= 0 (R8)."""
    R = scene.rotations()
    out = np.zeros((scene.n, 3))
    for i in range(scene.n):
        j = int(np.argmin(scene.scales[i]))          # argmin returns the lowest index on ties
        n = R[i][:, j]
        if np.dot(n, np.asarray(cam_center) - scene.means[i]) < 0:
            n = -n
        out[i] = n
    return out


# ----------------------------------------------------------------------------------------
# Per-camera preprocessing (liveness and culling, level-0 keys)
# ----------------------------------------------------------------------------------------

@dataclass
class CameraView:
    """Everything per (camera, Gaussian) that the per-pixel evaluation reuses."""
    cam: Camera
    live: np.ndarray       # bool [N]: o >= 1/255 and mean view z > tau_n
    prec: np.ndarray       # [N,3,3] world-space Sigma^{-1}
    zkey32: np.ndarray     # float32 [N] view z of the mean (R7)
    color: np.ndarray      # [N,3]
    normal: np.ndarray     # [N,3]


def view(scene: Scene, cam: Camera, appearance=True) -> CameraView:
    """Per-camera liveness, precisions and level-0 keys; appearance=False skips the colours and
    normals (the opacity field of Eq. (12) never reads them)."""
    mu_c = scene.means @ cam.R.T + cam.t[None, :]
    live = (scene.opac >= ALPHA_MIN) & (mu_c[:, 2] > NEAR)
    if not appearance:
        return CameraView(cam, live, scene.precisions(), mu_c[:, 2].astype(np.float32), None, None)
    return CameraView(cam, live, scene.precisions(), mu_c[:, 2].astype(np.float32),
                      gaussian_colors(scene, cam.center), gaussian_normals(scene, cam.center))


def views_geometry(scene: Scene, cams):
    """Geometry-only CameraViews of several cameras (what Eq. (12) reads), the world-space
    precisions computed once and shared."""
    prec = scene.precisions()
    out = []
    for cam in cams:
        mu_c = scene.means @ cam.R.T + cam.t[None, :]
        live = (scene.opac >= ALPHA_MIN) & (mu_c[:, 2] > NEAR)
        out.append(CameraView(cam, live, prec, mu_c[:, 2].astype(np.float32), None, None))
    return out


# ----------------------------------------------------------------------------------------
# Per-pixel candidates (Eq. (7)-(11))
# ----------------------------------------------------------------------------------------

def ray_abc(prec, means, o, d):
    """A = d^T S^-1 d, B = 2 d^T S^-1 (o - mu), C = (o - mu)^T S^-1 (o - mu)  (R1)."""
    w = o[None, :] - means
    Pd = prec @ d                                            # [N,3]
    A = Pd @ d
    B = 2.0 * np.einsum("ni,ni->n", Pd, w)
    C = np.einsum("ni,nij,nj->n", w, prec, w)
    return A, B, C


@dataclass
class Candidates:
    idx: np.ndarray        # Gaussian indices, in level-0 stream order (R7)
    tstar: np.ndarray      # ray distance of the peak, Eq. (9)
    gstar: np.ndarray      # peak value G(t*), Eq. (10)
    alpha: np.ndarray      # min(0.99, o G*)
    A: np.ndarray
    B: np.ndarray
    C: np.ndarray


def pixel_candidates(scene: Scene, v: CameraView, px, py, subset=None) -> Candidates:
    """All Gaussians that contribute to pixel (px, py), in level-0 stream order."""
    cam = v.cam
    o = cam.center
    d, dc = cam.pixel_ray(px, py)
    ids = np.nonzero(v.live)[0] if subset is None else np.asarray(subset)[v.live[subset]]
    A, B, C = ray_abc(v.prec[ids], scene.means[ids], o, d)
    tstar = -B / (2.0 * A)
    qstar = np.maximum(0.0, C - B * B / (4.0 * A))
    gstar = np.exp(-0.5 * qstar)
    alpha = np.minimum(ALPHA_MAX, scene.opac[ids] * gstar)
    zpeak = tstar / np.linalg.norm(dc)                       # view z of the peak point
    keep = (alpha >= ALPHA_MIN) & (zpeak > NEAR)
    ids, tstar, gstar, alpha, A, B, C = (a[keep] for a in (ids, tstar, gstar, alpha, A, B, C))
    order = np.lexsort((ids, v.zkey32[ids]))                 # by (float32 zkey, index)
    return Candidates(*(a[order] for a in (ids, tstar, gstar, alpha, A, B, C)))


# ----------------------------------------------------------------------------------------
# Per-pixel order: full sort and the hierarchical (windowed) resort
# ----------------------------------------------------------------------------------------

def full_sort_order(keys):
    """Exact per-ray order: ascending key, ties by stream position."""
    return list(np.argsort(np.asarray(keys), kind="stable"))


def hierarchical_order(keys, window):
    """Hierarchical resort on top of the level-0 stream (the paper's StopThePop reference).

    Reading used here: level 0 is the stream (already in per-tile key order); level 1 is a
    per-pixel buffer of at most `window` entries.  While the buffer is not full a new entry
    is simply added.  Once full, each arriving entry competes with the buffer: the entry
    with the smallest (key, stream position) among buffer + newcomer is emitted and the
    other one stays.  At the end of the stream the buffer is emitted in ascending order.
    window = 0 reproduces the stream; window >= len(keys) reproduces the full sort.
    Returns stream positions in emission order.
    """
    keys = list(keys)
    out, buf = [], []
    for pos, k in enumerate(keys):
        if len(buf) < window:
            buf.append(pos)
            continue
        pool = buf + [pos]
        m = min(pool, key=lambda p: (keys[p], p))
        out.append(m)
        buf = [p for p in pool if p != m]
    out.extend(sorted(buf, key=lambda p: (keys[p], p)))
    return out


# ----------------------------------------------------------------------------------------
# Blending (Eq. (1)) and exact depth (Sec. 3.2, App. A.3)
# ----------------------------------------------------------------------------------------

@dataclass
class PixelResult:
    rgb: np.ndarray
    acc: float
    depth: float           # exact 0.5-level-set depth (R4, R5); 0 without crossing
    median_depth: float    # t*_k of the crossing Gaussian (GOF depth); 0 without crossing
    normal: np.ndarray     # sum_i w_i n_i (not normalised)
    T_end: float
    n_emitted: int
    k: int                 # Gaussian index of the crossing, -1 if none
    T_k: float
    order: list            # Gaussian indices in blending order
    order_t: list          # their t*
    weights: list          # their w = alpha T


def exact_depth(tstar, gstar, A, opac_k, T_k):
    """Solve T_k (1 - o_k G(t)) = 0.5 on the near side of the peak (R4).

    G(t) = G* exp(-A (t - t*)^2 / 2), so t = t* - sqrt(2 ln(G*/g) / A) with
    g = (T_k - 1/2) / (T_k o_k).
    """
    g = (T_k - 0.5) / (T_k * opac_k)
    return tstar - math.sqrt(max(0.0, 2.0 * math.log(gstar / g)) / A)


def blend(cands: Candidates, order, scene_opac, color, normal, bg=(0.0, 0.0, 0.0)):
    T = 1.0
    rgb = np.zeros(3)
    nrm = np.zeros(3)
    k = -1
    T_k = 0.0
    depth = 0.0
    median = 0.0
    emitted, emitted_t, weights = [], [], []
    for pos in order:
        a = cands.alpha[pos]
        test_T = T * (1.0 - a)
        if test_T < T_MIN:
            break
        gid = int(cands.idx[pos])
        w = a * T
        rgb += w * color[gid]
        nrm += w * normal[gid]
        if k < 0 and test_T <= 0.5:          # T > 0.5 holds while no crossing is recorded
            k, T_k = gid, T
            depth = exact_depth(cands.tstar[pos], cands.gstar[pos], cands.A[pos], scene_opac[gid], T)
            median = cands.tstar[pos]
        emitted.append(gid)
        emitted_t.append(float(cands.tstar[pos]))
        weights.append(w)
        T = test_T
    rgb = rgb + np.asarray(bg, np.float64) * T
    return PixelResult(rgb, 1.0 - T, depth, median, nrm, T, len(emitted), k, T_k,
                       emitted, emitted_t, weights)


def pixel_terms(scene: Scene, v: CameraView, px, py, ids):
    """t*, peak view z and alpha = min(0.99, o G*) of the listed Gaussians on the ray of pixel
    (px, py), whether or not they pass the candidate test (Eq. (9)-(10))."""
    ids = np.asarray(ids, np.int64)
    d, dc = v.cam.pixel_ray(px, py)
    A, B, C = ray_abc(v.prec[ids], scene.means[ids], v.cam.center, d)
    tstar = -B / (2.0 * A)
    gstar = np.exp(-0.5 * np.maximum(0.0, C - B * B / (4.0 * A)))
    alpha = np.minimum(ALPHA_MAX, scene.opac[ids] * gstar)
    return tstar, tstar / np.linalg.norm(dc), alpha, gstar, A


def blend_sequence(scene: Scene, v: CameraView, px, py, order_ids, k, bg=(0.0, 0.0, 0.0)):
    """Eq. (1) over a given sequence of Gaussians with a given crossing Gaussian.

    Every Gaussian of `order_ids` is blended in that order (no candidate, order or
    termination decision is taken here) and the exact depth (R4) is taken on Gaussian `k`
    (-1: no crossing) with T_k the transmittance in front of it.  This lets a result whose
    discrete decisions were taken elsewhere (for instance in float32, near a threshold) be
    recomputed in float64 with exactly those decisions."""
    ids = [int(i) for i in order_ids]
    T = 1.0
    rgb, nrm = np.zeros(3), np.zeros(3)
    depth = median = 0.0
    T_k = 0.0
    weights, ts = [], []
    if ids:
        tstar, _, alpha, gstar, A = pixel_terms(scene, v, px, py, ids)
    for j, gid in enumerate(ids):
        a = alpha[j]
        w = a * T
        rgb += w * v.color[gid]
        nrm += w * v.normal[gid]
        if gid == k:
            T_k = T
            depth = exact_depth(tstar[j], gstar[j], A[j], scene.opac[gid], T)
            median = tstar[j]
        weights.append(w)
        ts.append(float(tstar[j]))
        T *= 1.0 - a
    rgb = rgb + np.asarray(bg, np.float64) * T
    return PixelResult(rgb, 1.0 - T, depth, median, nrm, T, len(ids), int(k), T_k, ids, ts, weights)


def render_pixel(scene: Scene, v: CameraView, px, py, window, bg=(0.0, 0.0, 0.0), subset=None):
    """One pixel: candidates -> hierarchical order (window >= 2**30 means full sort) -> blend."""
    cands = pixel_candidates(scene, v, px, py, subset)
    if window >= 2 ** 30:
        order = full_sort_order(cands.tstar)
    else:
        order = hierarchical_order(cands.tstar, window)
    return blend(cands, order, scene.opac, v.color, v.normal, bg)


FULL_SORT = 2 ** 30


def render(scene: Scene, cam: Camera, window, pixels=None, bg=(0.0, 0.0, 0.0)):
    """Render `pixels` (list of (px, py); default every pixel).  Returns dict of arrays
    indexed like `pixels` plus the per-pixel PixelResult list."""
    v = view(scene, cam)
    if pixels is None:
        pixels = [(x, y) for y in range(cam.height) for x in range(cam.width)]
    res = [render_pixel(scene, v, px, py, window, bg) for (px, py) in pixels]
    return {
        "rgb": np.array([r.rgb for r in res]).reshape(-1, 3),
        "acc": np.array([r.acc for r in res]),
        "depth": np.array([r.depth for r in res]),
        "median_depth": np.array([r.median_depth for r in res]),
        "normal": np.array([r.normal for r in res]).reshape(-1, 3),
        "T_end": np.array([r.T_end for r in res]),
        "n_emitted": np.array([r.n_emitted for r in res]),
        "k": np.array([r.k for r in res]),
        "T_k": np.array([r.T_k for r in res]),
        "results": res,
        "pixels": pixels,
    }


# ----------------------------------------------------------------------------------------
# Opacity field (Eq. (12)-(13)); order independent by App. A.2
# ----------------------------------------------------------------------------------------

def point_view_valid(cam: Camera, x):
    xc = cam.R @ x + cam.t
    if not xc[2] > NEAR:
        return False
    u = cam.fx * xc[0] / xc[2] + cam.cx
    w = cam.fy * xc[1] / xc[2] + cam.cy
    return (0.0 <= u < cam.width) and (0.0 <= w < cam.height)


def view_alphas(scene: Scene, v: CameraView, x):
    """alpha_i(t_eval) of every contributing Gaussian for point x seen from camera v."""
    cam = v.cam
    o = cam.center
    t = np.linalg.norm(x - o)
    d = (x - o) / t
    ids = np.nonzero(v.live)[0]
    A, B, C = ray_abc(v.prec[ids], scene.means[ids], o, d)
    tstar = -B / (2.0 * A)
    te = np.minimum(tstar, t)
    q = np.maximum(0.0, A * te * te + B * te + C)
    alpha = np.minimum(ALPHA_MAX, scene.opac[ids] * np.exp(-0.5 * q))
    zc = (cam.R @ d)[2] * te                                 # view z of the evaluated point
    keep = (alpha >= ALPHA_MIN) & (zc > NEAR)
    return ids[keep], alpha[keep]


def opacity_field_view(scene: Scene, v: CameraView, x):
    """O_N(x) for one camera: sum_i alpha_i prod_{j<i} (1 - alpha_j), evaluated here in the
    product form 1 - prod(1 - alpha) that App. A.2 proves equal."""
    _, alpha = view_alphas(scene, v, x)
    return 1.0 - float(np.prod(1.0 - alpha))


def opacity_field_view_sum(scene: Scene, v: CameraView, x):
    """O_N(x) in the literal front-to-back sum form of Eq. (12) (any order)."""
    _, alpha = view_alphas(scene, v, x)
    s, T = 0.0, 1.0
    for a in alpha:
        s += a * T
        T *= 1.0 - a
    return s


def opacity_field(scene: Scene, cams, points, views=None):
    """O(x) = min over cameras that see x of O_N(x)  (Eq. (13), R10)."""
    views = views or [view(scene, c) for c in cams]
    out = np.ones(len(points))
    for i, x in enumerate(np.asarray(points, np.float64)):
        best = 1.0
        for v in views:
            if point_view_valid(v.cam, x):
                best = min(best, opacity_field_view(scene, v, x))
        out[i] = best
    return out


# ----------------------------------------------------------------------------------------
# Tile lists (conservative screen bounds of the E-ellipsoid, then the per-tile key sort)
# ----------------------------------------------------------------------------------------

def gaussian_bounds(scene: Scene, cam: Camera):
    """Per Gaussian: (live, u_min, u_max, v_min, v_max) in pixels, and z_min.

    If the E-ellipsoid lies in front of the near plane, the bound is its exact silhouette
    (the image of the dual quadric, N = mu mu^T - E^2 Sigma in camera space).  Otherwise it
    is the projection of the camera-space bounding box clipped to z >= tau_n.
    z_min = mu_z - E sqrt(Sigma_zz) is the smallest view z on the ellipsoid (Eq. (15),
    with sqrt of the view-space z variance as the extent along z).
    """
    mu_c = scene.means @ cam.R.T + cam.t[None, :]
    Sc = np.einsum("ij,njk,lk->nil", cam.R, scene.covariances(), cam.R)
    E = opacity_cutoff(np.maximum(scene.opac, ALPHA_MIN))
    live = (scene.opac >= ALPHA_MIN) & (mu_c[:, 2] > NEAR)
    n = scene.n
    box = np.zeros((n, 4))
    zmin = mu_c[:, 2] - E * np.sqrt(Sc[:, 2, 2])
    for i in range(n):
        if not live[i]:
            continue
        m, S, e = mu_c[i], Sc[i], E[i]
        if zmin[i] > NEAR:
            N = np.outer(m, m) - e * e * S
            r = []
            for a in (0, 1):
                disc = max(0.0, N[a, 2] ** 2 - N[a, a] * N[2, 2])
                lo = (N[a, 2] - math.sqrt(disc)) / N[2, 2]
                hi = (N[a, 2] + math.sqrt(disc)) / N[2, 2]
                r.append((lo, hi))
            (xl, xh), (yl, yh) = r
        else:
            ex = e * np.sqrt(np.diag(S))
            zs = (NEAR, m[2] + ex[2])
            xs = [(m[0] + sx * ex[0]) / z for sx in (-1, 1) for z in zs]
            ys = [(m[1] + sy * ex[1]) / z for sy in (-1, 1) for z in zs]
            xl, xh, yl, yh = min(xs), max(xs), min(ys), max(ys)
        box[i] = (cam.fx * xl + cam.cx, cam.fx * xh + cam.cx, cam.fy * yl + cam.cy, cam.fy * yh + cam.cy)
    return live, box, zmin


def pixel_rects(live, box, width, height):
    """Inclusive pixel rectangles [x0, x1] x [y0, y1] with a one-pixel margin, clamped to
    the image; an empty rectangle has x0 > x1 or y0 > y1."""
    lim = 1e7
    b = np.clip(box, -lim, lim)
    x0 = np.floor(b[:, 0]).astype(np.int64) - 1
    x1 = np.floor(b[:, 1]).astype(np.int64) + 1
    y0 = np.floor(b[:, 2]).astype(np.int64) - 1
    y1 = np.floor(b[:, 3]).astype(np.int64) + 1
    x0, y0 = np.maximum(x0, 0), np.maximum(y0, 0)
    x1, y1 = np.minimum(x1, width - 1), np.minimum(y1, height - 1)
    rect = np.stack([x0, y0, x1, y1], axis=1)
    rect[~live] = (0, 0, -1, -1)
    empty = (rect[:, 0] > rect[:, 2]) | (rect[:, 1] > rect[:, 3])
    rect[empty] = (0, 0, -1, -1)
    return rect


def tile_lists(rect, key32, tile, width, height):
    """Integer stage: every (tile, Gaussian) pair covered by `rect`, ordered by
    (tile, float32 key, index) -- one global sort, then split per tile.

    Returns (ids_sorted, tile_of_each, ranges[n_tiles, 2])."""
    tx = (width + tile - 1) // tile
    ty = (height + tile - 1) // tile
    tiles, ids = [], []
    for i in range(rect.shape[0]):
        x0, y0, x1, y1 = rect[i]
        if x0 > x1 or y0 > y1:
            continue
        for yy in range(y0 // tile, y1 // tile + 1):
            for xx in range(x0 // tile, x1 // tile + 1):
                tiles.append(yy * tx + xx)
                ids.append(i)
    tiles = np.array(tiles, np.int64)
    ids = np.array(ids, np.int64)
    keys = np.asarray(key32, np.float32)[ids] if len(ids) else np.zeros(0, np.float32)
    order = np.lexsort((ids, keys, tiles))
    tiles, ids = tiles[order], ids[order]
    ranges = np.zeros((tx * ty, 2), np.int64)
    for t in range(tx * ty):
        ranges[t] = (np.searchsorted(tiles, t, "left"), np.searchsorted(tiles, t, "right"))
    return ids, tiles, ranges


# ----------------------------------------------------------------------------------------
# Finite-difference gradients of the composite render (the backward pass's reference)
# ----------------------------------------------------------------------------------------

PARAM_NAMES = ("means", "scales", "quats", "opac", "sh")


def _scene_with(scene: Scene, name, flat_index, value):
    arrs = {k: getattr(scene, k).copy() for k in PARAM_NAMES}
    a = arrs[name].reshape(-1)
    a[flat_index] = value
    arrs[name] = a.reshape(getattr(scene, name).shape)
    return Scene(arrs["means"], arrs["scales"], arrs["quats"], arrs["opac"], arrs["sh"], scene.sh_degree)


def opacity_at_depth(scene: Scene, v: CameraView, px, py, res: PixelResult, t_r=None):
    """O_N(o + t_r d) over the Gaussians blended at this pixel (R17), or None without a
    crossing.  t_r defaults to the pixel's exact depth.  Also returns the ids that count
    (alpha at t_eval >= 1/255 and evaluated point beyond the near plane)."""
    if res.k < 0:
        return None, []
    cam = v.cam
    o = cam.center
    d, dc = cam.pixel_ray(px, py)
    t_r = res.depth if t_r is None else t_r
    ids = np.asarray(res.order, dtype=np.int64)
    A, B, C = ray_abc(v.prec[ids], scene.means[ids], o, d)
    tstar = -B / (2.0 * A)
    te = np.minimum(tstar, t_r)
    q = np.maximum(0.0, A * te * te + B * te + C)
    alpha = np.minimum(ALPHA_MAX, scene.opac[ids] * np.exp(-0.5 * q))
    zc = te / np.linalg.norm(dc)                              # view z of the evaluated point
    keep = (alpha >= ALPHA_MIN) & (zc > NEAR)
    return 1.0 - float(np.prod(1.0 - alpha[keep])), [int(i) for i in ids[keep]]


NDC_NEAR, NDC_FAR = 0.2, 100.0


def ndc(t):
    """Ray distance -> NDC depth in [0, 1] over [n, f] (R18)."""
    return NDC_FAR * (t - NDC_NEAR) / ((NDC_FAR - NDC_NEAR) * t)


def distortion_extent(scene: Scene, v: CameraView, px, py, res: PixelResult):
    """Per-pixel distortion loss sum_ij w_i w_j (NDC(t*_i) - NDC(t*_j))^2 and extent loss
    f n / (f - n) sum_i w_i 2 A_i sqrt(B_i^2 - 4 A_i (C_i - E_i^2)) / B_i^2 over the blended
    Gaussians (A, B, C of the unit pixel ray, E_i^2 = 2 ln(255 o_i))."""
    if not res.order:
        return 0.0, 0.0
    w = np.asarray(res.weights)
    d = ndc(np.asarray(res.order_t))
    dist = float(np.sum(w[:, None] * w[None, :] * (d[:, None] - d[None, :]) ** 2))
    ids = np.asarray(res.order, dtype=np.int64)
    dvec, _ = v.cam.pixel_ray(px, py)
    A, B, C = ray_abc(v.prec[ids], scene.means[ids], v.cam.center, dvec)
    E2 = 2.0 * np.log(255.0 * scene.opac[ids])
    ext_i = 2.0 * A * np.sqrt(np.maximum(B * B - 4.0 * A * (C - E2), 0.0)) / (B * B)
    ext = NDC_FAR * NDC_NEAR / (NDC_FAR - NDC_NEAR) * float(np.sum(w * ext_i))
    return dist, ext


def linear_loss(scene: Scene, cams, window, pixel_lists, weights, depth_mode="exact", bg=(0, 0, 0),
                opa_weights=None, opa_depths=None, loss_weights=None):
    """L = sum over cameras and listed pixels of <weights, (rgb, acc, depth, normal)>.

    weights[c] is [len(pixel_lists[c]), 8] = (rgb 3, acc, depth, normal 3).  depth_mode
    'exact' uses the 0.5-level-set depth; 'median' uses t*_k (what a detached exact-depth
    correction differentiates to).  opa_weights[c][i] adds that multiple of the opacity at
    the rendered depth (R17; pixels without a crossing add nothing), evaluated at the fixed
    ray distance opa_depths[c][i] when given (a detached depth); loss_weights[c][i] weighs
    the pixel's (distortion, extent) losses (R18).  Returns (loss, signature);
    the signature (emitted ids, crossing index and the ids that count in the opacity per
    pixel) tells whether two evaluations lie in the same smooth piece of the function."""
    loss = 0.0
    sig = []
    for c, (cam, pix, wts) in enumerate(zip(cams, pixel_lists, weights)):
        v = view(scene, cam)
        for i, ((px, py), w) in enumerate(zip(pix, wts)):
            r = render_pixel(scene, v, px, py, window, bg)
            dep = r.depth if depth_mode == "exact" else r.median_depth
            vec = np.concatenate([r.rgb, [r.acc, dep], r.normal])
            loss += float(np.dot(vec, w))
            if loss_weights is not None:
                dist, ext = distortion_extent(scene, v, px, py, r)
                loss += loss_weights[c][i][0] * dist + loss_weights[c][i][1] * ext
            used = []
            if opa_weights is not None:
                t_r = None if opa_depths is None else opa_depths[c][i]
                on, used = opacity_at_depth(scene, v, px, py, r, t_r)
                if on is not None:
                    loss += opa_weights[c][i] * on
            sig.append((tuple(r.order), r.k, tuple(used)))
    return loss, sig


def fd_gradient(scene: Scene, cams, window, pixel_lists, weights, depth_mode="exact",
                names=PARAM_NAMES, h_rel=1e-6, bg=(0, 0, 0), opa_weights=None, opa_depths=None, loss_weights=None):
    """Central differences of `linear_loss` for every element of the named parameters.

    Returns {name: (grad, smooth)}; smooth[i] is False where the two evaluations fall in
    different smooth pieces (another candidate set, order, termination or crossing)."""
    out = {}
    for name in names:
        base = getattr(scene, name)
        flat = base.reshape(-1)
        g = np.zeros(flat.shape)
        ok = np.ones(flat.shape, bool)
        for i in range(flat.size):
            h = h_rel * max(1.0, abs(flat[i]))
            lp, sp = linear_loss(_scene_with(scene, name, i, flat[i] + h), cams, window, pixel_lists, weights, depth_mode,
                                 bg, opa_weights, opa_depths, loss_weights)
            lm, sm = linear_loss(_scene_with(scene, name, i, flat[i] - h), cams, window, pixel_lists, weights, depth_mode,
                                 bg, opa_weights, opa_depths, loss_weights)
            g[i] = (lp - lm) / (2.0 * h)
            ok[i] = sp == sm
        out[name] = (g.reshape(base.shape), ok.reshape(base.shape))
    return out


# ----------------------------------------------------------------------------------------
# Level set of the opacity field: classification and binary search (Sec. 3.4)
# ----------------------------------------------------------------------------------------

def inside(scene: Scene, cams, points, views=None):
    """O(x) > 0.5 for every point (the only thing the binary search needs)."""
    return opacity_field(scene, cams, points, views) > 0.5


def bisect_level_set(scene: Scene, cams, a, b, steps=8):
    """Binary search on edges (a[i] inside, b[i] outside) for the 0.5 level set (R16).

    Returns the final midpoints and the per-step decisions [steps, n] (True: the midpoint
    was inside, so it replaced a)."""
    views = [view(scene, c) for c in cams]
    a = np.array(a, np.float64)
    b = np.array(b, np.float64)
    decisions = []
    for _ in range(steps):
        mid = 0.5 * (a + b)
        ins = inside(scene, cams, mid, views)
        a = np.where(ins[:, None], mid, a)
        b = np.where(ins[:, None], b, mid)
        decisions.append(ins)
    return 0.5 * (a + b), np.array(decisions).reshape(steps, len(a))


# ----------------------------------------------------------------------------------------
# 3D filter (App. "Dead Gaussians"; filter size per R19)
# ----------------------------------------------------------------------------------------

def filter3d_variance(scene: Scene, cams, k=0.2):
    """s_i = (k / nu_i)^2, nu_i = max f_x / z over cameras that see the centre (R19)."""
    s = np.zeros(scene.n)
    for i in range(scene.n):
        best = 0.0
        for cam in cams:
            if point_view_valid(cam, scene.means[i]):
                z = (cam.R @ scene.means[i] + cam.t)[2]
                best = max(best, cam.fx / z)
        s[i] = (k / best) ** 2 if best > 0.0 else 0.0
    return s


def filter3d(scene: Scene, var):
    """Sigma + s I keeps the rotation and adds s to every squared scale; the opacity is
    scaled by sqrt(|Sigma| / |Sigma + s I|).  Returns (scales, opacities)."""
    s2 = scene.scales ** 2
    new_s2 = s2 + var[:, None]
    det_ratio = np.linalg.det(scene.covariances()) / np.linalg.det(
        scene.covariances() + var[:, None, None] * np.eye(3)[None])
    return np.sqrt(new_s2), scene.opac * np.sqrt(det_ratio)
