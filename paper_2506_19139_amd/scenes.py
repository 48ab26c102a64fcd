"""Seeded synthetic inputs: Gaussian clouds, cameras and query points.

These generators hold none of the method's arithmetic; they only draw random numbers and
place pinhole cameras.  The same float32 arrays feed the HIP library and the CPU oracle.

Workloads (all float32, numpy PCG64 `default_rng(seed)`, draws in the order means,
log-scales, rotations, opacity logits, SH):

* ``small``      1,000 Gaussians, means U[-1,1]^3, log-scales N(-3,0.5), opacities
                 sigmoid(N(0,1)), SH degree 0 (colours U[0,1]); one 64x64 camera at
                 (0,0,-4) looking at the origin, fov 60 deg.
* ``clusters``   200k Gaussians in 50 anisotropic clusters inside a 10 m box, SH degree 3
                 coefficients N(0,0.2), opacities sigmoid(N(0,1.5)); one 1280x720 camera on
                 a circle of radius 8 m.
* ``unbounded``  1M Gaussians: 70 % uniform in a 10 m box, 30 % background at log-uniform
                 radius 10..1000 m; log-scales ln(0.005 max(|mu|,1)) + N(0,0.5); SH degree 3;
                 one 1920x1080 camera at radius 8 m.
* ``query``      the unbounded recipe at 3M Gaussians; query points are every centre plus
                 the 8 corners of its 3-sigma box (9 points per Gaussian); 96 cameras on two
                 rings of 48 (radius 8 m, heights +-2 m), 960x540.
* ``multiview``  the unbounded recipe at 1M Gaussians; 8 cameras every 45 deg on the radius
                 8 m circle with resolutions from 640x360 up to 1920x1080.
"""

from __future__ import annotations

import math

import numpy as np

SH_C0 = 0.28209479177387814      # Y_0^0, used only to store a plain colour as an SH coefficient


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _unit_quats(rng, n):
    q = rng.standard_normal((n, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def look_at(center, width, height, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0), fov_x_deg=60.0):
    """World->camera pinhole with OpenCV axes (x right, y down, z forward)."""
    c = np.asarray(center, np.float64)
    f = np.asarray(target, np.float64) - c
    f /= np.linalg.norm(f)
    down = -np.asarray(up, np.float64)
    x = np.cross(down, f)
    x /= np.linalg.norm(x)
    y = np.cross(f, x)
    R = np.stack([x, y, f])
    t = -R @ c
    fx = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    return dict(R=R.astype(np.float32), t=t.astype(np.float32), fx=np.float32(fx), fy=np.float32(fx),
                cx=np.float32(width / 2.0), cy=np.float32(height / 2.0), width=int(width), height=int(height))


def _pack(means, log_scales, quats, opac_logit, sh, deg):
    return dict(means=np.ascontiguousarray(means, np.float32),
                scales=np.ascontiguousarray(np.exp(log_scales), np.float32),
                quats=np.ascontiguousarray(quats, np.float32),
                opac=np.ascontiguousarray(_sigmoid(opac_logit), np.float32),
                sh=np.ascontiguousarray(sh, np.float32),
                sh_degree=int(deg))


def small_scene(n=1000, seed=0):
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, (n, 3))
    log_s = rng.normal(-3.0, 0.5, (n, 3))
    quats = _unit_quats(rng, n)
    logit = rng.normal(0.0, 1.0, n)
    col = rng.uniform(0.0, 1.0, (n, 3))
    sh = ((col - 0.5) / SH_C0).reshape(n, 1, 3)
    return _pack(means, log_s, quats, logit, sh, 0)


def small_camera(width=64, height=64):
    fx = (width / 2.0) / math.tan(math.radians(30.0))
    return dict(R=np.eye(3, dtype=np.float32), t=np.array([0, 0, 4], np.float32), fx=np.float32(fx),
                fy=np.float32(fx), cx=np.float32(width / 2.0), cy=np.float32(height / 2.0),
                width=int(width), height=int(height))


def cluster_scene(n=200_000, seed=0, n_clusters=50):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-4.0, 4.0, (n_clusters, 3))
    stds = rng.uniform(0.2, 1.0, (n_clusters, 3))
    rots = np.stack([np.linalg.qr(rng.standard_normal((3, 3)))[0] for _ in range(n_clusters)])
    which = rng.integers(0, n_clusters, n)
    local = rng.standard_normal((n, 3)) * stds[which]
    means = np.clip(centres[which] + np.einsum("nij,nj->ni", rots[which], local), -5.0, 5.0)
    log_s = rng.normal(-3.0, 0.5, (n, 3))
    quats = _unit_quats(rng, n)
    logit = rng.normal(0.0, 1.5, n)
    sh = rng.normal(0.0, 0.2, (n, 16, 3))
    return _pack(means, log_s, quats, logit, sh, 3)


def unbounded_scene(n=1_000_000, seed=0, fg_fraction=0.7, sh_degree=3):
    rng = np.random.default_rng(seed)
    n_fg = int(round(n * fg_fraction))
    n_bg = n - n_fg
    fg = rng.uniform(-5.0, 5.0, (n_fg, 3))
    dirs = rng.standard_normal((n_bg, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    radius = 10.0 ** rng.uniform(1.0, 3.0, n_bg)
    means = np.concatenate([fg, dirs * radius[:, None]])
    dist = np.maximum(np.linalg.norm(means, axis=1), 1.0)
    log_s = np.log(0.005 * dist)[:, None] + rng.normal(0.0, 0.5, (n, 3))
    quats = _unit_quats(rng, n)
    logit = rng.normal(0.0, 1.5, n)
    k = (sh_degree + 1) ** 2
    sh = rng.normal(0.0, 0.2, (n, k, 3))
    return _pack(means, log_s, quats, logit, sh, sh_degree)


def circle_camera(azimuth_rad, width, height, radius=8.0, height_y=0.0):
    c = (radius * math.cos(azimuth_rad), height_y, radius * math.sin(azimuth_rad))
    return look_at(c, width, height)


def ring_cameras(n_per_ring=48, width=960, height=540, radius=8.0, heights=(2.0, -2.0)):
    cams = []
    for ring, hy in enumerate(heights):
        for j in range(n_per_ring):
            az = 2.0 * math.pi * (j + 0.5 * ring) / n_per_ring
            cams.append(circle_camera(az, width, height, radius, hy))
    return cams


MULTIVIEW_SIZES = [(640, 360), (800, 450), (960, 540), (1120, 630),
                   (1280, 720), (1440, 810), (1600, 900), (1920, 1080)]


def multiview_cameras(sizes=MULTIVIEW_SIZES):
    return [circle_camera(math.radians(45.0 * k), w, h) for k, (w, h) in enumerate(sizes)]


def box_corner_points(scene, sigmas=3.0):
    """Every centre and the 8 corners mu + R (+-3 s_x, +-3 s_y, +-3 s_z), binary sign order
    (9 points per Gaussian, centre first).  The rotation comes from scipy."""
    from scipy.spatial.transform import Rotation
    q = scene["quats"].astype(np.float64)
    rot = Rotation.from_quat(q[:, [1, 2, 3, 0]])
    s = scene["scales"].astype(np.float64) * sigmas
    mu = scene["means"].astype(np.float64)
    pts = [mu]
    for b in range(8):
        sign = np.array([1.0 if (b >> 2) & 1 else -1.0, 1.0 if (b >> 1) & 1 else -1.0,
                         1.0 if b & 1 else -1.0])
        pts.append(mu + rot.apply(s * sign[None, :]))
    return np.ascontiguousarray(np.stack(pts, axis=1).reshape(-1, 3), np.float32)


def random_points(n, seed, low=-5.0, high=5.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(low, high, (n, 3)).astype(np.float32)


def target_image(height, width, seed=1):
    return np.random.default_rng(seed).uniform(0.0, 1.0, (3, height, width)).astype(np.float32)


def tiny_scene(n=6, seed=0, sh_degree=1, spread=0.35, log_scale=-1.6):
    """A handful of well-separated, fairly large Gaussians in front of a small camera, for
    finite-difference gradient checks."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-spread, spread, (n, 3))
    log_s = rng.normal(log_scale, 0.25, (n, 3))
    quats = _unit_quats(rng, n)
    logit = rng.normal(0.0, 1.0, n)
    sh = rng.normal(0.0, 0.3, (n, (sh_degree + 1) ** 2, 3))
    return _pack(means, log_s, quats, logit, sh, sh_degree)


def subset_scene(scene, ids):
    out = {k: np.ascontiguousarray(v[ids]) for k, v in scene.items() if k != "sh_degree"}
    out["sh_degree"] = scene["sh_degree"]
    return out
