"""GPU opacity-field queries (sof_opacity_query through the C ABI) against the FP64
oracle's brute-force evaluation over all Gaussians and views (Eq. (12)-(13)).  Bar: 1e-4
absolute; batched (all views, one persistent launch) equals per-view launches exactly."""
import numpy as np
import pytest
import torch

from oracle import sof_oracle as O
from paper_2506_19139_amd import scenes, sof

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _run(scene, cams, pts, tile=16):
    g = sof.Gaussians.from_numpy(scene)
    C = sof.Cameras(cams)
    q = sof.OpacityQuery(C, sof.Options(tile=tile))
    out = q(g, torch.from_numpy(pts).cuda())
    torch.cuda.synchronize()
    return out.cpu().numpy(), q


def _oracle(scene, cams, pts):
    sc = O.Scene.from_arrays(**scene)
    return O.opacity_field(sc, [O.Camera.from_arrays(**c) for c in cams], pts)


def _ring(n, w=64, h=48, radius=3.0):
    return [scenes.circle_camera(2 * np.pi * k / n, w, h, radius=radius, height_y=0.5 * (-1) ** k) for k in range(n)]


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_query_small_scene_many_views(tile):
    scene = scenes.small_scene(400, seed=4)
    cams = _ring(6)
    pts = np.concatenate([scenes.box_corner_points(scenes.subset_scene(scene, np.arange(60))),
                          scenes.random_points(200, seed=7, low=-1.2, high=1.2)])
    print(f"[case] query small scene 6 views tile {tile}, {len(pts)} points", flush=True)
    got, q = _run(scene, cams, pts, tile)
    ref = _oracle(scene, cams, pts)
    err = np.abs(got - ref)
    print(f"max err {err.max():.2e}, unobserved {np.sum(ref == 1.0)}, pairs {q.last[1]}")
    assert err.max() <= TOL


def test_query_points_on_pixel_rays_match_render():
    """Points beyond every Gaussian on a pixel-centre ray see O_N = the pixel's acc (up to
    early termination of the render): render <-> query cross-check on the GPU."""
    scene = scenes.small_scene(300, seed=9)
    cam = scenes.small_camera(32, 32)
    C = sof.Cameras([cam])
    g = sof.Gaussians.from_numpy(scene)
    r = sof.Rasterizer(C, sof.Options(tile=16, window=8))
    out = r.forward(g)
    acc = out["acc"].cpu().numpy().reshape(32, 32)
    T_end = out["aux"][:1024].cpu().numpy().reshape(32, 32)
    pix = [(x, y) for y in range(4, 28, 3) for x in range(4, 28, 3)]
    f = float(cam["fx"])
    pts = []
    for x, y in pix:
        d = np.array([(x + 0.5 - 16) / f, (y + 0.5 - 16) / f, 1.0])
        pts.append(np.array([0, 0, -4.0]) + 40.0 * d / np.linalg.norm(d))
    pts = np.array(pts, np.float32)
    got, _ = _run(scene, [cam], pts)
    for i, (x, y) in enumerate(pix):
        if T_end[y, x] > 2e-4:                         # no early termination in the render
            assert abs(got[i] - acc[y, x]) <= 2e-5, (x, y, got[i], acc[y, x])


def test_batched_equals_per_view():
    scene = scenes.small_scene(400, seed=5)
    cams = _ring(5)
    pts = scenes.random_points(500, seed=8, low=-1.0, high=1.0)
    batched, _ = _run(scene, cams, pts)
    per = np.ones(len(pts), np.float32)
    for c in cams:
        o, _ = _run(scene, [c], pts)
        per = np.minimum(per, o)
    assert np.array_equal(batched, per)


def test_query_unbounded_sampled():
    """Unbounded recipe (foreground box + far background), 8 views, sampled points."""
    scene = scenes.unbounded_scene(20000, seed=3)
    cams = [scenes.circle_camera(2 * np.pi * k / 8, 240, 135, height_y=(2.0 if k % 2 else -2.0)) for k in range(8)]
    pts = scenes.box_corner_points(scenes.subset_scene(scene, np.arange(0, 20000, 100)))
    print(f"[case] query unbounded 20k Gaussians 8 views, {len(pts)} points", flush=True)
    got, q = _run(scene, cams, pts)
    ref = _oracle(scene, cams, pts)
    err = np.abs(got - ref)
    print(f"max err {err.max():.2e} mean {err.mean():.2e}")
    assert err.max() <= TOL


def test_query_capacity_growth_and_empty():
    scene = scenes.small_scene(100, seed=1)
    cams = _ring(3)
    pts = np.zeros((0, 3), np.float32)
    got, _ = _run(scene, cams, pts)
    assert got.shape == (0,)
    far = np.full((10, 3), 100.0, np.float32)             # seen by no camera -> 1
    got, _ = _run(scene, cams, far)
    assert np.all(got == 1.0)


def test_query_wide_tile_ids_use_exact_lists():
    """More than 2^20 tiles (36 views of 1920x1080 at tile 8): the tile lists fall back to
    64-bit keys with exact z_min order.  Matches the oracle, and the compact lists of three
    12-view calls to 1e-6 (the two list orders multiply the same factors in another order)."""
    scene = scenes.small_scene(300, seed=12)
    cams = [scenes.circle_camera(2 * np.pi * k / 36, 1920, 1080, radius=3.0, height_y=0.4 * (-1) ** k)
            for k in range(36)]
    tiles = sum(((c["width"] + 7) // 8) * ((c["height"] + 7) // 8) for c in cams)
    assert tiles > 2 ** 20
    pts = scenes.random_points(300, seed=13, low=-1.0, high=1.0)
    print(f"[case] query {tiles} tiles, 36 views 1920x1080, {len(pts)} points", flush=True)
    got, _ = _run(scene, cams, pts, tile=8)
    ref = _oracle(scene, cams, pts)
    err = np.abs(got - ref)
    print(f"max err {err.max():.2e}")
    assert err.max() <= TOL
    per = np.ones(len(pts), np.float32)
    for k in range(0, 36, 12):                       # 12 views per call: compact lists
        o, _ = _run(scene, cams[k:k + 12], pts, tile=8)
        per = np.minimum(per, o)
    assert np.abs(got - per).max() <= 1e-6


def test_reuse_of_the_gaussian_side_matches_a_fresh_query():
    """SOF_QUERY_REUSE: a second point set against the projection and tile lists left by the
    previous call gives exactly what a fresh call gives."""
    scene = scenes.small_scene(300, seed=14)
    cams = _ring(4)
    g = sof.Gaussians.from_numpy(scene)
    C = sof.Cameras(cams)
    q = sof.OpacityQuery(C, sof.Options(tile=8))
    p1 = torch.from_numpy(scenes.random_points(400, seed=15, low=-1.0, high=1.0)).cuda()
    p2 = torch.from_numpy(scenes.random_points(700, seed=16, low=-1.0, high=1.0)).cuda()
    q(g, p1)
    reused = q(g, p2, reuse_gaussians=True).cpu().numpy()
    fresh = sof.OpacityQuery(C, sof.Options(tile=8))(g, p2).cpu().numpy()
    assert np.array_equal(reused, fresh)
