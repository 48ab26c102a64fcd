"""Distortion and extent losses inside the rasteriser (Sec. 3.3; App. C.1, C.2), against the
FP64 oracle's definitions: per-pixel values on a full small frame and gradients by central
differences on tiny scenes (per-tensor relative error <= 1e-3)."""
import numpy as np
import pytest
import torch

from gpu_helpers import fragile, gpu_render, oracle_scene_cam, unpack
from oracle import sof_oracle as O
from paper_2506_19139_amd import scenes, sof

pytestmark = pytest.mark.gpu
NAMES = ("means", "scales", "quats", "opac", "sh")


@pytest.mark.parametrize("tile,window", [(16, 8), (8, 0)])
def test_losses_full_frame(tile, window):
    scene, cam = scenes.small_scene(), scenes.small_camera()
    print(f"[case] losses, small scene 64x64 tile {tile} window {window}", flush=True)
    g = sof.Gaussians.from_numpy(scene)
    C = sof.Cameras([cam])
    r = sof.Rasterizer(C, sof.Options(tile=tile, window=window))
    out = r.forward(g, losses=True)
    torch.cuda.synchronize()
    host = {k: v.cpu().numpy() for k, v in out.items()}
    gpu = unpack(host, [cam])
    W, H = cam["width"], cam["height"]
    L = host["losses"].reshape(sof.LOSS_CHANNELS, H * W)
    sc, oc = oracle_scene_cam(scene, cam)
    v = O.view(sc, oc)
    worst = [0.0, 0.0]
    compared = skipped = 0
    for py in range(H):
        for px in range(W):
            res = O.render_pixel(sc, v, px, py, window)
            gi = py * W + px
            if gpu["n_emitted"][gi] != res.n_emitted:
                assert fragile(sc, v, px, py, res), (px, py)
                skipped += 1
                continue
            dist, ext = O.distortion_extent(sc, v, px, py, res)
            for c, ref in enumerate((dist, ext)):
                err = abs(L[c, gi] - ref) / max(1e-3, abs(ref))
                worst[c] = max(worst[c], err)
            compared += 1
    print(f"  compared {compared} pixels, skipped {skipped}; worst relative error distortion {worst[0]:.2e}, "
          f"extent {worst[1]:.2e}")
    assert compared > 4000 and skipped <= 3
    assert max(worst) <= 1e-4


def _camera(w=16, h=12):
    f = (w / 2) / np.tan(np.radians(14.0))
    return dict(R=np.eye(3, dtype=np.float32), t=np.array([0, 0, 2.0], np.float32), fx=np.float32(f),
                fy=np.float32(f), cx=np.float32(w / 2), cy=np.float32(h / 2), width=w, height=h)


@pytest.mark.parametrize("seed,window", [(0, 4), (1, 8), (2, 0)])
def test_loss_gradients_match_finite_differences(seed, window):
    scene = scenes.tiny_scene(n=8, seed=seed, sh_degree=1, log_scale=-1.4)
    cam = _camera()
    W, H = cam["width"], cam["height"]
    P = W * H
    rng = np.random.default_rng(300 + seed)
    up = rng.normal(0, 1, (P, 8)).astype(np.float32)
    wl = rng.normal(0, 1, (P, 2)).astype(np.float32) * np.array([20.0, 1.0], np.float32)
    g = sof.Gaussians.from_numpy(scene)
    rast = sof.Rasterizer(sof.Cameras([cam]), sof.Options(tile=8, window=window))
    out = rast.forward(g, losses=True)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    gr = rast.backward(g, out, dev(up[:, 0:3].T.reshape(-1)), dev(up[:, 3]), dev(up[:, 4]), dev(up[:, 5:8].T.reshape(-1)),
                       d_losses=dev(wl.T.reshape(-1)))
    torch.cuda.synchronize()
    gpu = {k: v.cpu().numpy().astype(np.float64) for k, v in gr.items()}
    sc = O.Scene.from_arrays(**scene)
    oc = O.Camera.from_arrays(**cam)
    pix = [(x, y) for y in range(H) for x in range(W)]
    print(f"[case] loss gradients seed {seed} window {window}", flush=True)
    fd = O.fd_gradient(sc, [oc], window, [pix], [up.astype(np.float64)], depth_mode="median",
                       loss_weights=[wl.astype(np.float64)])
    for name in NAMES:
        ref, smooth = fd[name]
        got = gpu[name].reshape(ref.shape)
        m = smooth.astype(bool)
        rel = np.linalg.norm(got[m] - ref[m]) / max(np.linalg.norm(ref[m]), 1e-30)
        print(f"  {name}: rel err {rel:.2e} over {m.sum()} entries ({int((~m).sum())} excluded)")
        assert rel <= 1e-3, (name, rel)
