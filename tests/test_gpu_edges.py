"""Degenerate inputs of the optional terms: no Gaussians, pixels without a crossing, no
cameras for the 3D filter, empty edge sets."""
import numpy as np
import pytest
import torch

from paper_2506_19139_amd import scenes, sof

pytestmark = pytest.mark.gpu


def test_empty_scene_gives_zero_losses_and_opacity():
    scene = scenes.subset_scene(scenes.small_scene(10, seed=1), np.arange(0))
    cam = scenes.small_camera(32, 32)
    g = sof.Gaussians.from_numpy(scene)
    r = sof.Rasterizer(sof.Cameras([cam]), sof.Options(tile=16, window=8))
    out = r.forward(g, losses=True)
    opa = r.opacity(g, out)
    d = torch.ones(2 * 32 * 32, device="cuda")
    gr = r.backward(g, out, d_rgb=torch.ones_like(out["rgb"]), d_opa=torch.ones_like(opa), d_losses=d)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out["losses"].view(sof.LOSS_CHANNELS, -1)[:2]).item() == 0
    assert torch.count_nonzero(opa).item() == 0
    assert all(v.numel() == 0 for v in gr.values())


def test_opacity_is_zero_where_no_crossing():
    scene = scenes.small_scene(200, seed=3)
    scene["opac"] = np.full_like(scene["opac"], 0.3)          # no pixel can reach T <= 1/2 with few layers
    cam = scenes.small_camera(48, 48)
    g = sof.Gaussians.from_numpy(scene)
    r = sof.Rasterizer(sof.Cameras([cam]), sof.Options(tile=8, window=4))
    out = r.forward(g)
    opa = r.opacity(g, out).cpu().numpy()
    k = out["aux"].view(sof.AUX_CHANNELS, -1)[2].view(torch.int32).cpu().numpy()
    assert np.all(opa[k < 0] == 0.0)
    assert np.all((opa[k >= 0] > 0.0) & (opa[k >= 0] < 1.0))


def test_filter3d_without_cameras_is_the_identity():
    scene = scenes.small_scene(100, seed=4)
    g = sof.Gaussians.from_numpy(scene)
    gf, var = sof.filter3d(g, None)
    torch.cuda.synchronize()
    assert torch.count_nonzero(var).item() == 0
    assert torch.equal(gf.scales, g.scales) and torch.equal(gf.opac, g.opac)


def test_bisection_with_no_edges():
    a = torch.empty(0, 3, device="cuda")
    sof.bisect_step(a, a.clone(), a.clone())
    search = sof.LevelSetSearch(sof.Cameras([scenes.small_camera(32, 32)]), tile=8)
    g = sof.Gaussians.from_numpy(scenes.small_scene(50, seed=5))
    out = search(g, a.clone(), a.clone(), steps=8)
    assert out.shape == (0, 3)
