"""sof_render_bwd_static, the backward entry point that allocates nothing (its per-instance
partials live in the library's static per-device scratch), against sof_render_bwd with a
caller workspace: two calls in a row, the second on a smaller scene, so the second reads
scratch the first left behind.  The two backwards add the same partials in scheduling order
(LDS float atomics), so they agree to float rounding, not bitwise."""
import numpy as np
import pytest
import torch

from paper_2506_19139_amd import scenes, sof

pytestmark = pytest.mark.gpu


def _case(n, w, h, seed):
    scene = scenes.small_scene(n, seed=seed)
    cam = scenes.small_camera(w, h)
    g = sof.Gaussians.from_numpy(scene)
    C = sof.Cameras([cam])
    r = sof.Rasterizer(C, sof.Options(tile=16, window=8))
    out = r.forward(g)
    gen = torch.Generator(device="cuda").manual_seed(seed)
    P = C.n_pixels
    d_rgb = torch.randn(3 * P, device="cuda", generator=gen) / P
    d_acc = torch.randn(P, device="cuda", generator=gen) / P
    d_depth = torch.randn(P, device="cuda", generator=gen) / P
    d_nrm = torch.randn(3 * P, device="cuda", generator=gen) / P
    return r, g, C, out, (d_rgb, d_acc, d_depth, d_nrm)


def _static(r, g, C, out, ups):
    res = dict(means=torch.full_like(g.means, float("nan")), scales=torch.full_like(g.scales, float("nan")),
               quats=torch.full_like(g.quats, float("nan")), opac=torch.full_like(g.opac, float("nan")),
               sh=torch.full_like(g.sh, float("nan")))
    sof.render_bwd_static(g, C, r.opts, r.proj, r.bins, out["rgb"], out["normal"], out["aux"], *ups, res["means"],
                          res["scales"], res["quats"], res["opac"], res["sh"], order=out["order"])
    return res


def test_static_scratch_backward_matches_the_workspace_backward():
    for n, w, h, seed in ((1000, 64, 64, 0), (300, 40, 24, 1)):
        print(f"[case] static-scratch backward n={n} {w}x{h}", flush=True)
        r, g, C, out, ups = _case(n, w, h, seed)
        assert r.opts.capacity <= sof.STATIC_SCRATCH_INSTANCES
        got = _static(r, g, C, out, ups)
        ref = r.backward(g, out, *ups)
        torch.cuda.synchronize()
        for k in ("means", "scales", "quats", "opac", "sh"):
            a, b = got[k].cpu().numpy(), ref[k].cpu().numpy()
            assert np.all(np.isfinite(a)), k
            scale = max(float(np.abs(b).max()), 1e-30)
            err = float(np.abs(a - b).max()) / scale
            print(f"  {k}: max |static - workspace| / max |workspace| = {err:.2e}")
            assert err <= 1e-5, (k, err)


def test_static_scratch_rejects_a_capacity_above_its_size():
    r, g, C, out, ups = _case(300, 40, 24, 2)
    opts = sof.Options(**{**r.opts.__dict__, "capacity": sof.STATIC_SCRATCH_INSTANCES + 1})
    z = [torch.empty_like(t) for t in (g.means, g.scales, g.quats, g.opac, g.sh)]
    with pytest.raises(sof.SofError, match=r"\(-6\)"):
        sof.render_bwd_static(g, C, opts, r.proj, r.bins, out["rgb"], out["normal"], out["aux"], *ups, *z)
