"""Shared helpers for the GPU parity tests: run the HIP path through the C ABI, run the
oracle on the same float32 inputs, and flag pixels whose result may legitimately differ
between a float32 and a float64 evaluation (near-ties and near-thresholds)."""
import numpy as np
import torch

from oracle import sof_oracle as O
from paper_2506_19139_amd import sof

TOL_ABS = 1e-4          # rgb / acc / normal, absolute
TOL_DEPTH_REL = 1e-4    # depth, relative


def gpu_render(scene, cams, tile=16, window=8, flags=0, bg=(0.0, 0.0, 0.0), capacity=0, auto_capacity=True):
    g = sof.Gaussians.from_numpy(scene)
    C = sof.Cameras(cams)
    opts = sof.Options(tile=tile, window=window, flags=flags, bg=bg, capacity=capacity)
    r = sof.Rasterizer(C, opts, auto_capacity=auto_capacity)
    out = r.forward(g)
    torch.cuda.synchronize()
    host = {k: v.cpu().numpy() for k, v in out.items()}
    return r, g, C, opts, out, host


def unpack(host, cams, idx=0):
    """Per-camera planar outputs of camera `idx` as [H*W, C] arrays (row-major pixels)."""
    off = 0
    for i, c in enumerate(cams):
        w, h = c["width"], c["height"]
        if i == idx:
            hw = w * h
            rgb = host["rgb"][3 * off:3 * off + 3 * hw].reshape(3, hw).T
            nrm = host["normal"][3 * off:3 * off + 3 * hw].reshape(3, hw).T
            A = sof.AUX_CHANNELS
            aux = host["aux"][A * off:A * off + A * hw].reshape(A, hw)
            return dict(rgb=rgb, acc=host["acc"][off:off + hw], depth=host["depth"][off:off + hw], normal=nrm,
                        T_end=aux[0], n_emitted=aux[1].view(np.int32), k=aux[2].view(np.int32), T_k=aux[3],
                        walked=aux[4].view(np.int32), cands=aux[5].view(np.int32))
        off += w * h
    raise IndexError(idx)


def oracle_scene_cam(scene, cam):
    return O.Scene.from_arrays(**scene), O.Camera.from_arrays(**cam)


def fragile(sc, v, px, py, res: "O.PixelResult"):
    """True if float32 vs float64 evaluation may flip a discrete decision at this pixel:
    two candidates with near-equal peak depth (|dt| <= 1e-5 t) or near-equal mean depth,
    an alpha within 1e-5 (relative) of 1/255, or a transmittance step within 1e-5 of the
    termination (1e-4) or crossing (0.5) thresholds."""
    c = O.pixel_candidates(sc, v, px, py)
    t = np.sort(c.tstar)
    if len(t) > 1 and np.any(np.diff(t) <= 1e-5 * t[1:]):
        return True
    z = np.sort(v.zkey32[c.idx].astype(np.float64))
    if len(z) > 1 and np.any(np.diff(z) <= 1e-6 * np.abs(z[1:])):
        return True
    # every Gaussian near the alpha cut, candidate or not
    d, dc = v.cam.pixel_ray(px, py)
    ids = np.nonzero(v.live)[0]
    A, B, C = O.ray_abc(v.prec[ids], sc.means[ids], v.cam.center, d)
    a = sc.opac[ids] * np.exp(-0.5 * np.maximum(0, C - B * B / (4 * A)))
    if np.any(np.abs(a - O.ALPHA_MIN) <= 1e-5 * O.ALPHA_MIN):
        return True
    # transmittance steps along the emitted sequence (+ the step that terminated it)
    Ts = [1.0]
    for w in res.weights:
        a_ = w / Ts[-1]
        Ts.append(Ts[-1] * (1 - a_))
    for Tn in Ts[1:]:
        if abs(Tn - 0.5) <= 1e-5 or abs(Tn - O.T_MIN) <= 1e-8:
            return True
    if len(res.order) < len(c.idx):
        # the next candidate would have crossed the termination threshold
        emitted = set(res.order)
        rest = [i for i in range(len(c.idx)) if int(c.idx[i]) not in emitted]
        for i in rest:
            if abs(Ts[-1] * (1 - c.alpha[i]) - O.T_MIN) <= 1e-8:
                return True
    return False


def depth_rounding_bound(sc, v, px, py, res: "O.PixelResult"):
    """Bound on the depth change caused by float32 rounding of T_k alone.

    depth = t*_k - S with S = sqrt(2 ln(G*_k / g) / A_k), g = (T_k - 1/2) / (T_k o_k), so
    d depth / d T_k = (1 / (S A_k)) (1 / (T_k - 1/2) - 1 / T_k).  Each factor (1 - alpha_j)
    of T_k carries a relative error of about 2^-23 + alpha_j eps / (1 - alpha_j), with
    eps = 4e-7 the relative error of a float32 alpha (exp2 and reciprocal approximations)."""
    if res.k < 0:
        return 0.0
    c = O.pixel_candidates(sc, v, px, py)
    i = int(np.nonzero(c.idx == res.k)[0][0])
    S = c.tstar[i] - res.depth
    if S <= 0:
        return 0.0
    sens = (1.0 / (S * c.A[i])) * abs(1.0 / (res.T_k - 0.5) - 1.0 / res.T_k)
    rank = res.order.index(res.k)
    rel = 0.0
    Tj = 1.0
    for w in res.weights[:rank]:
        a = w / Tj
        rel += 2.0 ** -23 + a * 4e-7 / (1.0 - a)
        Tj *= 1.0 - a
    dT = rel * res.T_k
    return sens * dT


def compare_images(gpu, orc, sc, v, pixels, check_depth=True):
    """Element-wise comparison; returns (n_bad, n_bad_unflagged, n_fragile, worst).

    A depth that misses the relative tolerance but lies within 4x the float32 rounding
    bound of `depth_rounding_bound` counts as fragile (ill-conditioned), not as a pass."""
    bad = bad_unflagged = n_frag = 0
    worst = dict(rgb=0.0, acc=0.0, normal=0.0, depth=0.0)
    for i, (px, py) in enumerate(pixels):
        gi = py * v.cam.width + px
        e_rgb = float(np.max(np.abs(gpu["rgb"][gi] - orc["rgb"][i])))
        e_acc = float(abs(gpu["acc"][gi] - orc["acc"][i]))
        e_nrm = float(np.max(np.abs(gpu["normal"][gi] - orc["normal"][i])))
        od = orc["depth"][i]
        e_dep = float(abs(gpu["depth"][gi] - od) / max(abs(od), 1e-12)) if (od != 0 or gpu["depth"][gi] != 0) else 0.0
        ok = e_rgb <= TOL_ABS and e_acc <= TOL_ABS and e_nrm <= TOL_ABS
        ok = ok and gpu["n_emitted"][gi] == orc["n_emitted"][i] and gpu["k"][gi] == orc["k"][i]
        if check_depth:
            ok = ok and e_dep <= TOL_DEPTH_REL
        if not ok:
            bad += 1
            res = orc["results"][i]
            int_ok = gpu["n_emitted"][gi] == orc["n_emitted"][i] and gpu["k"][gi] == orc["k"][i]
            only_depth = int_ok and e_rgb <= TOL_ABS and e_acc <= TOL_ABS and e_nrm <= TOL_ABS
            ill = only_depth and abs(gpu["depth"][gi] - od) <= 4.0 * depth_rounding_bound(sc, v, px, py, res)
            if ill or fragile(sc, v, px, py, res):
                n_frag += 1
            else:
                bad_unflagged += 1
                for k_, e in (("rgb", e_rgb), ("acc", e_acc), ("normal", e_nrm), ("depth", e_dep)):
                    worst[k_] = max(worst[k_], e)
    return bad, bad_unflagged, n_frag, worst
