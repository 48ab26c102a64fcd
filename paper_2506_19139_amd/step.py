"""Training-step runtime on top of the C ABI: fixed buffers, HIP-graph capture of the whole
step, and an autotuner for the launch configuration.

A step is project -> bin_sort -> render_fwd -> L1 loss gradient -> render_bwd for all the
cameras of one `Cameras` set (uneven resolutions share one grid through per-camera tile
offsets).  Every buffer is allocated before capture, the instance capacity is fixed (the
device status word reports an overflow), so the captured graph replays without any host
work.
"""
from __future__ import annotations

import json
import os
import time

import torch

from . import sof


class TrainStep:
    def __init__(self, g: sof.Gaussians, cams: sof.Cameras, opts: sof.Options, target: torch.Tensor,
                 extra_grads=None, capacity_margin=1.25):
        self.g, self.cams, self.opts = g, cams, opts
        self.target = target
        self.rast = sof.Rasterizer(cams, opts, auto_capacity=True)
        self.rast.prepare(g)
        opts.capacity = int(self.rast.last_count * capacity_margin) + 4096
        self.rast.auto_capacity = False
        self.rast._alloc(g.n)
        self.out = self.rast.alloc_outputs()
        self.grads = dict(means=torch.empty_like(g.means), scales=torch.empty_like(g.scales),
                          quats=torch.empty_like(g.quats), opac=torch.empty_like(g.opac), sh=torch.empty_like(g.sh))
        self.d_rgb = torch.empty_like(self.out["rgb"])
        self.extra = extra_grads or {}
        self.graph = None

    def run(self):
        r, o = self.rast, self.out
        sof.project(self.g, self.cams, self.opts, r.proj)
        sof.bin_sort(self.g.n, self.cams, self.opts, r.proj, r.bins)
        sof.render_fwd(self.g.n, self.cams, self.opts, r.proj, r.bins, o["rgb"], o["acc"], o["depth"], o["normal"],
                       o["aux"], order=o["order"])
        torch.sign(o["rgb"] - self.target, out=self.d_rgb)
        self.d_rgb.mul_(1.0 / self.d_rgb.numel())                         # d(mean |rgb - target|)
        r.backward(self.g, o, self.d_rgb, self.extra.get("acc"), self.extra.get("depth"), self.extra.get("normal"),
                   grads_out=self.grads)

    def capture(self, warmup=2):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(warmup):
                self.run()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.run()
        return self

    def replay(self):
        if self.graph is None:
            self.run()
        else:
            self.graph.replay()

    def status(self):
        return sof.read_status(self.rast.bins)


def _time(fn, reps=5, warmup=2):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


CACHE = os.path.join(os.path.expanduser("~"), ".cache", "sof_tune.json")


def autotune(g: sof.Gaussians, cams: sof.Cameras, target: torch.Tensor, window: int, tiles=(8, 16, 32),
             windows=None, reps=3, cache_path=CACHE, verbose=False):
    """Time a full training step for every tile size (and, if given, every window size) and
    return the fastest (tile, window, ms).  The tile size does not change any output (results
    are bit-identical across tile sizes); changing the window changes the approximation, so
    windows are only searched when the caller passes them.  Results are cached per
    (Gaussian count, camera sizes, window set)."""
    windows = tuple(windows) if windows else (window,)
    key = json.dumps([g.n, cams.sizes, list(tiles), list(windows)])
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except Exception:
            cache = {}
    if key in cache:
        return tuple(cache[key])
    best = None
    for w in windows:
        for t in tiles:
            if not (w in sof.WINDOWS and t in sof.TILES):
                continue
            if t == 32 and w > 8:       # 1024-lane workgroups cannot hold large windows without spilling
                continue
            st = TrainStep(g, cams, sof.Options(tile=t, window=w), target)
            ms = _time(st.run, reps=reps)
            if verbose:
                print(f"[tune] tile {t} window {w}: {ms:.3f} ms")
            if best is None or ms < best[2]:
                best = (t, w, ms)
            del st
            torch.cuda.empty_cache()
    if cache_path:
        try:
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            cache[key] = list(best)
            json.dump(cache, open(cache_path, "w"))
        except OSError:
            pass
    return best
