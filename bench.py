#!/usr/bin/env python
"""Benchmark of the Sorted Opacity Fields hot path on one MI355X.  Prints ONE JSON line.

Headline (`value`): one training step (project -> bin_sort -> render_fwd -> L1 loss
gradient -> render_bwd) at 1M Gaussians (unbounded recipe: 70 % in a 10 m box, 30 %
background at 10..1000 m, SH degree 3) rendered at 1920x1080 with depth and normal outputs,
in ms per iteration.  Inputs are resident in HBM before timing starts.

Also reported: batched opacity-field queries (3M Gaussians, 27M points = centres + 3-sigma
box corners, min over 96 views of 960x540, one persistent launch) in points/s; the
roofline of the dominant kernel (algorithmic work / measured kernel time); and the FP64
oracle timed on the host cores on a bounded sample of the same frame.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd ms/iter at 1M Gaussians 1080p; opacity queries/s; % HBM roofline"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3       # 256 CUs x 128 FP32 FMA lanes/clk (packed) x 2 x 2.4 GHz

# Algorithmic FP32 work per unit of the rasteriser (the flops the method needs, counted from
# its formulas; the window, exec-mask, address and reduction instructions are not counted):
FLOP_EVAL = 23      # quadric of one (pixel, list entry): offsets, b', c', den', n', cut test
FLOP_CAND = 9       # candidate: z test, reciprocal, exponent, alpha, key
FLOP_BLEND = 15     # one blended Gaussian: transmittance, weight, colour and normal sums
FLOP_ADJ = 110      # one blended Gaussian in the backward: dalpha, chain to (mu_c, P_c), partials
# (the backward's own share of the candidate test and window is FLOP_EVAL / FLOP_CAND again
# when it replays the order; with the order the forward recorded it has none)


# Counter figures (HBM bytes, vector and LDS instructions) are taken with rocprofv3 over this
# benchmark and written by `bench.py --summarize` into the profile summaries below (the training
# step alone, then the query workload), one line per kernel with the hash of the sources the
# kernel is built from.  The bench line reports a kernel's counter figures only while its
# sources still hash to that value and the workload is the default one; a changed source needs
# a new measurement.  A kernel in both summaries takes the step's line (its launches there are
# all of the step's size).
PROFILES = [os.path.join(ROOT, "profiles", "query_3M_27M_counters.txt"),
            os.path.join(ROOT, "profiles", "step_1M_1080p_counters.txt")]
CSRC = os.path.join(ROOT, "paper_2506_19139_amd", "csrc")
VALU_CYCLES = 4                     # a wave64 vector instruction holds a 16-lane SIMD for 4 cycles
N_SIMDS, CLOCK_GHZ = 1024, 2.4      # 256 CUs x 4 SIMDs


def kernel_short_name(full):
    """`void sof::k_render_bwd<16, 8, false>(sof::RenderBwdArgs)` -> `k_render_bwd<16, 8, false>`."""
    n = full.split("(")[0]
    n = n.split("sof::")[-1] if "sof::" in n else n.split()[-1]
    return n.strip()


def kernel_source_file(short):
    """The .hip file of csrc that defines the kernel (None for kernels from other libraries)."""
    import re
    base = short.split("<")[0]
    for f in sorted(os.listdir(CSRC)):
        if f.endswith(".hip") and re.search(r"void\s+" + re.escape(base) + r"\s*\(", open(os.path.join(CSRC, f)).read()):
            return f
    return None


def kernel_source_hash(short):
    """Hash of the kernel's .hip file, every header of csrc and the public header."""
    import hashlib
    f = kernel_source_file(short)
    if f is None:
        return None
    h = hashlib.sha256()
    for name in [f] + sorted(x for x in os.listdir(CSRC) if x.endswith(".h")):
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, "include", "sof.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def read_profile(path=None):
    """Per-kernel records of a profile summary (lines `kernel=... src=... key=value ...`); with
    no path, of the default summaries (a later file's line replaces an earlier one's)."""
    rec = {}
    for pth in ([path] if path else PROFILES):
        if not os.path.exists(pth):
            continue
        for line in open(pth):
            if not line.startswith("kernel="):
                continue
            fields = dict(tok.split("=", 1) for tok in line.strip().split("\t"))
            rec[fields["kernel"]] = fields
    return rec


def counter_figures(short, args, profile=None):
    """Counter figures of one kernel from the profile, or None when they do not apply (another
    workload, or sources changed since they were taken)."""
    default = (args.n, args.tile, args.window) == (1_000_000, 16, 8)
    rec = (profile if profile is not None else read_profile()).get(short)
    if not default or not rec or rec.get("src") != kernel_source_hash(short):
        return None
    return rec


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--window", type=int, default=8)
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--query-gaussians", type=int, default=3_000_000)
    ap.add_argument("--query-steps", type=int, default=2)
    ap.add_argument("--no-query", action="store_true")
    ap.add_argument("--query-tile", type=int, default=8)
    ap.add_argument("--no-per-view", action="store_true",
                    help="skip the comparison against one query launch per view")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph-step", action="store_true",
                    help="skip the headline step replayed as one captured HIP graph")
    ap.add_argument("--no-window-sweep", action="store_true",
                    help="skip the headline step at resort windows 4, 8 and 16")
    ap.add_argument("--no-opacity-term", action="store_true",
                    help="skip the training step with the distortion, extent and opacity-at-depth terms")
    ap.add_argument("--no-levelset", action="store_true",
                    help="skip the level-set query and the binary search")
    ap.add_argument("--no-multiview", action="store_true",
                    help="skip the 8-camera graph-captured training step")
    ap.add_argument("--cpu-pixels", type=int, default=512)
    ap.add_argument("--cpu-query-points", type=int, default=4)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device copy of this many MiB first (scale reference for HBM byte counters)")
    ap.add_argument("--no-peaks", action="store_true", help="skip the measured copy and FMA peaks")
    ap.add_argument("--summarize", default=None,
                    help="write a profile summary to this file from --trace-db/--read-db/--write-db/--sq-db and exit")
    ap.add_argument("--trace-db")
    ap.add_argument("--read-db")
    ap.add_argument("--write-db")
    ap.add_argument("--sq-db")
    ap.add_argument("--header", default="", help="text put at the top of the summary (\\n for new lines)")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# --------------------------------------------------------------------------- profile summary

READ_COUNTERS = ("TCC_EA0_RDREQ", "TCC_EA0_RDREQ_32B", "TCC_EA0_RDREQ_64B", "TCC_EA0_RDREQ_128B")
WRITE_COUNTERS = ("TCC_EA0_WRREQ", "TCC_EA0_WRREQ_64B")
SQ_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT",
               "SQ_INSTS_VMEM", "SQ_BUSY_CYCLES", "SQ_WAIT_INST_LDS")


def _db_trace(db):
    import sqlite3
    import collections
    cur = sqlite3.connect(db).cursor()
    out = collections.defaultdict(list)
    for name, t0, t1 in cur.execute("select name, start, end from kernels"):
        out[kernel_short_name(name)].append((t1 - t0) / 1e3)
    return out


def _db_counters(db):
    import sqlite3
    import collections
    cur = sqlite3.connect(db).cursor()
    out = collections.defaultdict(lambda: collections.defaultdict(list))
    for name, counter, value in cur.execute("select kernel_name, counter_name, value from counters_collection"):
        out[kernel_short_name(name)][counter].append(float(value))
    return out


def summarize(args):
    """Write the profile summary from the rocprofv3 databases of this benchmark: one kernel trace
    and three counter passes (read requests by size, write requests by size, SQ instruction
    counts).  HBM bytes are counted from request sizes (32 x 32B + 64 x 64B + 128 x 128B reads,
    32 / 64 B writes) and checked against a streaming copy of known size run in the same passes."""
    trace = _db_trace(args.trace_db)
    rd, wr, sq = _db_counters(args.read_db), _db_counters(args.write_db), _db_counters(args.sq_db)
    avg = lambda v: sum(v) / len(v) if v else 0.0

    def read_bytes(c):
        return (32 * avg(c.get("TCC_EA0_RDREQ_32B", [])) + 64 * avg(c.get("TCC_EA0_RDREQ_64B", []))
                + 128 * avg(c.get("TCC_EA0_RDREQ_128B", [])))

    def write_bytes(c):
        n, n64 = avg(c.get("TCC_EA0_WRREQ", [])), avg(c.get("TCC_EA0_WRREQ_64B", []))
        return 64 * n64 + 32 * (n - n64)
    copy_bytes = args.calib_copy_mib * (1 << 20)
    cal_r = read_bytes(rd["k_peak_copy"]) / copy_bytes if "k_peak_copy" in rd else None
    cal_w = write_bytes(wr["k_peak_copy"]) / copy_bytes if "k_peak_copy" in wr else None
    lines = []
    for k in sorted(trace, key=lambda k: -sum(trace[k])):
        src = kernel_source_hash(k)
        if src is None or k.startswith("k_peak"):
            continue
        t = avg(trace[k])
        rb, wb = read_bytes(rd.get(k, {})), write_bytes(wr.get(k, {}))
        c = sq.get(k, {})
        valu = avg(c.get("SQ_INSTS_VALU", []))
        issue_us = valu * VALU_CYCLES / (N_SIMDS * CLOCK_GHZ * 1e9) * 1e6
        f = {"kernel": k, "src": src, "calls": len(trace[k]), "avg_us": f"{t:.2f}", "read_bytes": f"{rb:.0f}",
             "write_bytes": f"{wb:.0f}", "GBps": f"{(rb + wb) / (t * 1e-6) / 1e9:.1f}",
             "hbm_frac": f"{(rb + wb) / (t * 1e-6) / (HBM_PEAK_GBS * 1e9):.4f}",
             "valu": f"{valu:.4g}", "salu": f"{avg(c.get('SQ_INSTS_SALU', [])):.4g}",
             "lds": f"{avg(c.get('SQ_INSTS_LDS', [])):.4g}",
             "lds_bank_conflict": f"{avg(c.get('SQ_LDS_BANK_CONFLICT', [])):.4g}",
             "valu_issue_us": f"{issue_us:.2f}", "issue_frac": f"{issue_us / t:.3f}"}
        lines.append("\t".join(f"{a}={b}" for a, b in f.items()))
    with open(args.summarize, "w") as fh:
        fh.write(args.header.replace("\\n", "\n") + "\n" if args.header else "")
        fh.write(f"calibration: streaming copy of {copy_bytes} bytes read as {cal_r:.4f} x its size (reads) and "
                 f"{cal_w:.4f} x (writes) by the request-size counts; bytes below are the counts, unscaled\n"
                 if cal_r is not None and cal_w is not None else "calibration: no copy in the counter passes\n")
        fh.write("fields: avg_us = kernel-trace average duration; read/write_bytes per dispatch from TCC_EA0 "
                 "request counts by size; GBps and hbm_frac (of 8 TB/s) over avg_us; valu/salu/lds = SQ_INSTS_* "
                 "wave instructions per dispatch; lds_bank_conflict = SQ_LDS_BANK_CONFLICT cycles; valu_issue_us "
                 "= valu x 4 cycles / (1024 SIMDs x 2.4 GHz) and issue_frac its share of avg_us; src = hash of the "
                 "kernel's sources (bench.py kernel_source_hash)\n")
        for l in lines:
            fh.write(l + "\n")
    print(f"wrote {args.summarize}: {len(lines)} kernels", file=sys.stderr)


# --------------------------------------------------------------------------- CPU oracle

_CPU = {}


def _oracle_view_chunk(ids):
    """Camera view of a chunk of the scene's Gaussians (colours, normals, precisions)."""
    from oracle import sof_oracle as O
    from paper_2506_19139_amd import scenes
    sc = O.Scene.from_arrays(**scenes.subset_scene(_CPU["scene"], ids))
    v = O.view(sc, _CPU["ocam"])
    return v.live, v.prec, v.zkey32, v.color, v.normal


def _oracle_pixel(px_py):
    from oracle import sof_oracle as O
    r = O.render_pixel(_CPU["sc"], _CPU["v"], px_py[0], px_py[1], _CPU["window"])
    return r.acc


def _oracle_query_chunk(ids):
    """prod (1 - alpha_i(x)) over a chunk of the Gaussians for every (sampled point, view), and
    whether the view sees the point: the opacity field factorises over Gaussians (App. A.2)."""
    from oracle import sof_oracle as O
    from paper_2506_19139_amd import scenes
    sc = O.Scene.from_arrays(**scenes.subset_scene(_CPU["qscene"], ids))
    views = O.views_geometry(sc, _CPU["qcams"])
    pts = _CPU["qpts"]
    prod = np.ones((len(pts), len(views)))
    for i, x in enumerate(pts):
        for j, v in enumerate(views):
            _, alpha = O.view_alphas(sc, v, x)
            prod[i, j] = float(np.prod(1.0 - alpha))
    return prod


def cpu_baseline(scene, cam, window, n_pixels, qscene=None, qcams=None, qpts=None, n_query_total=0):
    """The oracle as it stands, on the host cores, on bounded samples of the two workloads.

    Render: the camera view of all N Gaussians (computed in Gaussian chunks, one per process),
    then `n_pixels` random pixels of the frame by brute force over all N, one per process;
    extrapolated linearly to the full frame.  Query: the sampled points against all Gaussians
    and all views, the product over Gaussians split into chunks (one per process) and combined,
    then the minimum over the views that see each point; extrapolated to all points."""
    import multiprocessing as mp
    from oracle import sof_oracle as O
    cores = len(os.sched_getaffinity(0))
    workers = max(1, min(cores, 15))
    ctx = mp.get_context("fork")
    n = scene["means"].shape[0]
    chunks = np.array_split(np.arange(n), workers)
    oc = O.Camera.from_arrays(**cam)
    _CPU.update(scene=scene, ocam=oc, window=window)
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        parts = pool.map(_oracle_view_chunk, chunks)
    v = O.CameraView(oc, *(np.concatenate([p[k] for p in parts]) for k in range(5)))
    t_setup = time.perf_counter() - t0
    log(f"cpu baseline: view of {n} Gaussians in {t_setup:.1f} s")
    _CPU.update(sc=O.Scene.from_arrays(**scene), v=v)
    rng = np.random.default_rng(0)
    pix = [(int(x), int(y)) for x, y in zip(rng.integers(0, cam["width"], n_pixels), rng.integers(0, cam["height"], n_pixels))]
    t1 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        pool.map(_oracle_pixel, pix, chunksize=max(1, n_pixels // (4 * workers)))
    t_pix = time.perf_counter() - t1
    log(f"cpu baseline: {n_pixels} pixels in {t_pix:.1f} s")
    full = cam["width"] * cam["height"]
    ms = (t_setup + full * t_pix / n_pixels) * 1e3
    res = {"value": round(ms, 1), "unit": "ms/iter (forward render only, extrapolated)", "cores": workers,
           "kind": "oracle", "pixels_per_s": round(n_pixels / t_pix, 3),
           "sample": f"render: camera view of all {n} Gaussians ({t_setup:.1f} s, chunked over {workers} processes) "
                     f"and {n_pixels} random pixels of the 1920x1080 frame by float64 brute force over all of them "
                     f"({n_pixels / t_pix:.2f} px/s on {workers} processes), extrapolated linearly to the {full} "
                     f"pixels; no backward (the oracle's gradient is finite differences)"}
    if qscene is None:
        return res
    # query sample
    qcams_o = [O.Camera.from_arrays(**c) for c in qcams]
    _CPU.update(qscene=qscene, qcams=qcams_o, qpts=np.asarray(qpts, np.float64))
    nq = qscene["means"].shape[0]
    t2 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        prods = pool.map(_oracle_query_chunk, np.array_split(np.arange(nq), workers))
    prod = np.prod(np.stack(prods), axis=0)
    O_pts = [min([1.0] + [1.0 - prod[i, j] for j, c in enumerate(qcams_o) if O.point_view_valid(c, x)])
             for i, x in enumerate(_CPU["qpts"])]
    t_q = time.perf_counter() - t2
    log(f"cpu baseline: {len(qpts)} query points in {t_q:.1f} s")
    pts_per_s = len(qpts) / t_q
    for k in ("scene", "sc", "v", "qscene", "qpts"):
        _CPU.pop(k, None)
    res["sample"] += (f"; query: {len(qpts)} of the points against all {nq} Gaussians and {len(qcams)} views "
                      f"({t_q:.1f} s, the product over Gaussians split over {workers} processes), extrapolated to "
                      f"all {n_query_total} points")
    res["query_points_per_s"] = round(pts_per_s, 4)
    res["query_ms_extrapolated"] = round(n_query_total / pts_per_s * 1e3, 1)
    res["query_sample_opacity"] = [round(float(o), 7) for o in O_pts]
    return res


def per_view_query(qg, pts, qcams, tile, batched, t_batched, stream):
    """The same query as one launch per view: 96 single-camera calls (buffers sized by an
    untimed pass, then fixed), each followed by a running minimum on the device."""
    import torch
    from paper_2506_19139_amd import sof
    views = [sof.Cameras([c]) for c in qcams.list]
    q = sof.OpacityQuery(views[0], sof.Options(tile=tile))
    out = torch.empty_like(batched)
    acc = torch.empty_like(batched)
    for v in views:                                   # sizing pass (host read-backs)
        q.cams = v
        q(qg, pts, out=out)
    q.auto_capacity = False
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    acc.fill_(1.0)
    for v in views:
        q.cams = v
        q(qg, pts, out=out)
        torch.minimum(acc, out, out=acc)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    diff = (acc - batched).abs().max().item()
    return {"ms": round(ms, 2), "points_per_s": round(pts.shape[0] / (ms * 1e-3), 1),
            "batched_speedup": round(ms / t_batched, 3), "max_abs_diff_vs_batched": diff}


def multiview_step(g, stream, reps=10):
    """Eight cameras of uneven resolution (640x360 .. 1920x1080) in one training step: the
    tile size (and, separately, the window) picked by the autotuner, then the whole step
    (project, bin_sort, render_fwd, L1 gradient, render_bwd) captured in one HIP graph."""
    import torch
    from paper_2506_19139_amd import scenes, sof, step
    cams = sof.Cameras(scenes.multiview_cameras())
    target = torch.from_numpy(np.concatenate([scenes.target_image(h, w, seed=1 + k).reshape(-1)
                                              for k, (w, h) in enumerate(scenes.MULTIVIEW_SIZES)])).cuda()
    tile8 = step.autotune(g, cams, target, window=8, tiles=(8, 16, 32), cache_path=None)
    full = step.autotune(g, cams, target, window=8, tiles=(8, 16, 32), windows=(4, 8, 16), cache_path=None)
    st = step.TrainStep(g, cams, sof.Options(tile=tile8[0], window=8), target).capture()
    for _ in range(2):
        st.replay()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        st.replay()
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    k_used, flags = st.status()
    assert flags == 0, "instance capacity exceeded in the captured step"
    return {"workload": f"{g.n} Gaussians, 8 cameras " + ", ".join(f"{w}x{h}" for w, h in scenes.MULTIVIEW_SIZES)
                        + f" ({cams.n_pixels / 1e6:.2f} Mpx), fwd+bwd, L1, one HIP graph",
            "window": 8, "tile": tile8[0], "graph_ms": round(ms, 3),
            "mpx_per_s": round(cams.n_pixels / (ms * 1e-3) / 1e6, 1), "instances": int(k_used),
            "tuner_window8_ms": round(tile8[2], 3),
            "tuner_over_tile_and_window": {"tile": full[0], "window": full[1], "ms": round(full[2], 3)}}


def graph_step(g, C, tile, window, target, d_acc, d_depth, d_normal, stream, reps=10):
    """The headline step (same scene, camera, upstream gradients) captured once in a HIP graph
    and replayed: what a training loop that replays the step pays per iteration."""
    import torch
    from paper_2506_19139_amd import sof, step
    st = step.TrainStep(g, C, sof.Options(tile=tile, window=window), target,
                        extra_grads=dict(acc=d_acc, depth=d_depth, normal=d_normal)).capture()
    for _ in range(2):
        st.replay()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        st.replay()
    b.record(stream)
    torch.cuda.synchronize()
    k_used, flags = st.status()
    assert flags == 0, "instance capacity exceeded in the captured step"
    ms = a.elapsed_time(b) / reps
    del st
    return round(ms, 4)


def levelset_search(qg, pts, qcams, tile, t_exact, stream, steps=8):
    """The query in level-set mode (only O > 0.5 or not) over the same 27M points, then eight
    binary-search steps on edges from each Gaussian's centre to one of its 3-sigma box corners
    that cross the level set (synthetic stand-ins for the edges of a tetrahedral grid)."""
    import torch
    from paper_2506_19139_amd import sof
    search = sof.LevelSetSearch(qcams, tile=tile)
    o = search.query(qg, pts)
    search.query.auto_capacity = False
    times = []
    for _ in range(2):
        a_, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a_.record(stream)
        search.query(qg, pts, out=o)
        b_.record(stream)
        torch.cuda.synchronize()
        times.append(a_.elapsed_time(b_))
    tl = float(np.median(times))
    n = pts.shape[0] // 9
    ins = (o > 0.5).view(n, 9)
    corner = 1 + torch.arange(n, device=pts.device) % 8
    p9 = pts.view(n, 9, 3)
    keep = ins[:, 0] != ins[torch.arange(n, device=pts.device), corner]
    cen, cor = p9[keep, 0], p9[torch.nonzero(keep).squeeze(1), corner[keep]]
    cin = ins[keep, 0]
    a = torch.where(cin[:, None], cen, cor).contiguous()
    b = torch.where(cin[:, None], cor, cen).contiguous()
    search.query.pv_capacity = 0                         # new point set: size the pair buffers again
    search.query.auto_capacity = True
    a1, b1 = a.clone(), b.clone()
    search(qg, a1, b1, steps=1)                          # sizing pass
    search.query.auto_capacity = False
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    search(qg, a, b, steps=steps)
    e1.record(stream)
    torch.cuda.synchronize()
    tb = e0.elapsed_time(e1)
    return {"query_ms": round(tl, 2), "points_per_s": round(pts.shape[0] / (tl * 1e-3), 1),
            "speedup_vs_exact": round(t_exact / tl, 2), "inside_fraction": round(float((o > 0.5).float().mean()), 4),
            "bisection": {"edges": int(a.shape[0]), "steps": steps, "ms": round(tb, 2),
                          "ms_per_step": round(tb / steps, 2)}}


def opacity_term_step(g, C, opts, rast, out, grads, target, d_acc, d_depth, d_normal, stream, steps):
    """The headline step plus the paper's rasteriser-side training terms: the distortion and
    extent losses computed in the forward, the second pass that evaluates the opacity field at
    each pixel's rendered depth, and the backward with all their gradients (upstream 2 lambda
    (O_N - 0.5) / P with lambda = 0.04, and lambda_ext = 0.1 and a distortion weight of 1000 /
    P, the order of magnitude GOF uses)."""
    import torch
    from paper_2506_19139_amd import sof
    timer = sof.KernelTimer()
    t_opa, t_step = [], []
    P = C.n_pixels
    out["losses"] = torch.empty(sof.LOSS_CHANNELS * P, device=out["rgb"].device)
    d_losses = torch.cat([torch.full((P,), 1000.0 / P, device=out["rgb"].device),
                          torch.full((P,), 0.1 / P, device=out["rgb"].device)])

    def step(record):
        a = [torch.cuda.Event(enable_timing=True) for _ in range(4)] if record else None
        if record: a[0].record(stream)
        sof.project(g, C, opts, rast.proj)
        sof.bin_sort(g.n, C, opts, rast.proj, rast.bins)
        sof.render_fwd(g.n, C, opts, rast.proj, rast.bins, out["rgb"], out["acc"], out["depth"], out["normal"],
                       out["aux"], out["losses"], order=out["order"])
        if record: a[1].record(stream)
        opa = rast.opacity(g, out)
        if record: a[2].record(stream)
        d_rgb = torch.sign(out["rgb"] - target) * (1.0 / out["rgb"].numel())
        d_opa = (opa - 0.5) * (2.0 * 0.04 / opa.numel())
        rast.backward(g, out, d_rgb, d_acc, d_depth, d_normal, grads_out=grads, d_opa=d_opa, d_losses=d_losses)
        if record:
            a[3].record(stream)
            t_opa.append((a[1], a[2]))
            t_step.append((a[0], a[3]))

    for _ in range(2):
        step(False)
    torch.cuda.synchronize()
    for _ in range(steps):
        with timer:
            step(True)
    torch.cuda.synchronize()
    ms = lambda v: float(np.mean([x.elapsed_time(y) for x, y in v]))
    return {"k_render_fwd_ms": round(float(np.mean(timer.ms("render_fwd"))), 4),
            "opacity_pass_ms": round(ms(t_opa), 4), "k_render_bwd_ms": round(float(np.mean(timer.ms("render_bwd"))), 4),
            "step_ms": round(ms(t_step), 4),
            "workload": "headline step + distortion and extent losses + opacity at the rendered depth, "
                        "with all their gradients"}


def window_sweep(g, C, capacity, target, d_acc, d_depth, d_normal, stream, steps, tile, windows=(4, 8, 16)):
    """The headline step (project, bin_sort, forward, L1 gradient, backward) at each resort
    window of the sweep, same scene, camera and instance capacity; kernel times from the
    library's HIP events, step time from stream events."""
    import torch
    from paper_2506_19139_amd import sof
    res = {}
    for w in windows:
        opts = sof.Options(tile=tile, window=w, capacity=capacity)
        r = sof.Rasterizer(C, opts)
        r.auto_capacity = False
        r._alloc(g.n)
        o = r.alloc_outputs()
        gr = dict(means=torch.empty_like(g.means), scales=torch.empty_like(g.scales), quats=torch.empty_like(g.quats),
                  opac=torch.empty_like(g.opac), sh=torch.empty_like(g.sh))
        timer = sof.KernelTimer()
        t_step = []

        def step(record):
            a = [torch.cuda.Event(enable_timing=True) for _ in range(2)] if record else None
            if record: a[0].record(stream)
            sof.project(g, C, opts, r.proj)
            sof.bin_sort(g.n, C, opts, r.proj, r.bins)
            sof.render_fwd(g.n, C, opts, r.proj, r.bins, o["rgb"], o["acc"], o["depth"], o["normal"], o["aux"],
                           order=o["order"])
            d_rgb = torch.sign(o["rgb"] - target) * (1.0 / o["rgb"].numel())
            r.backward(g, o, d_rgb, d_acc, d_depth, d_normal, grads_out=gr)
            if record:
                a[1].record(stream)
                t_step.append((a[0], a[1]))

        for _ in range(2):
            step(False)
        torch.cuda.synchronize()
        for _ in range(steps):
            with timer:
                step(True)
        torch.cuda.synchronize()
        k_used, flags = sof.read_status(r.bins)
        assert flags == 0 and k_used <= capacity, "instance capacity exceeded"
        n_emit = o["aux"].view(sof.AUX_CHANNELS, C.n_pixels)[1].view(torch.int32).double().sum().item()
        res[str(w)] = {"step_ms": round(float(np.mean([x.elapsed_time(y) for x, y in t_step])), 4),
                       "k_render_fwd_ms": round(float(np.mean(timer.ms("render_fwd"))), 4),
                       "k_render_bwd_ms": round(float(np.mean(timer.ms("render_bwd"))), 4),
                       "blended_per_pixel": round(n_emit / C.n_pixels, 2)}
        del r, o, gr
    return res


# --------------------------------------------------------------------------- GPU

def main():
    args = parse()
    if args.summarize:
        summarize(args)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU path is design-only.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2506_19139_amd import scenes, sof

    torch.cuda.set_device(0)
    if args.calib_copy_mib > 0:                  # reference for the byte counters: a copy of known size
        n4 = args.calib_copy_mib * (1 << 20) // 16
        src = torch.ones(4 * n4, device="cuda")
        dst = torch.empty_like(src)
        assert sof.lib().sof_bench_copy(sof._ptr(src), sof._ptr(dst), n4, sof._stream()) == 0
        torch.cuda.synchronize()
        del src, dst
    peaks = None if args.no_peaks else sof.measure_peaks()
    log("scene: unbounded 1M")
    scene = scenes.unbounded_scene(args.n, seed=0)
    cam = scenes.circle_camera(0.0, 1920, 1080)
    g = sof.Gaussians.from_numpy(scene)
    C = sof.Cameras([cam])
    opts = sof.Options(tile=args.tile, window=args.window)
    rast = sof.Rasterizer(C, opts)
    H, W = cam["height"], cam["width"]
    P = H * W
    target = torch.from_numpy(scenes.target_image(H, W, seed=1).reshape(-1)).cuda()
    up = np.random.default_rng(2).normal(0.0, 1.0, (5, P)).astype(np.float32) / P
    d_acc = torch.from_numpy(up[0]).cuda()
    d_depth = torch.from_numpy(up[1]).cuda()
    d_normal = torch.from_numpy(up[2:5].reshape(-1)).cuda()

    # capacity from one counted pass (+25 %), then fixed: no host read-back while timing
    rast.prepare(g)
    opts.capacity = int(rast.last_count * 1.25) + 4096
    rast.auto_capacity = False
    rast._alloc(g.n)
    out = rast.alloc_outputs()
    grads = dict(means=torch.empty_like(g.means), scales=torch.empty_like(g.scales), quats=torch.empty_like(g.quats),
                 opac=torch.empty_like(g.opac), sh=torch.empty_like(g.sh))
    stream = torch.cuda.current_stream()
    ev = {k: [] for k in ("project", "bin_sort", "render_fwd_call", "render_bwd_call")}
    timer = sof.KernelTimer()

    def step(record):
        marks = [torch.cuda.Event(enable_timing=True) for _ in range(6)] if record else None
        if record: marks[0].record(stream)
        sof.project(g, C, opts, rast.proj)
        if record: marks[1].record(stream)
        sof.bin_sort(g.n, C, opts, rast.proj, rast.bins)
        if record: marks[2].record(stream)
        sof.render_fwd(g.n, C, opts, rast.proj, rast.bins, out["rgb"], out["acc"], out["depth"], out["normal"],
                       out["aux"], order=out["order"])
        if record: marks[3].record(stream)
        d_rgb = torch.sign(out["rgb"] - target) * (1.0 / out["rgb"].numel())       # L1 loss gradient
        if record: marks[4].record(stream)
        rast.backward(g, out, d_rgb, d_acc, d_depth, d_normal, grads_out=grads)
        if record: marks[5].record(stream)
        if record:
            for k, (a, b) in zip(ev, ((0, 1), (1, 2), (2, 3), (4, 5))):
                ev[k].append((marks[a], marks[b]))

    log("warmup")
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    k_used, flags = sof.read_status(rast.bins)
    assert flags == 0 and k_used <= opts.capacity, "instance capacity exceeded"
    log("timed", args.steps, "steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        with timer:                        # HIP events around the two rasteriser kernels
            step(True)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps * 1e3
    per = {k: float(np.mean([a.elapsed_time(b) for a, b in v])) for k, v in ev.items()}
    kern = {k: float(np.mean(timer.ms(k))) for k in ("render_fwd", "render_bwd")}
    per["k_render_fwd"], per["k_render_bwd"] = kern["render_fwd"], kern["render_bwd"]

    aux = out["aux"].view(sof.AUX_CHANNELS, P)
    n_emit = aux[1].view(torch.int32).double().sum().item()
    walked = aux[4].view(torch.int32).double().sum().item()
    cands = aux[5].view(torch.int32).double().sum().item()
    recorded = out.get("order") is not None       # the backward reads the forward's order
    fwd_flops = FLOP_EVAL * walked + FLOP_CAND * cands + FLOP_BLEND * n_emit
    bwd_flops = FLOP_ADJ * n_emit + (0 if recorded else FLOP_EVAL * walked + FLOP_CAND * cands)
    dominant = "render_bwd" if kern["render_bwd"] >= kern["render_fwd"] else "render_fwd"
    flops = bwd_flops if dominant == "render_bwd" else fwd_flops
    achieved = flops / (kern[dominant] * 1e-3) / 1e12
    profile = read_profile()
    if dominant == "render_bwd":
        dom_short = (f"k_render_bwd<{args.tile}, 0, false, true>" if recorded
                     else f"k_render_bwd<{args.tile}, {args.window}, false, false>")
    else:
        dom_short = f"k_render_fwd<{args.tile}, {args.window}, 0>"
    cf = counter_figures(dom_short, args, profile)
    roofline = {"bound": "alu", "kernel": dom_short, "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                "traffic": (int(float(cf["read_bytes"]) + float(cf["write_bytes"])) if cf else None),
                "hbm_frac": None,
                "kernel_ms": round(kern[dominant], 4),
                "valu_issue": None,
                "work": {"entries_tested": int(walked), "candidates": int(cands), "blended": int(n_emit),
                         "flop": int(flops)}}
    if cf:                                 # counted HBM bytes over the live kernel time, against 8 TB/s
        roofline["hbm_frac"] = round(roofline["traffic"] / (kern[dominant] * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)
        issue_ms = float(cf["valu"]) * VALU_CYCLES / (N_SIMDS * CLOCK_GHZ * 1e9) * 1e3
        roofline["valu_issue"] = {"valu_wave_insts": float(cf["valu"]), "issue_ms": round(issue_ms, 4),
                                  "frac": round(issue_ms / kern[dominant], 3)}
    if peaks:
        roofline["measured_peaks"] = peaks
        roofline["frac_of_measured_fma"] = round(achieved / peaks["fma_TFLOPs"], 4)
    # the two rasteriser kernels together (the recorded order moves the per-pixel order's work
    # from the backward to the forward, so the pair is the fairer unit of the step)
    pair_ms = kern["render_fwd"] + kern["render_bwd"]
    pair_tflops = (fwd_flops + bwd_flops) / (pair_ms * 1e-3) / 1e12
    roofline["rasteriser_pair"] = {"flop": int(fwd_flops + bwd_flops), "kernel_ms": round(pair_ms, 4),
                                   "achieved": round(pair_tflops, 3), "frac": round(pair_tflops / FP32_PEAK_TFLOPS, 4)}
    # every kernel of the step and the query with counter figures taken on its current sources
    per_kernel = {k: {"us": float(r["avg_us"]), "bytes": int(float(r["read_bytes"]) + float(r["write_bytes"])),
                      "hbm_frac": float(r["hbm_frac"]), "issue_frac": float(r["issue_frac"]),
                      "lds_bank_conflict": float(r["lds_bank_conflict"])}
                  for k, r in profile.items() if counter_figures(k, args, profile)}

    result = {
        "metric": METRIC,
        "value": round(wall, 3),
        "unit": "ms/iter",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"unbounded {args.n} Gaussians SH3, 1920x1080, fwd+bwd training step, "
                               f"window {args.window}, tile {args.tile}, depth+normal on, L1 loss",
                   "instances": int(k_used), "blended_per_pixel": round(n_emit / P, 2)},
        "per_call_ms": {k: round(v, 4) for k, v in per.items()},
        "roofline": roofline,
        "per_kernel": {"source": [os.path.relpath(p, ROOT) for p in PROFILES], "kernels": per_kernel},
    }

    if not args.no_graph_step:
        log("graph-captured step")
        result["graph_step_ms"] = graph_step(g, C, args.tile, args.window, target, d_acc, d_depth, d_normal, stream)
        torch.cuda.empty_cache()

    if not args.no_window_sweep:
        log("window sweep")
        result["window_sweep"] = window_sweep(g, C, opts.capacity, target, d_acc, d_depth, d_normal, stream,
                                              min(args.steps, 10), args.tile)
        torch.cuda.empty_cache()

    if not args.no_opacity_term:
        log("step with the opacity term")
        result["opacity_term"] = opacity_term_step(g, C, opts, rast, out, grads, target, d_acc, d_depth, d_normal,
                                                   stream, args.steps)

    if not args.no_multiview:
        log("multiview step")
        result["multiview"] = multiview_step(g, stream)
        torch.cuda.empty_cache()

    if not args.no_query:
        log("query workload")
        del rast, out, grads
        torch.cuda.empty_cache()
        qscene = scenes.unbounded_scene(args.query_gaussians, seed=0)
        pts_np = scenes.box_corner_points(qscene)
        qcams = sof.Cameras(scenes.ring_cameras(48, 960, 540))
        qg = sof.Gaussians.from_numpy(qscene)
        pts = torch.from_numpy(pts_np).cuda()
        q_sample = np.random.default_rng(7).choice(pts_np.shape[0], args.cpu_query_points, replace=False)
        q_sample_pts = pts_np[q_sample].copy()
        del pts_np
        q = sof.OpacityQuery(qcams, sof.Options(tile=args.query_tile))
        o = q(qg, pts)                                  # sizes the buffers (host read-back)
        q.auto_capacity = False
        torch.cuda.synchronize()
        times = []
        qtimer = sof.KernelTimer()
        for _ in range(args.query_steps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            with qtimer:
                a.record(stream)
                q(qg, pts, out=o)
                b.record(stream)
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        tq = float(np.median(times))
        tk = float(np.median(qtimer.ms("query")))
        q_sample_gpu = o[torch.from_numpy(q_sample).cuda()].cpu().numpy()
        n_query_points = int(pts.shape[0])
        npts = int(pts.shape[0])
        result["query"] = {"workload": f"{args.query_gaussians} Gaussians, {npts} points (centres + 3-sigma box "
                                       f"corners), min over {len(qcams)} views 960x540, one persistent launch",
                           "ms": round(tq, 2), "eval_kernel_ms": round(tk, 2),
                           "points_per_s": round(npts / (tq * 1e-3), 1),
                           "point_views_per_s": round(q.last[1] / (tq * 1e-3), 1),
                           "point_view_pairs": int(q.last[1]), "instances": int(q.last[0])}
        if not args.no_per_view:
            log("query, one launch per view")
            result["query"]["per_view_launches"] = per_view_query(qg, pts, qcams, args.query_tile, o, tq, stream)
        log("3D filter")
        sof.filter3d(qg, qcams)
        torch.cuda.synchronize()
        f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        f0.record(stream)
        gf, fvar = sof.filter3d(qg, qcams)
        f1.record(stream)
        torch.cuda.synchronize()
        result["filter3d"] = {"workload": f"{qg.n} Gaussians, {len(qcams)} cameras", "ms": round(f0.elapsed_time(f1), 3),
                              "below_1_255_after_filter": round(float((gf.opac < 1.0 / 255).float().mean()), 4)}
        del gf, fvar
        if not args.no_levelset:
            log("level-set query and binary search")
            result["levelset"] = levelset_search(qg, pts, qcams, args.query_tile, tq, stream)
        del q, qg, pts, o
        torch.cuda.empty_cache()
    else:
        qscene = qcams = q_sample_pts = q_sample_gpu = None
        n_query_points = 0

    if not args.no_cpu_baseline:
        log("cpu baseline")
        cb = cpu_baseline(scene, cam, args.window, args.cpu_pixels, qscene,
                          None if qcams is None else qcams.list, q_sample_pts, n_query_points)
        if q_sample_gpu is not None:           # the GPU's values of the same points beside the oracle's
            cb["query_sample_gpu"] = [round(float(o), 7) for o in q_sample_gpu]
            cb["query_sample_max_abs_diff"] = float(np.max(np.abs(np.asarray(cb["query_sample_opacity"]) -
                                                                  q_sample_gpu)))
        result["cpu_baseline"] = cb

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
