"""Thin ctypes binding of libsof.so.

Only argument marshalling lives here: every step of the hot path runs in the HIP kernels
behind the C ABI.  PyTorch supplies device memory and the current stream.  The library
must be built (``python -m paper_2506_19139_amd.build``); nothing falls back to another
implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsof.so")

SOF_OK, SOF_E_ARG, SOF_E_WORKSPACE, SOF_E_CAPACITY, SOF_E_HIP, SOF_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
SOF_E_SCRATCH = -6
STATIC_SCRATCH_INSTANCES = 1 << 20    # capacity limit of sof_render_bwd_static
SOF_DEPTH_MEDIAN = 1 << 0
SOF_DEPTH_GRAD_FULL = 1 << 1
SOF_QUERY_KEYS = 1 << 2
SOF_QUERY_LEVELSET = 1 << 3
SOF_QUERY_REUSE = 1 << 4

WINDOWS = (0, 1, 2, 4, 8, 16, 32)
AUX_CHANNELS = 6      # T_end, n_emitted, k, T_k, entries tested, candidates
LOSS_CHANNELS = 6     # distortion, extent, mean and moment of d, opacity tail, position of k
# Gaussians per pixel the recorded blend order holds by default; a tile with a pixel that blends
# more is replayed by the backward instead (at 1M Gaussians and 1080p the most is ~150)
DEFAULT_ORDER_SLOTS = 256
TILES = (8, 16, 32)


class SofError(RuntimeError):
    pass


class CGaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("means", ctypes.c_void_p), ("scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("opacities", ctypes.c_void_p), ("sh", ctypes.c_void_p)]


class CCamera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class COptions(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("window", ctypes.c_int32), ("near_plane", ctypes.c_float),
                ("bg", ctypes.c_float * 3), ("flags", ctypes.c_uint32), ("order_slots", ctypes.c_int32),
                ("capacity", ctypes.c_int64)]


assert ctypes.sizeof(CCamera) == 72

_lib = None
_P = ctypes.c_void_p
_SZ = ctypes.POINTER(ctypes.c_size_t)

_SIGS = {
    "sof_workspace_size": (ctypes.c_int, [ctypes.c_int64, _P, ctypes.c_int32, _P, _SZ, _SZ, _SZ, _SZ]),
    "sof_read_status_offset": (ctypes.c_size_t, []),
    "sof_project": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P, _P, ctypes.c_size_t, _P]),
    "sof_bin_sort": (ctypes.c_int, [ctypes.c_int64, _P, _P, ctypes.c_int32, _P, _P, ctypes.c_size_t, _P,
                                    ctypes.c_size_t, _P]),
    "sof_render_fwd": (ctypes.c_int, [ctypes.c_int64, _P, _P, ctypes.c_int32, _P, _P, ctypes.c_size_t, _P,
                                      ctypes.c_size_t, _P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "sof_render_order": (ctypes.c_int, [ctypes.c_int64, _P, _P, ctypes.c_int32, _P, _P, ctypes.c_size_t, _P,
                                        ctypes.c_size_t, _P, ctypes.c_int64, ctypes.c_int32, _P, _P, _P, _P, _P]),
    "sof_render_opacity": (ctypes.c_int, [ctypes.c_int64, _P, _P, ctypes.c_int32, _P, _P, ctypes.c_size_t, _P,
                                          ctypes.c_size_t, _P, _P, _P, _P, ctypes.c_size_t, _P, _P]),
    "sof_render_bwd": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P, _P, ctypes.c_size_t, _P, ctypes.c_size_t,
                                      _P, _P, _P, _P, ctypes.c_size_t, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                      ctypes.c_size_t, _P, _P, _P, _P, _P, _P]),
    "sof_render_bwd_static": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P, _P, ctypes.c_size_t, _P,
                                             ctypes.c_size_t, _P, _P, _P, _P, ctypes.c_size_t, _P, _P, _P, _P, _P,
                                             _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "sof_query_workspace_size": (ctypes.c_int, [ctypes.c_int64, _P, ctypes.c_int32, _P, ctypes.c_int64,
                                                ctypes.c_int64, _SZ, _SZ, _SZ]),
    "sof_opacity_query": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P, _P, ctypes.c_int64, ctypes.c_int64,
                                         _P, _P, ctypes.c_size_t, _P, ctypes.c_size_t, _P, ctypes.c_size_t, _P]),
    "sof_filter3d": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.c_float, ctypes.c_float, _P, _P, _P, _P]),
    "sof_filter3d_bwd": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "sof_set_timing_events": (ctypes.c_int, [_P]),
    "sof_bisect_step": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int64, _P]),
    "sof_bench_copy": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P]),
    "sof_bench_fma": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int32, _P]),
    "sof_strerror": (ctypes.c_char_p, [ctypes.c_int]),
}

EXPORTED = tuple(_SIGS)


def lib():
    """Load libsof.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SofError(f"{LIB_PATH} is missing: build it with `python -m paper_2506_19139_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(code, what):
    if code != SOF_OK:
        msg = lib().sof_strerror(code).decode()
        raise SofError(f"{what}: {msg} ({code})")


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _nbytes(t):
    return 0 if t is None else t.numel() * t.element_size()


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# ------------------------------------------------------------------------------ inputs

@dataclass
class Gaussians:
    means: torch.Tensor
    scales: torch.Tensor
    quats: torch.Tensor
    opac: torch.Tensor
    sh: torch.Tensor
    sh_degree: int

    @staticmethod
    def from_numpy(d, device="cuda"):
        f = lambda k: torch.from_numpy(np.ascontiguousarray(d[k], np.float32)).to(device)
        return Gaussians(f("means"), f("scales"), f("quats"), f("opac").reshape(-1), f("sh"), int(d["sh_degree"]))

    @property
    def n(self):
        return int(self.means.shape[0])

    def c_struct(self):
        for t in (self.means, self.scales, self.quats, self.opac, self.sh):
            if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
                raise SofError("Gaussian parameters must be contiguous float32 CUDA tensors")
        return CGaussians(self.n, self.sh_degree, 0, self.means.data_ptr(), self.scales.data_ptr(),
                          self.quats.data_ptr(), self.opac.data_ptr(), self.sh.data_ptr())


class Cameras:
    """Host and device copies of an array of sof_camera."""

    def __init__(self, cams, device="cuda"):
        if isinstance(cams, dict):
            cams = [cams]
        self.list = list(cams)
        n = len(self.list)
        self.host = (CCamera * n)()
        for i, c in enumerate(self.list):
            R = np.asarray(c["R"], np.float32).reshape(9)
            t = np.asarray(c["t"], np.float32).reshape(3)
            self.host[i].R[:] = [float(x) for x in R]
            self.host[i].t[:] = [float(x) for x in t]
            self.host[i].fx, self.host[i].fy = float(c["fx"]), float(c["fy"])
            self.host[i].cx, self.host[i].cy = float(c["cx"]), float(c["cy"])
            self.host[i].width, self.host[i].height = int(c["width"]), int(c["height"])
        raw = np.frombuffer(bytes(self.host), dtype=np.uint8).copy()
        self.device = torch.from_numpy(raw).to(device)

    def __len__(self):
        return len(self.list)

    @property
    def sizes(self):
        return [(int(c["width"]), int(c["height"])) for c in self.list]

    @property
    def n_pixels(self):
        return sum(w * h for w, h in self.sizes)

    def hp(self):
        return ctypes.cast(self.host, ctypes.c_void_p)

    def dp(self):
        return ctypes.c_void_p(self.device.data_ptr())


@dataclass
class Options:
    tile: int = 16
    window: int = 8
    near_plane: float = 0.2
    bg: tuple = (0.0, 0.0, 0.0)
    flags: int = 0
    capacity: int = 0
    # per-pixel capacity of the recorded blend order (0: none; the backward then replays)
    order_slots: int = DEFAULT_ORDER_SLOTS

    def c_struct(self):
        o = COptions()
        o.tile, o.window, o.near_plane = int(self.tile), int(self.window), float(self.near_plane)
        o.bg[:] = [float(x) for x in self.bg]
        o.flags, o.order_slots, o.capacity = int(self.flags), int(self.order_slots), int(self.capacity)
        return o


# ------------------------------------------------------------------------------ raw calls

def workspace_size(n, cams: Cameras, opts: Options):
    """(proj, bins, grads, order) buffer sizes in bytes."""
    p, b, g, r = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    o = opts.c_struct()
    _check(lib().sof_workspace_size(n, cams.hp(), len(cams), ctypes.byref(o), ctypes.byref(p), ctypes.byref(b),
                                    ctypes.byref(g), ctypes.byref(r)), "sof_workspace_size")
    return p.value, b.value, g.value, r.value


def project(g: Gaussians, cams: Cameras, opts: Options, proj: torch.Tensor):
    gs, o = g.c_struct(), opts.c_struct()
    _check(lib().sof_project(ctypes.byref(gs), cams.hp(), cams.dp(), len(cams), ctypes.byref(o), _ptr(proj),
                             proj.numel(), _stream()), "sof_project")


def bin_sort(n, cams: Cameras, opts: Options, proj, bins):
    o = opts.c_struct()
    _check(lib().sof_bin_sort(n, cams.hp(), cams.dp(), len(cams), ctypes.byref(o), _ptr(proj), proj.numel(),
                              _ptr(bins), bins.numel(), _stream()), "sof_bin_sort")


def render_fwd(n, cams: Cameras, opts: Options, proj, bins, rgb=None, acc=None, depth=None, normal=None, aux=None,
               losses=None, order=None):
    o = opts.c_struct()
    _check(lib().sof_render_fwd(n, cams.hp(), cams.dp(), len(cams), ctypes.byref(o), _ptr(proj), proj.numel(),
                                _ptr(bins), bins.numel(), _ptr(rgb), _ptr(acc), _ptr(depth), _ptr(normal), _ptr(aux),
                                _ptr(losses), _ptr(order), _nbytes(order), _stream()), "sof_render_fwd")


def render_order(n, cams: Cameras, opts: Options, proj, bins, slot, n_slots, max_entries):
    """Per-pixel order output (sof_render_order) for the pixels whose slot is in [0, n_slots):
    (stream_ids, stream_keys, emit_ids [n_slots, M], counts [n_slots, 2]) device tensors."""
    dev = slot.device
    M = int(max_entries)
    stream_ids = torch.full((max(n_slots, 1), max(M, 1)), -1, dtype=torch.int32, device=dev)
    stream_keys = torch.full((max(n_slots, 1), max(M, 1)), float("nan"), dtype=torch.float32, device=dev)
    emit_ids = torch.full((max(n_slots, 1), max(M, 1)), -1, dtype=torch.int32, device=dev)
    counts = torch.zeros((max(n_slots, 1), 2), dtype=torch.int32, device=dev)
    if not (slot.dtype == torch.int32 and slot.is_contiguous() and slot.numel() == cams.n_pixels):
        raise SofError("slot must be a contiguous int32 tensor with one entry per pixel")
    o = opts.c_struct()
    _check(lib().sof_render_order(n, cams.hp(), cams.dp(), len(cams), ctypes.byref(o), _ptr(proj), proj.numel(),
                                  _ptr(bins), bins.numel(), _ptr(slot), int(n_slots), M, _ptr(stream_ids),
                                  _ptr(stream_keys), _ptr(emit_ids), _ptr(counts), _stream()), "sof_render_order")
    return stream_ids[:n_slots], stream_keys[:n_slots], emit_ids[:n_slots], counts[:n_slots]


def render_opacity(n, cams: Cameras, opts: Options, proj, bins, depth, aux, opacity, losses=None, order=None):
    o = opts.c_struct()
    _check(lib().sof_render_opacity(n, cams.hp(), cams.dp(), len(cams), ctypes.byref(o), _ptr(proj), proj.numel(),
                                    _ptr(bins), bins.numel(), _ptr(depth), _ptr(aux), _ptr(losses), _ptr(order),
                                    _nbytes(order), _ptr(opacity), _stream()), "sof_render_opacity")


def render_bwd(g: Gaussians, cams: Cameras, opts: Options, proj, bins, rgb, normal, aux, d_rgb, d_acc, d_depth,
               d_normal, grads, d_means, d_scales, d_quats, d_opac, d_sh, depth=None, opacity=None, d_opacity=None,
               losses=None, d_losses=None, order=None):
    gs, o = g.c_struct(), opts.c_struct()
    _check(lib().sof_render_bwd(ctypes.byref(gs), cams.hp(), cams.dp(), len(cams), ctypes.byref(o), _ptr(proj),
                                proj.numel(), _ptr(bins), bins.numel(), _ptr(rgb), _ptr(normal), _ptr(aux),
                                _ptr(order), _nbytes(order), _ptr(d_rgb), _ptr(d_acc), _ptr(d_depth), _ptr(d_normal), _ptr(depth), _ptr(opacity),
                                _ptr(d_opacity), _ptr(losses), _ptr(d_losses), _ptr(grads),
                                grads.numel() if grads is not None else 0,
                                _ptr(d_means), _ptr(d_scales), _ptr(d_quats), _ptr(d_opac), _ptr(d_sh), _stream()),
           "sof_render_bwd")


def render_bwd_static(g: Gaussians, cams: Cameras, opts: Options, proj, bins, rgb, normal, aux, d_rgb, d_acc,
                      d_depth, d_normal, d_means, d_scales, d_quats, d_opac, d_sh, depth=None, opacity=None,
                      d_opacity=None, losses=None, d_losses=None, order=None):
    """sof_render_bwd_static: the backward without a caller workspace (the library's static
    per-device scratch holds the per-instance partials; opts.capacity <= 2^20)."""
    gs, o = g.c_struct(), opts.c_struct()
    _check(lib().sof_render_bwd_static(ctypes.byref(gs), cams.hp(), cams.dp(), len(cams), ctypes.byref(o),
                                       _ptr(proj), proj.numel(), _ptr(bins), bins.numel(), _ptr(rgb), _ptr(normal),
                                       _ptr(aux), _ptr(order), _nbytes(order), _ptr(d_rgb), _ptr(d_acc), _ptr(d_depth), _ptr(d_normal),
                                       _ptr(depth), _ptr(opacity), _ptr(d_opacity), _ptr(losses), _ptr(d_losses),
                                       _ptr(d_means), _ptr(d_scales), _ptr(d_quats), _ptr(d_opac), _ptr(d_sh),
                                       _stream()), "sof_render_bwd_static")


def filter3d(g: Gaussians, cams: Cameras, k=0.2, near_plane=0.2):
    """3D filter: (filtered Gaussians, per-Gaussian filter size s).  The filtered set shares
    means, rotations and colours with g."""
    var = torch.empty_like(g.opac)
    scales, opac = torch.empty_like(g.scales), torch.empty_like(g.opac)
    gs = g.c_struct()
    n_cams = len(cams) if cams is not None else 0
    _check(lib().sof_filter3d(ctypes.byref(gs), cams.hp() if n_cams else None, cams.dp() if n_cams else None, n_cams,
                              float(near_plane), float(k), _ptr(var), _ptr(scales), _ptr(opac), _stream()),
           "sof_filter3d")
    return Gaussians(g.means, scales, g.quats, opac, g.sh, g.sh_degree), var


def filter3d_bwd(g: Gaussians, var, d_scales_out, d_opac_out):
    """Gradients with respect to g's scales and opacities from those of the filtered set."""
    d_scales, d_opac = torch.empty_like(g.scales), torch.empty_like(g.opac)
    gs = g.c_struct()
    _check(lib().sof_filter3d_bwd(ctypes.byref(gs), _ptr(var), _ptr(d_scales_out), _ptr(d_opac_out), _ptr(d_scales),
                                  _ptr(d_opac), _stream()), "sof_filter3d_bwd")
    return d_scales, d_opac


def read_status(buf: torch.Tensor):
    """(instances requested, status flags) from a bins / schedule buffer (synchronises)."""
    off = lib().sof_read_status_offset()
    raw = buf[off:off + 16].cpu().numpy()
    return int(raw[:8].view(np.int64)[0]), int(raw[8:12].view(np.int32)[0])


def measure_peaks(copy_mib=2048, fma_blocks=256 * 64, fma_iters=4096, reps=5):
    """Reachable machine peaks on the current device (instrumentation kernels of the library):
    HBM GB/s of a streaming copy (bytes read + written) and float32 TFLOP/s of FMA chains,
    each the best of `reps` timed launches after one warm-up."""
    n4 = copy_mib * (1 << 20) // 16
    src = torch.ones(4 * n4, device="cuda")
    dst = torch.empty_like(src)
    out = torch.empty(fma_blocks * 256, device="cuda")
    s = _stream()

    def best(fn):
        fn()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return min(ts)
    t_copy = best(lambda: _check(lib().sof_bench_copy(_ptr(src), _ptr(dst), n4, s), "sof_bench_copy"))
    t_fma = best(lambda: _check(lib().sof_bench_fma(_ptr(out), fma_blocks, fma_iters, s), "sof_bench_fma"))
    assert torch.equal(dst, src)
    flops = 2.0 * 16 * fma_iters * fma_blocks * 256
    return {"copy_GBps": round(2 * 16 * n4 / (t_copy * 1e-3) / 1e9, 1), "copy_bytes": 2 * 16 * n4,
            "fma_TFLOPs": round(flops / (t_fma * 1e-3) / 1e12, 2), "fma_flops": int(flops)}


TIMED_KERNELS = ("render_fwd", "render_bwd", "query")


class KernelTimer:
    """HIP events recorded by the library immediately around its rasteriser and query
    kernels (sof_set_timing_events), for per-kernel durations on the launch stream.  Usage:
    `with timer: <calls>` then `timer.ms("render_bwd")` after a synchronisation.  Each use
    of the context holds one fresh set of events."""

    def __init__(self):
        self.sets = []

    def __enter__(self):
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * len(TIMED_KERNELS))]
        for e in evs:
            e.record()                        # creates the underlying hipEvent
        torch.cuda.synchronize()
        handles = (ctypes.c_void_p * len(evs))(*[e.cuda_event for e in evs])
        _check(lib().sof_set_timing_events(handles), "sof_set_timing_events")
        self.sets.append(evs)
        return self

    def __exit__(self, *exc):
        lib().sof_set_timing_events(None)
        return False

    def ms(self, kernel):
        """Per-use durations (ms) of `kernel`, one entry per context use."""
        k = TIMED_KERNELS.index(kernel)
        return [evs[2 * k].elapsed_time(evs[2 * k + 1]) for evs in self.sets]


# ------------------------------------------------------------------------------ views of bins

def sorted_instances(bins: torch.Tensor, n, cams: Cameras, opts: Options):
    """Debug view of the sorted tile lists: (bucket keys uint64, gaussian ids, ranges[n_tiles,2])
    as numpy arrays (synchronises).  Layout mirrors the internal bins layout."""
    vn = n * len(cams)
    n_tiles = sum(((w + opts.tile - 1) // opts.tile) * ((h + opts.tile - 1) // opts.tile) for w, h in cams.sizes)
    L = _bins_layout(vn, len(cams), opts.capacity, n_tiles)
    b = bins.cpu().numpy()
    k, _ = read_status(bins)
    k = min(k, opts.capacity)
    keys = b[L["keys0"]:][: 8 * k].view(np.uint64)           # tile buckets: depth key << 32 | emission index
    vals = b[L["vals0"]:][: 4 * k].view(np.uint32)           # sorted emission indices
    gid = b[L["gid"]:][: 4 * opts.capacity].view(np.int32)
    ids = gid[vals]
    ranges = b[L["ranges"]:][: 8 * n_tiles].view(np.int32).reshape(n_tiles, 2)
    return keys, ids, ranges


def recorded_order(order: torch.Tensor, cams: Cameras, opts: Options):
    """Debug view of the recorded blend order (synchronises): (flags [n_tiles] int32,
    positions [n_tiles, TS*TS/64, order_slots, 64] uint16) as numpy arrays."""
    T = opts.tile
    n_tiles = sum(((w + T - 1) // T) * ((h + T - 1) // T) for w, h in cams.sizes)
    b = order.cpu().numpy()
    rec = _align(4 * max(n_tiles, 1))
    flags = b[:4 * n_tiles].view(np.int32)
    pos = b[rec:rec + 2 * n_tiles * T * T * opts.order_slots].view(np.uint16)
    return flags, pos.reshape(n_tiles, T * T // 64, opts.order_slots, 64)


def proj_view(proj: torch.Tensor, n, n_cams):
    """Debug view of sof_project's per (camera, Gaussian) records as numpy arrays
    (synchronises): rect [V*N,4] int16, mu_z [V*N] float32, zmin [V*N] float32."""
    vn = n * n_cams
    o, L = 0, {}
    for name, size in [("geom", vn * 64), ("app", vn * 32), ("bwdr", vn * 32), ("rect", vn * 8), ("zmin", vn * 4)]:
        L[name] = o
        o = _align(o + size)
    b = proj.cpu().numpy()
    geom = b[L["geom"]:L["geom"] + vn * 64].view(np.float32).reshape(vn, 16)
    rect = b[L["rect"]:L["rect"] + vn * 8].view(np.int16).reshape(vn, 4)
    zmin = b[L["zmin"]:L["zmin"] + vn * 4].view(np.float32)
    app = b[L["app"]:L["app"] + vn * 32].view(np.float32).reshape(vn, 8)
    return dict(rect=rect.copy(), mu_z=geom[:, 12].copy(), zmin=zmin.copy(), color=app[:, :3].copy(),
                normal=app[:, 4:7].copy(), geom=geom.copy())


def _align(x, a=256):
    return (x + a - 1) // a * a


def _bins_layout(vn, n_cams, cap, n_tiles):
    """Python mirror of the BinsLayout offsets (for debug views only)."""
    sort_tile, scan_chunk = 8 * 256, 16 * 256
    nb = -(-max(cap, 1) // sort_tile)
    L, o = {}, 0
    for name, size in [("status", 256), ("cams", (n_cams + 1) * 32), ("counts", vn * 4), ("offsets", vn * 8),
                       ("scan_tmp", (-(-max(vn, 1) // scan_chunk) + 1) * 8), ("keys0", cap * 8), ("keys1", cap * 8),
                       ("vals0", cap * 4), ("vals1", cap * 4), ("gid", cap * 4), ("hist", 256 * nb * 4),
                       ("hist_tmp", (-(-(256 * nb) // scan_chunk) + 1) * 8), ("ranges", max(n_tiles, 1) * 8)]:
        L[name] = o
        o = _align(o + size)
    L["total"] = o
    return L


# ------------------------------------------------------------------------------ high level

class Rasterizer:
    """Owns the three workspace buffers for one camera set and grows the instance capacity
    on demand (the only host read-back happens when `auto_capacity` is on)."""

    def __init__(self, cams: Cameras, opts: Options, auto_capacity=True, device="cuda"):
        self.cams, self.opts, self.device = cams, opts, device
        self.auto_capacity = auto_capacity
        self.proj = self.bins = self.grads = self.order_rec = None
        self._n = -1
        self.last_count = 0
        # bumped by every prepare(): proj and bins then hold another frame's lists, so a
        # backward saved against an older generation would replay the wrong frame
        self.generation = 0

    def _alloc(self, n):
        p, b, g, r = workspace_size(n, self.cams, self.opts)
        if self.proj is None or self.proj.numel() < p:
            self.proj = torch.empty(p, dtype=torch.uint8, device=self.device)
        if self.bins is None or self.bins.numel() < b:
            self.bins = torch.empty(b, dtype=torch.uint8, device=self.device)
        if self.grads is None or self.grads.numel() < g:
            self.grads = torch.empty(max(g, 16), dtype=torch.uint8, device=self.device)
        if r == 0:
            self.order_rec = None
        elif self.order_rec is None or self.order_rec.numel() < r:
            self.order_rec = torch.empty(r, dtype=torch.uint8, device=self.device)

    def prepare(self, g: Gaussians):
        """project + bin_sort; returns the instance count (read back only in auto mode)."""
        n = g.n
        if self.opts.capacity <= 0:
            self.opts.capacity = max(1024, 4 * n * len(self.cams))
        self.generation += 1
        self._alloc(n)
        project(g, self.cams, self.opts, self.proj)
        bin_sort(n, self.cams, self.opts, self.proj, self.bins)
        if self.auto_capacity:
            k, flags = read_status(self.bins)
            self.last_count = k
            if k > self.opts.capacity:
                self.opts.capacity = int(k * 1.25) + 1024
                self._alloc(n)
                bin_sort(n, self.cams, self.opts, self.proj, self.bins)
        return self.last_count

    def alloc_outputs(self):
        P = self.cams.n_pixels
        dev = self.device
        # "order" is the rasterizer's own recorded-order buffer (None until allocated or when
        # opts.order_slots is 0): a forward writes it, the backward of that forward reads it
        return dict(rgb=torch.empty(3 * P, device=dev), acc=torch.empty(P, device=dev), depth=torch.empty(P, device=dev),
                    normal=torch.empty(3 * P, device=dev), aux=torch.empty(AUX_CHANNELS * P, device=dev),
                    order=self.order_rec)

    def forward(self, g: Gaussians, out=None, losses=False):
        """Render; with losses=True also the per-pixel distortion and extent losses in
        out["losses"] ([6, P]: distortion, extent, and four channels the backward and the
        opacity pass read).  With opts.order_slots > 0 the blend order is recorded into the
        rasterizer's order buffer (out["order"]) for the backward."""
        self.prepare(g)
        out = out or self.alloc_outputs()
        if losses and "losses" not in out:
            out["losses"] = torch.empty(LOSS_CHANNELS * self.cams.n_pixels, device=self.device)
        out["order"] = self.order_rec
        render_fwd(g.n, self.cams, self.opts, self.proj, self.bins, out["rgb"], out["acc"], out["depth"],
                   out["normal"], out["aux"], out["losses"] if losses else None, order=out["order"])
        return out

    def order(self, g: Gaussians, pixels_per_cam, max_entries=512):
        """Per-pixel order of the last forward for the listed pixels ((px, py) per camera).
        Returns, per camera, a list of dicts: stream ids / keys (candidates in the order the
        window received them), emitted ids (in the order they left it), as numpy arrays."""
        slot = torch.full((self.cams.n_pixels,), -1, dtype=torch.int32)
        where, off, n_slots = [], 0, 0
        for (w, h), pixels in zip(self.cams.sizes, pixels_per_cam):
            for px, py in pixels:
                slot[off + py * w + px] = n_slots
                where.append(n_slots)
                n_slots += 1
            off += w * h
        sid, skey, eid, cnt = render_order(g.n, self.cams, self.opts, self.proj, self.bins, slot.to(self.device),
                                           n_slots, max_entries)
        sid, skey, eid, cnt = (t.cpu().numpy() for t in (sid, skey, eid, cnt))
        res, i = [], 0
        for pixels in pixels_per_cam:
            cam_res = []
            for _ in pixels:
                nf, no = int(cnt[i, 0]), int(cnt[i, 1])
                if nf > max_entries or no > max_entries:
                    raise SofError(f"order output truncated ({nf} fed, {no} out > {max_entries})")
                cam_res.append(dict(stream_ids=sid[i, :nf].copy(), stream_keys=skey[i, :nf].copy(),
                                    emit_ids=eid[i, :no].copy()))
                i += 1
            res.append(cam_res)
        return res

    def opacity(self, g: Gaussians, out, split=True):
        """Opacity field at each pixel's rendered depth (second pass after forward); stored in
        out["opa"] (0 where a pixel has no 0.5 crossing).  With split (and a forward run with
        losses=True) the pass visits only the Gaussians in front of the crossing and takes the
        rest from the forward; otherwise it replays every blended Gaussian."""
        if "opa" not in out:
            out["opa"] = torch.empty(self.cams.n_pixels, device=self.device)
        losses = out.get("losses") if split else None
        render_opacity(g.n, self.cams, self.opts, self.proj, self.bins, out["depth"], out["aux"], out["opa"],
                       losses=losses, order=out.get("order"))
        return out["opa"]

    def backward(self, g: Gaussians, out, d_rgb=None, d_acc=None, d_depth=None, d_normal=None, grads_out=None,
                 d_opa=None, d_losses=None):
        """Gradients of a loss with upstream d_rgb, d_acc, d_depth, d_normal, d_opa (of
        out["opa"]) and d_losses ([2, P], of the distortion and extent rows of out["losses"])."""
        if grads_out is None:
            grads_out = dict(means=torch.empty_like(g.means), scales=torch.empty_like(g.scales),
                             quats=torch.empty_like(g.quats), opac=torch.empty_like(g.opac),
                             sh=torch.empty_like(g.sh))
        render_bwd(g, self.cams, self.opts, self.proj, self.bins, out["rgb"], out["normal"], out["aux"], d_rgb, d_acc,
                   d_depth, d_normal, self.grads, grads_out["means"], grads_out["scales"], grads_out["quats"],
                   grads_out["opac"], grads_out["sh"], depth=out["depth"] if d_opa is not None else None,
                   opacity=out.get("opa") if d_opa is not None else None, d_opacity=d_opa,
                   losses=out.get("losses") if d_losses is not None else None, d_losses=d_losses,
                   order=out.get("order"))
        return grads_out

    def split(self, flat, channels):
        """Split a concatenated output into per-camera [C,H,W] views."""
        res, off = [], 0
        for w, h in self.cams.sizes:
            res.append(flat[off:off + channels * w * h].view(channels, h, w))
            off += channels * w * h
        return res


class SofRasterize(torch.autograd.Function):
    """Differentiable render of activated Gaussian parameters.

    forward(means, scales, quats, opac, sh, rasterizer) -> (rgb, acc, depth, normal), each the
    concatenation over the rasterizer's cameras ([3*P], [P], [P], [3*P])."""

    @staticmethod
    def forward(ctx, means, scales, quats, opac, sh, rast: Rasterizer, sh_degree: int):
        g = Gaussians(means.contiguous(), scales.contiguous(), quats.contiguous(), opac.contiguous(),
                      sh.contiguous(), int(sh_degree))
        out = rast.forward(g)
        # the backward replays from the rasterizer's proj / bins buffers: remember which
        # frame they hold, so that a later forward through the same rasterizer is caught
        ctx.rast, ctx.generation, ctx.sh_degree = rast, rast.generation, int(sh_degree)
        ctx.order = out["order"]          # the rasterizer's buffer, guarded by the generation
        ctx.save_for_backward(g.means, g.scales, g.quats, g.opac, g.sh, out["rgb"], out["normal"], out["aux"])
        return out["rgb"], out["acc"], out["depth"], out["normal"]

    @staticmethod
    def backward(ctx, d_rgb, d_acc, d_depth, d_normal):
        if ctx.rast.generation != ctx.generation:
            raise SofError("SofRasterize.backward: the rasterizer rendered another frame after this forward "
                           "(its tile lists were overwritten); use one Rasterizer per pending backward")
        means, scales, quats, opac, sh, rgb, normal, aux = ctx.saved_tensors
        g = Gaussians(means, scales, quats, opac, sh, ctx.sh_degree)
        out = dict(rgb=rgb, normal=normal, aux=aux, order=ctx.order)
        c = lambda t: None if t is None else t.contiguous()
        gr = ctx.rast.backward(g, out, c(d_rgb), c(d_acc), c(d_depth), c(d_normal))
        return gr["means"], gr["scales"], gr["quats"], gr["opac"], gr["sh"], None, None


# ------------------------------------------------------------------------------ queries

def query_workspace_size(n, cams: Cameras, opts: Options, n_points, pv_capacity):
    p, b, s = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    o = opts.c_struct()
    _check(lib().sof_query_workspace_size(n, cams.hp(), len(cams), ctypes.byref(o), n_points, pv_capacity,
                                          ctypes.byref(p), ctypes.byref(b), ctypes.byref(s)),
           "sof_query_workspace_size")
    return p.value, b.value, s.value


def opacity_query_raw(g: Gaussians, cams: Cameras, opts: Options, points, pv_capacity, out, proj, bins, sched):
    gs, o = g.c_struct(), opts.c_struct()
    n_points = int(points.shape[0])
    _check(lib().sof_opacity_query(ctypes.byref(gs), cams.hp(), cams.dp(), len(cams), ctypes.byref(o), _ptr(points),
                                   n_points, int(pv_capacity), _ptr(out), _ptr(proj), proj.numel(), _ptr(bins),
                                   bins.numel(), _ptr(sched), sched.numel(), _stream()), "sof_opacity_query")


class OpacityQuery:
    """Buffers for repeated opacity-field queries over one camera set.  Instance and
    (point, view) capacities grow on demand (read-back of the status words, then one rerun)."""

    def __init__(self, cams: Cameras, opts: Options = None, device="cuda", auto_capacity=True):
        self.cams = cams
        self.opts = opts or Options()
        self.device = device
        self.auto_capacity = auto_capacity
        self.pv_capacity = 0
        self.proj = self.bins = self.sched = None
        self.last = (0, 0)

    def _alloc(self, n, n_points):
        """Size the buffers; True if the Gaussian-side buffers were (re)allocated."""
        p, b, s = query_workspace_size(n, self.cams, self.opts, n_points, self.pv_capacity)
        grown = False
        if self.proj is None or self.proj.numel() < p:
            self.proj = torch.empty(p, dtype=torch.uint8, device=self.device)
            grown = True
        if self.bins is None or self.bins.numel() < b:
            self.bins = torch.empty(b, dtype=torch.uint8, device=self.device)
            grown = True
        if self.sched is None or self.sched.numel() < s:
            self.sched = torch.empty(s, dtype=torch.uint8, device=self.device)
        return grown

    def __call__(self, g: Gaussians, points: torch.Tensor, out=None, reuse_gaussians=False):
        """O(x) for every point.  reuse_gaussians: the buffers still hold the Gaussian side of
        the previous call with these same Gaussians (skips their projection and sort)."""
        n_points = int(points.shape[0])
        if self.opts.capacity <= 0:
            self.opts.capacity = max(1024, 2 * g.n * len(self.cams))
        if self.pv_capacity <= 0:
            self.pv_capacity = min(n_points * len(self.cams), 2 ** 31 - 1)
        out = torch.empty(n_points, dtype=torch.float32, device=self.device) if out is None else out
        for attempt in range(3):
            grown = self._alloc(g.n, n_points)
            reuse = reuse_gaussians and attempt == 0 and not grown and self.proj is not None
            opts = Options(**{**self.opts.__dict__, "flags": self.opts.flags | (SOF_QUERY_REUSE if reuse else 0)})
            opacity_query_raw(g, self.cams, opts, points, self.pv_capacity, out, self.proj, self.bins, self.sched)
            if not self.auto_capacity:
                break
            k_inst, f_inst = read_status(self.bins)
            k_pv, f_pv = read_status(self.sched)
            self.last = (k_inst, k_pv)
            grow = False
            if k_inst > self.opts.capacity:
                self.opts.capacity = min(int(k_inst * 1.1) + 1024, 2 ** 31 - 1)
                grow = True
            if k_pv > self.pv_capacity:
                self.pv_capacity = min(int(k_pv * 1.05) + 1024, 2 ** 31 - 1)
                grow = True
            if not grow:
                break
        return out


def bisect_step(a: torch.Tensor, b: torch.Tensor, mid: torch.Tensor, opacity: torch.Tensor = None):
    """One binary-search step on edges (a inside, b outside; [n, 3] float32, updated in place):
    with `opacity` (at mid) the midpoint replaces a or b, then mid = (a + b) / 2."""
    n = int(a.shape[0])
    assert a.shape == b.shape == mid.shape and a.dtype == b.dtype == mid.dtype == torch.float32
    assert a.is_contiguous() and b.is_contiguous() and mid.is_contiguous()
    if opacity is not None:
        assert opacity.shape == (n,) and opacity.dtype == torch.float32 and opacity.is_contiguous()
    _check(lib().sof_bisect_step(_ptr(a), _ptr(b), _ptr(mid), _ptr(opacity), n, _stream()), "sof_bisect_step")


class LevelSetSearch:
    """Binary search towards the 0.5 level set of the opacity field over a camera set
    (Sec. 3.4): the opacity at the midpoints comes from level-set queries (stop a view
    at O_N > 0.5, skip points some view put at or below 0.5), one launch per step."""

    def __init__(self, cams: Cameras, tile=8, device="cuda"):
        self.query = OpacityQuery(cams, Options(tile=tile, flags=SOF_QUERY_LEVELSET), device=device)

    def orient(self, g: Gaussians, p: torch.Tensor, q: torch.Tensor):
        """Edges (p, q) whose ends lie on opposite sides of the level set, as (inside, outside)
        pairs."""
        op = self.query(g, p).clone()
        oq = self.query(g, q)
        ip, iq = op > 0.5, oq > 0.5
        keep = ip != iq
        a = torch.where(ip[keep, None], p[keep], q[keep]).contiguous()
        b = torch.where(ip[keep, None], q[keep], p[keep]).contiguous()
        return a, b

    def __call__(self, g: Gaussians, a: torch.Tensor, b: torch.Tensor, steps=8):
        """Final midpoints after `steps` halvings (a and b are updated in place)."""
        mid = torch.empty_like(a)
        bisect_step(a, b, mid)
        o = torch.empty(a.shape[0], dtype=torch.float32, device=a.device)
        for step in range(steps):
            # the Gaussian side (projection, tile lists) is built once per search
            self.query(g, mid, out=o, reuse_gaussians=step > 0)
            bisect_step(a, b, mid, o)
        return mid


def opacity_query(g: Gaussians, cams: Cameras, points: torch.Tensor, opts: Options = None):
    """O(x) = min over views of O_N(x) for every point (one call, fresh buffers)."""
    return OpacityQuery(cams, opts or Options())(g, points.contiguous())
