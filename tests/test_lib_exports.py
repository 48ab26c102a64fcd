"""The C-ABI library loads and exports every entry point include/sof.h declares; host-side
argument checks work without a GPU (no compute call is made here)."""
import ctypes
import os
import re

import pytest

from paper_2506_19139_amd import sof

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "sof.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sof_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_five_hot_path_calls():
    names = declared_functions()
    for n in ("sof_project", "sof_bin_sort", "sof_render_fwd", "sof_render_bwd", "sof_opacity_query"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(sof.LIB_PATH):
        pytest.fail("libsof.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(sof.LIB_PATH)
    for n in declared_functions():
        assert hasattr(L, n), n
    assert set(declared_functions()) == set(sof.EXPORTED)


def test_host_argument_checks():
    L = sof.lib()
    assert L.sof_strerror(sof.SOF_E_ARG) == b"invalid argument"
    cams = sof.Cameras.__new__(sof.Cameras)
    cam = (sof.CCamera * 1)()
    cam[0].fx = cam[0].fy = 50.0
    cam[0].width, cam[0].height = 64, 48
    p, b, g, r = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    o = sof.Options(tile=16, window=8, capacity=1000, order_slots=100).c_struct()
    hp = ctypes.cast(cam, ctypes.c_void_p)
    assert L.sof_workspace_size(100, hp, 1, ctypes.byref(o), ctypes.byref(p), ctypes.byref(b), ctypes.byref(g),
                                ctypes.byref(r)) == 0
    assert p.value > 0 and b.value > 0 and g.value == 1000 * 64
    # recorded order: a 256-byte aligned flag per tile (12 tiles of 16 x 16), then 2 bytes per
    # slot and tile-padded pixel
    assert r.value == 256 + 12 * 256 * 100 * 2
    none = sof.Options(tile=16, window=8, capacity=1000, order_slots=0).c_struct()
    assert L.sof_workspace_size(100, hp, 1, ctypes.byref(none), None, None, None, ctypes.byref(r)) == 0
    assert r.value == 0
    for slots in (-1, 4097):
        bad = sof.Options(tile=16, window=8, capacity=1000, order_slots=slots).c_struct()
        assert L.sof_workspace_size(100, hp, 1, ctypes.byref(bad), None, None, None, None) == sof.SOF_E_ARG
    bad = sof.Options(tile=12, window=8, capacity=1000).c_struct()
    assert L.sof_workspace_size(100, hp, 1, ctypes.byref(bad), None, None, None, None) == sof.SOF_E_ARG
    bad = sof.Options(tile=16, window=5, capacity=1000).c_struct()
    assert L.sof_workspace_size(100, hp, 1, ctypes.byref(bad), None, None, None, None) == sof.SOF_E_UNSUPPORTED
    assert L.sof_workspace_size(-1, hp, 1, ctypes.byref(o), None, None, None, None) == sof.SOF_E_ARG
    cam[0].width = 0
    assert L.sof_workspace_size(100, hp, 1, ctypes.byref(o), None, None, None, None) == sof.SOF_E_ARG
    cam[0].width = 64
    # binary-search step: empty input is a no-op, missing arrays or a negative size are rejected
    assert L.sof_bisect_step(None, None, None, None, 0, None) == sof.SOF_OK
    assert L.sof_bisect_step(None, None, None, None, 5, None) == sof.SOF_E_ARG
    assert L.sof_bisect_step(None, None, None, None, -1, None) == sof.SOF_E_ARG
    # 3D filter: no Gaussians is a no-op; a missing Gaussian set or a bad near plane is rejected
    gs = sof.CGaussians(0, 0, 0, None, None, None, None, None)
    assert L.sof_filter3d(ctypes.byref(gs), hp, None, 1, 0.2, 0.2, None, None, None, None) == sof.SOF_E_ARG
    assert L.sof_filter3d(ctypes.byref(gs), None, None, 0, 0.2, 0.2, None, None, None, None) == sof.SOF_OK
    assert L.sof_filter3d(None, None, None, 0, 0.2, 0.2, None, None, None, None) == sof.SOF_E_ARG
    assert L.sof_filter3d(ctypes.byref(gs), None, None, 0, 0.0, 0.2, None, None, None, None) == sof.SOF_E_ARG
    assert L.sof_filter3d_bwd(ctypes.byref(gs), None, None, None, None, None, None) == sof.SOF_OK
    # opacity pass: the forward's depth and aux are required
    assert L.sof_render_opacity(0, hp, hp, 1, ctypes.byref(o), None, 0, None, 0, None, None, None, None, 0, None,
                                None) == sof.SOF_E_ARG
    # backward: a normal gradient needs the forward's normal (checked before any launch; with
    # the normal given, the next check reached is the too-small partials buffer)
    fake = ctypes.c_void_p(256)
    big = ctypes.c_size_t(1 << 40)
    gs0 = sof.CGaussians(0, 0, 0, None, None, None, None, None)

    def bwd(normal, grads, grad_bytes, order=None, order_bytes=0, opts=o):
        return L.sof_render_bwd(ctypes.byref(gs0), hp, fake, 1, ctypes.byref(opts), None, 0, fake, big, fake, normal,
                                fake, order, order_bytes, fake, None, None, fake, None, None, None, None, None, grads,
                                grad_bytes, None, None, None, None, None, None)
    assert bwd(None, fake, big) == sof.SOF_E_ARG
    assert bwd(fake, fake, 0) == sof.SOF_E_WORKSPACE
    # a recorded order: smaller than its size, or given with order_slots = 0, is rejected
    L.sof_workspace_size(100, hp, 1, ctypes.byref(o), None, None, None, ctypes.byref(r))
    assert bwd(fake, fake, big, order=fake, order_bytes=r.value - 1) == sof.SOF_E_WORKSPACE
    assert bwd(fake, fake, big, order=fake, order_bytes=big, opts=none) == sof.SOF_E_ARG
    # the forward: the same checks, and a recorded order needs aux
    def fwd(order, order_bytes, aux, opts=o):
        return L.sof_render_fwd(0, hp, hp, 1, ctypes.byref(opts), None, 0, fake, big, None, None, None, None, aux,
                                None, order, order_bytes, None)
    assert fwd(fake, r.value - 1, fake) == sof.SOF_E_WORKSPACE
    assert fwd(fake, big, fake, opts=none) == sof.SOF_E_ARG
    assert fwd(fake, big, None) == sof.SOF_E_ARG


def test_render_order_argument_checks():
    """sof_render_order rejects a missing slot map, missing counts, negative sizes and null
    lists with max_entries > 0, before anything is enqueued."""
    L = sof.lib()
    cam = sof.CCamera()
    cam.R[:] = [1, 0, 0, 0, 1, 0, 0, 0, 1]
    cam.fx = cam.fy = 50.0
    cam.cx = cam.cy = 8.0
    cam.width = cam.height = 16
    hp = ctypes.cast(ctypes.pointer(cam), ctypes.c_void_p)
    o = sof.Options(tile=16, window=8, capacity=1024).c_struct()
    fake = ctypes.c_void_p(256)
    big = ctypes.c_size_t(1 << 40)

    def order(slot, n_slots, m, lists, counts):
        return L.sof_render_order(0, hp, hp, 1, ctypes.byref(o), None, 0, fake, big, slot, n_slots, m,
                                  lists, lists, lists, counts, None)
    assert order(None, 4, 8, fake, fake) == sof.SOF_E_ARG
    assert order(fake, -1, 8, fake, fake) == sof.SOF_E_ARG
    assert order(fake, 4, -1, fake, fake) == sof.SOF_E_ARG
    assert order(fake, 4, 8, None, fake) == sof.SOF_E_ARG
    assert order(fake, 4, 8, fake, None) == sof.SOF_E_ARG


def test_static_backward_rejects_capacity_above_its_scratch():
    """sof_render_bwd_static refuses a capacity above its fixed scratch before any device call."""
    L = sof.lib()
    o = sof.Options(tile=16, window=8, capacity=sof.STATIC_SCRATCH_INSTANCES + 1).c_struct()
    args = [None] * 29
    args[3], args[6], args[8], args[13] = 1, 0, 0, 0     # n_cams, proj_bytes, bins_bytes, order_bytes
    plain = list(args)
    args[4] = ctypes.byref(o)
    assert L.sof_render_bwd_static(*args) == sof.SOF_E_SCRATCH
    assert L.sof_render_bwd_static(*plain) == sof.SOF_E_ARG
    assert b"static scratch" in L.sof_strerror(sof.SOF_E_SCRATCH)
