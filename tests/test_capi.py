"""The C ABI on the CPU: the library loads, exports every function that
include/gdf.h declares, and rejects invalid arguments on the host before any
device work (no GPU needed)."""
import ctypes
import os
import re

import pytest

import paper_1506_02079_amd as gdf

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "gdf.h")


def _declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(\w+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "for", "sizeof")))


def test_exports_every_declared_function():
    names = _declared()
    assert {"fuse_stack", "solve_slices", "solve_slices_backward", "gdf_last_error"} <= set(names)
    L = gdf.lib()
    for n in names:
        assert hasattr(L, n), n
        assert n in gdf.SIGNATURES, n


def _fuse(**kw):
    a = dict(stack=1 << 20, S=4, H=32, W=32, pr=32, ps=32 * 32, alpha=0.01, bc=0, tol=1e-6,
             sxy=1.0, sz=3.0, f=1 << 21, gsm=None, opts=None, ws=1 << 22, wsb=16, rep=None)
    a.update(kw)
    o = a["opts"] or gdf.make_opts()
    return gdf.lib().fuse_stack(a["stack"], a["S"], a["H"], a["W"], a["pr"], a["ps"], a["alpha"],
                                a["bc"], a["tol"], a["sxy"], a["sz"], a["f"], a["gsm"],
                                ctypes.byref(o), a["ws"], a["wsb"], a["rep"], None)


def _robust(v, **kw):
    o = gdf.make_opts(**kw)
    o.robust = v
    return o


def _sor(**kw):
    o = gdf.make_opts(**kw)
    o.sor = 1
    return o


def _zr(z0, z1):
    o = gdf.make_opts()
    o.z_begin, o.z_end = z0, z1
    return o


@pytest.mark.parametrize("kw,status", [
    (dict(S=0), gdf.GDF_EINVAL),
    (dict(H=-1), gdf.GDF_EINVAL),
    # the widest slice is 4194304 columns (32-bit byte offsets within a row band)
    (dict(H=1, W=4194305, pr=4194305, ps=4194305), gdf.GDF_EINVAL),
    (dict(H=1, W=4194304, pr=4194304, ps=4194304, wsb=16), gdf.GDF_ENOMEM),
    (dict(stack=None), gdf.GDF_EINVAL),
    (dict(f=None), gdf.GDF_EINVAL),
    (dict(alpha=0.0), gdf.GDF_EINVAL),
    (dict(alpha=-1.0), gdf.GDF_EINVAL),
    (dict(alpha=float("nan")), gdf.GDF_EINVAL),
    (dict(alpha=float("inf")), gdf.GDF_EINVAL),
    (dict(tol=0.0), gdf.GDF_EINVAL),
    (dict(tol=1.5), gdf.GDF_EINVAL),
    (dict(bc=1, wsb=16), gdf.GDF_ENOMEM),   # periodic: valid, fails on the workspace
    (dict(bc=2), gdf.GDF_EUNSUPPORTED),
    (dict(bc=7), gdf.GDF_EINVAL),
    (dict(sxy=-1.0), gdf.GDF_EINVAL),
    (dict(sz=5.0), gdf.GDF_EUNSUPPORTED),
    (dict(pr=16), gdf.GDF_EINVAL),
    (dict(ps=100), gdf.GDF_EINVAL),
    (dict(opts=gdf.make_opts(nu=3)), gdf.GDF_EINVAL),
    (dict(opts=gdf.make_opts(precision=5)), gdf.GDF_EINVAL),
    (dict(opts=gdf.make_opts(tile_rows=7)), gdf.GDF_EINVAL),
    (dict(opts=gdf.make_opts(out_dtype=0 + 9)), gdf.GDF_EINVAL),
    (dict(opts=gdf.make_opts(launch_mode=3)), gdf.GDF_EINVAL),
    (dict(opts=gdf.make_opts(nu=2, fine_sweeps=3)), gdf.GDF_EINVAL),
    (dict(opts=gdf.make_opts(nu=2, fine_sweeps=7)), gdf.GDF_EINVAL),
    (dict(opts=gdf.make_opts(nu=1, fine_sweeps=5)), gdf.GDF_EINVAL),
    (dict(opts=gdf.make_opts(coarse_sweeps=4)), gdf.GDF_EINVAL),
    (dict(opts=gdf.make_opts(coarse_sweeps=-1)), gdf.GDF_EINVAL),
    (dict(opts=_robust(2)), gdf.GDF_EINVAL),
    (dict(opts=_robust(1, precision="fp64")), gdf.GDF_EUNSUPPORTED),
    (dict(opts=gdf.make_opts(launch_mode=-1)), gdf.GDF_EINVAL),
    (dict(ws=None), gdf.GDF_EINVAL),
    (dict(wsb=16), gdf.GDF_ENOMEM),
    # over-relaxed sweeps: FP32 hierarchies, 4 or 5 fused sweeps, Neumann
    (dict(opts=_sor(precision="fp64")), gdf.GDF_EUNSUPPORTED),
    (dict(opts=_sor(nu=2, fine_sweeps=6)), gdf.GDF_EUNSUPPORTED),
    (dict(opts=_sor(nu=1)), gdf.GDF_EUNSUPPORTED),            # (2 fused sweeps)
    (dict(opts=_sor(), bc=1), gdf.GDF_EUNSUPPORTED),
    (dict(opts=_sor(), wsb=16), gdf.GDF_ENOMEM),              # valid, fails on the workspace
    (dict(opts=_sor(nu=1, fine_sweeps=4, precision="mixed"), wsb=16), gdf.GDF_ENOMEM),
    # the slices to solve: [z_begin, z_end) of the S = 4
    (dict(opts=_zr(1, 1)), gdf.GDF_EINVAL),
    (dict(opts=_zr(2, 1)), gdf.GDF_EINVAL),
    (dict(opts=_zr(-1, 2)), gdf.GDF_EINVAL),
    (dict(opts=_zr(0, 5)), gdf.GDF_EINVAL),
    (dict(opts=_zr(1, 3), wsb=16), gdf.GDF_ENOMEM),   # valid, fails on the workspace
    # the autotuner validates first; every candidate then fails the workspace check
    (dict(wsb=16, opts=gdf.make_opts(autotune=True)), gdf.GDF_ENOMEM),
    (dict(alpha=0.0, opts=gdf.make_opts(autotune=True)), gdf.GDF_EINVAL),
])
def test_fuse_stack_rejects_on_host(kw, status):
    assert _fuse(**kw) == status
    assert gdf.last_error() != ""


def test_workspace_sizes():
    L = gdf.lib()
    o = gdf.make_opts()
    a = L.gdf_fuse_workspace_size(64, 2048, 2048, ctypes.byref(o))
    assert a > 64 * 2048 * 2048 * 12  # u (2 buffers) + b in FP32, plus coarse levels
    assert L.gdf_fuse_workspace_size(0, 2048, 2048, ctypes.byref(o)) == 0
    # solving 32 of the 64 slices takes about half the workspace; a bad range none
    o.z_begin, o.z_end = 16, 48
    h = L.gdf_fuse_workspace_size(64, 2048, 2048, ctypes.byref(o))
    assert 0.45 * a < h < 0.55 * a
    o.z_begin, o.z_end = 48, 16
    assert L.gdf_fuse_workspace_size(64, 2048, 2048, ctypes.byref(o)) == 0
    o.z_begin = o.z_end = 0
    d = (gdf.SliceDesc * 2)()
    for i, (H, W) in enumerate(((17, 33), (1, 1))):
        d[i].H, d[i].W, d[i].alpha = H, W, 0.01
        d[i].pitch_gs = d[i].pitch_go = d[i].pitch_f = W
    assert L.gdf_solve_workspace_size(2, d, ctypes.byref(o)) > 0
    d[1].alpha = -1.0
    assert L.gdf_solve_workspace_size(2, d, ctypes.byref(o)) == 0


def test_solve_slices_rejects_on_host():
    L = gdf.lib()
    o = gdf.make_opts()
    d = (gdf.SliceDesc * 1)()
    d[0].H, d[0].W, d[0].alpha = 8, 8, 0.01
    d[0].pitch_gs = d[0].pitch_go = d[0].pitch_f = 8
    call = lambda **k: L.solve_slices(1, d, k.get("gsd", 1), 1 << 20, k.get("god", 0), 1 << 21,
                                      k.get("bc", 0), k.get("tol", 1e-6), 1 << 22, ctypes.byref(o),
                                      1 << 23, 16, None, None)
    assert call(gsd=0) == gdf.GDF_EINVAL
    assert call(god=5) == gdf.GDF_EINVAL
    assert call(bc=1) == gdf.GDF_ENOMEM   # periodic boundaries are valid
    assert call(bc=2) == gdf.GDF_EUNSUPPORTED
    assert call(bc=3) == gdf.GDF_EINVAL
    assert call() == gdf.GDF_ENOMEM
    d[0].pitch_f = 4
    assert call() == gdf.GDF_EINVAL
    d[0].pitch_f = 8
    d[0].off_go = -3
    assert call() == gdf.GDF_EINVAL
    d[0].off_go = 0
    # FP64 data needs the FP64 solver; every call here fails validation before
    # any device work (the pointers are placeholders)
    om = gdf.make_opts(precision="mixed")
    assert L.solve_slices_backward(1, d, 2, 1 << 20, 1 << 21, 1 << 22, 0, 1e-6, None, None, None, None,
                                   ctypes.byref(om), 1 << 23, 1 << 30, None, None) == gdf.GDF_EINVAL
    assert L.solve_slices_backward(1, d, 1, 1 << 20, 1 << 21, 1 << 22, 0, 1e-6, None, None, None, None,
                                   ctypes.byref(om), 1 << 23, 16, None, None) == gdf.GDF_ENOMEM


def test_autotune_flag_and_workspace():
    L = gdf.lib()
    o = gdf.make_opts()
    o.autotune = 2
    assert _fuse(opts=o) == gdf.GDF_EINVAL
    plain = L.gdf_fuse_workspace_size(8, 1000, 700, ctypes.byref(gdf.make_opts()))
    tuned = L.gdf_fuse_workspace_size(8, 1000, 700, ctypes.byref(gdf.make_opts(autotune=True)))
    small = L.gdf_fuse_workspace_size(8, 1000, 700, ctypes.byref(gdf.make_opts(tile_rows=32)))
    # candidates include 32-row items (more items, larger work tables)
    assert tuned >= max(plain, small) > 0


def test_streamed_rejects_device_or_float_stacks():
    import torch
    with pytest.raises(ValueError):
        gdf.fuse_stack_streamed(torch.zeros((2, 8, 8), dtype=torch.float32), 0.01)
    with pytest.raises(ValueError):
        gdf.fuse_stack_streamed(torch.zeros((2, 8, 8), dtype=torch.uint8), 0.01, chunk=0)
    with pytest.raises(ValueError):
        gdf.fuse_stack_streamed(torch.zeros((2, 8, 8), dtype=torch.uint8), 0.01, return_smooth=True)


def test_noalloc_rejects_on_host():
    # checks that return before any device work: a batch larger than the
    # static scratch, and graph capture (whose instantiation allocates)
    L = gdf.lib()
    d = (gdf.SliceDesc * 1)()
    d[0].H, d[0].W, d[0].alpha = 8192, 8192, 0.01
    d[0].pitch_gs = d[0].pitch_go = d[0].pitch_f = 8192
    o = gdf.make_opts()
    call = lambda o: L.solve_slices_noalloc(1, d, 1, 1 << 20, 0, 1 << 21, 0, 1e-6, 1 << 22, ctypes.byref(o),
                                            None, None)
    assert call(o) == gdf.GDF_ENOMEM
    assert "scratch" in gdf.last_error()
    assert call(gdf.make_opts(use_graph=True)) == gdf.GDF_EUNSUPPORTED
    d[0].alpha = -1.0
    assert call(o) == gdf.GDF_EINVAL
