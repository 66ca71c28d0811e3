"""Gradient-domain fusion of EM image stacks on MI355X (gfx950).

Python binding of ``libgdf.so`` (C ABI in ``include/gdf.h``).  This module
only marshals arguments: torch tensors provide device memory and the current
HIP stream; every step of the method runs in the library's HIP kernels.  If
the library is not built, calls raise immediately -- there is no CPU path.

Method (Kazhdan et al., arXiv 1506.02079): smooth the stack across slices
with an anisotropic Gaussian (Section III-A), then solve per slice the
screened-Poisson blend of Eq. (1), (alpha - Laplacian) f = alpha g_s -
Laplacian g_o, to a relative residual tolerance.
"""
from __future__ import annotations

import ctypes

import numpy as np
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgdf.so")

GDF_OK, GDF_EINVAL, GDF_EUNSUPPORTED, GDF_ENOMEM, GDF_EDEVICE, GDF_ENOCONV, GDF_ENONFINITE = range(7)
STATUS_NAMES = {0: "GDF_OK", 1: "GDF_EINVAL", 2: "GDF_EUNSUPPORTED", 3: "GDF_ENOMEM",
                4: "GDF_EDEVICE", 5: "GDF_ENOCONV", 6: "GDF_ENONFINITE"}
BC = {"neumann": 0, "periodic": 1, "dirichlet": 2}
DTYPE_U8, DTYPE_F32, DTYPE_F64 = 0, 1, 2
PRECISION = {"fp32": 0, "fp64": 1, "mixed": 2}
LAUNCH = {"default": 0, "grid": 1, "persistent": 2}


class GdfError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


class SolveOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("max_vcycles", ctypes.c_int), ("nu", ctypes.c_int),
                ("out_dtype", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("tile_rows", ctypes.c_int), ("inner_cycles", ctypes.c_int),
                ("launch_mode", ctypes.c_int), ("autotune", ctypes.c_int),
                ("fine_sweeps", ctypes.c_int), ("coarse_sweeps", ctypes.c_int),
                ("robust", ctypes.c_int), ("z_begin", ctypes.c_int), ("z_end", ctypes.c_int),
                ("sor", ctypes.c_int), ("reserved", ctypes.c_int * 1)]


class SliceReport(ctypes.Structure):
    _fields_ = [("vcycles", ctypes.c_int), ("status", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("rel_residual_init", ctypes.c_double)]


class SliceDesc(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int), ("W", ctypes.c_int), ("alpha", ctypes.c_double),
                ("off_gs", ctypes.c_longlong), ("pitch_gs", ctypes.c_longlong),
                ("off_go", ctypes.c_longlong), ("pitch_go", ctypes.c_longlong),
                ("off_f", ctypes.c_longlong), ("pitch_f", ctypes.c_longlong)]


_lib = None

# exported symbols, with their ctypes signatures
_P, _I, _D, _L, _S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong, ctypes.c_size_t
SIGNATURES = {
    "gdf_last_error": ([], ctypes.c_char_p),
    "gdf_version": ([], ctypes.c_char_p),
    "gdf_release": ([], None),
    "gdf_autotune_last": ([ctypes.POINTER(SolveOpts)], _I),
    "gdf_profile_enable": ([_I], None),
    "gdf_profile_reset": ([], None),
    "gdf_profile_read": ([ctypes.c_char_p, ctypes.POINTER(_D), ctypes.POINTER(_D)], _I),
    "gdf_fuse_workspace_size": ([_I, _I, _I, ctypes.POINTER(SolveOpts)], _S),
    "fuse_stack": ([_P, _I, _I, _I, _L, _L, _D, _I, _D, _D, _D, _P, _P, ctypes.POINTER(SolveOpts),
                    _P, _S, ctypes.POINTER(SliceReport), _P], _I),
    "gdf_solve_workspace_size": ([_I, ctypes.POINTER(SliceDesc), ctypes.POINTER(SolveOpts)], _S),
    "solve_slices": ([_I, ctypes.POINTER(SliceDesc), _I, _P, _I, _P, _I, _D, _P,
                      ctypes.POINTER(SolveOpts), _P, _S, ctypes.POINTER(SliceReport), _P], _I),
    "gdf_backward_workspace_size": ([_I, ctypes.POINTER(SliceDesc), ctypes.POINTER(SolveOpts)], _S),
    "solve_slices_backward": ([_I, ctypes.POINTER(SliceDesc), _I, _P, _P, _P, _I, _D, _P, _P,
                               ctypes.POINTER(_D), _P, ctypes.POINTER(SolveOpts), _P, _S,
                               ctypes.POINTER(SliceReport), _P], _I),
    "solve_slices_noalloc": ([_I, ctypes.POINTER(SliceDesc), _I, _P, _I, _P, _I, _D, _P,
                              ctypes.POINTER(SolveOpts), ctypes.POINTER(SliceReport), _P], _I),
    "gdf_smooth_transpose_workspace_size": ([_I, _I, _I], _S),
    "smooth_transpose": ([_P, _I, _I, _I, _D, _D, _P, _P, _P, _S, _P], _I),
}


def lib():
    """The loaded C library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libgdf.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def last_error() -> str:
    return lib().gdf_last_error().decode()


def version() -> str:
    return lib().gdf_version().decode()


def make_opts(precision="fp32", max_vcycles=0, nu=0, out_dtype=None, use_graph=False,
              tile_rows=0, inner_cycles=0, launch_mode=0, autotune=False, fine_sweeps=0,
              coarse_sweeps=0, sor=False) -> SolveOpts:
    o = SolveOpts()
    o.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    o.max_vcycles = int(max_vcycles)
    o.nu = int(nu)
    o.out_dtype = 0 if out_dtype is None else int(out_dtype)
    o.use_graph = int(bool(use_graph))
    o.tile_rows = int(tile_rows)
    o.inner_cycles = int(inner_cycles)
    o.launch_mode = LAUNCH[launch_mode] if isinstance(launch_mode, str) else int(launch_mode)
    o.autotune = int(bool(autotune))
    o.fine_sweeps = int(fine_sweeps)
    o.coarse_sweeps = int(coarse_sweeps)
    o.sor = int(bool(sor))
    return o


def autotune_last():
    """Settings chosen by the last autotuned call on this thread, or None:
    dict(nu, fine_sweeps, coarse_sweeps, tile_rows, launch_mode, sor)."""
    o = SolveOpts()
    if not lib().gdf_autotune_last(ctypes.byref(o)):
        return None
    return dict(nu=o.nu, fine_sweeps=o.fine_sweeps, coarse_sweeps=o.coarse_sweeps, tile_rows=o.tile_rows,
                launch_mode=o.launch_mode, sor=bool(o.sor))


def _check(status, allow_noconv=False):
    if status == GDF_OK or (allow_noconv and status in (GDF_ENOCONV, GDF_ENONFINITE)):
        return
    raise GdfError(status, last_error())


def _report_list(rep, n):
    return [dict(vcycles=rep[i].vcycles, status=rep[i].status, rel_residual=rep[i].rel_residual,
                 rel_residual_init=rep[i].rel_residual_init) for i in range(n)]


def _torch():
    import torch
    return torch


def _stream(dev):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


_SIDE = {}


def _side_stream(dev):
    torch = _torch()
    key = str(dev)
    if key not in _SIDE:
        _SIDE[key] = torch.cuda.Stream(device=dev)   # default priority
    return _SIDE[key]


def _on_side_stream(dev, call, tensors):
    """Runs call() (a library call on _stream(dev)) on a side stream ordered
    after the caller's current stream and joined back after it: stream
    capture needs a stream other than the default one."""
    torch = _torch()
    cur = torch.cuda.current_stream(dev)
    side = _side_stream(dev)
    side.wait_stream(cur)
    with torch.cuda.stream(side):
        st = call()
    cur.wait_stream(side)
    for t in tensors:
        t.record_stream(side)
    return st


def _dtype_code(t):
    torch = _torch()
    return {torch.uint8: DTYPE_U8, torch.float32: DTYPE_F32, torch.float64: DTYPE_F64}[t.dtype]


def _require_cuda(*ts):
    for t in ts:
        if not t.is_cuda:
            raise ValueError("tensors must live on the GPU (got %s)" % t.device)


# ------------------------------------------------------------------ fuse_stack

def fuse_stack(stack, alpha, bc="neumann", tol=1e-6, sigma_xy=1.0, sigma_z=3.0,
               precision="fp32", out_dtype=None, return_smooth=False, nu=0, max_vcycles=0,
               tile_rows=0, inner_cycles=0, launch_mode=0, autotune=False, fine_sweeps=0, coarse_sweeps=0,
               allow_noconv=False, robust=False, z_range=None, use_graph=False, wait=True, sor=False):
    """Smooth a uint8 stack [S, H, W] across slices and blend each slice (Eq. (1)).
    sor=True: over-relaxed sweeps in the fused finest passes (fine_sweeps 4 or 5).
    robust=True: robust cross-slice averaging (values more than two weighted
    standard deviations from the window's weighted mean are left out).
    z_range=(z0, z1): solve only slices z0 .. z1 - 1 (the others only enter
    their cross-slice windows); f, g_smooth and the report then hold z1 - z0
    slices.  use_graph=True: the whole schedule (smoothing and every V-cycle,
    with the convergence test on the device) is captured once per shape,
    pointers and options, then replayed; the host waits only for the report.
    use_graph=True, wait=False: asynchronous; the call returns (f, None) once
    the work is enqueued on the current stream (no report, no per-slice check).

    Returns (f, report) or (f, report, g_smooth) with return_smooth=True.
    f has dtype float32 (fp32) or float64 (fp64 / mixed) unless out_dtype is given.
    """
    torch = _torch()
    _require_cuda(stack)
    if stack.dtype != torch.uint8 or stack.dim() != 3:
        raise ValueError("stack must be a uint8 tensor [S, H, W]")
    if stack.stride(2) != 1:
        stack = stack.contiguous()
    S, H, W = stack.shape
    o = make_opts(precision, max_vcycles, nu, out_dtype, use_graph, tile_rows, inner_cycles,
                  launch_mode, autotune, fine_sweeps, coarse_sweeps, sor)
    o.robust = int(bool(robust))
    n = S
    if z_range is not None:
        o.z_begin, o.z_end = int(z_range[0]), int(z_range[1])
        n = o.z_end - o.z_begin
    L = lib()
    ws = L.gdf_fuse_workspace_size(S, H, W, ctypes.byref(o))
    if ws == 0:
        raise GdfError(GDF_EINVAL, last_error())
    od = o.out_dtype or (DTYPE_F32 if o.precision == 0 else DTYPE_F64)
    f = torch.empty((n, H, W), dtype=torch.float64 if od == DTYPE_F64 else torch.float32,
                    device=stack.device)
    gsm = None
    if return_smooth:
        gsm = torch.empty((n, H, W), dtype=torch.float64 if o.precision == 1 else torch.float32,
                          device=stack.device)
    if not wait and not use_graph:
        raise ValueError("wait=False needs use_graph=True (the eager schedule reads flags every cycle)")
    work = torch.empty(ws, dtype=torch.uint8, device=stack.device)
    rep = (SliceReport * n)() if wait else None
    call = lambda: L.fuse_stack(stack.data_ptr(), S, H, W, stack.stride(1), stack.stride(0), float(alpha),
                                BC[bc], float(tol), float(sigma_xy), float(sigma_z), f.data_ptr(),
                                gsm.data_ptr() if gsm is not None else None, ctypes.byref(o),
                                work.data_ptr(), ws, rep, _stream(stack.device))
    if use_graph:
        st = _on_side_stream(stack.device, call, [t for t in (work, stack, f, gsm) if t is not None])
    else:
        st = call()
    _check(st, allow_noconv)
    out = (f, _report_list(rep, n) if wait else None)
    return out + (gsm,) if return_smooth else out


# ---------------------------------------------------------------- solve_slices

def _descs(gs_list, go_list, f_list, alphas):
    """Slice descriptors for lists of 2D tensors, offsets from each list's lowest address."""
    n = len(gs_list)
    d = (SliceDesc * n)()
    bases = []
    for lst in (gs_list, go_list, f_list):
        base = min(t.data_ptr() for t in lst)
        bases.append(base)
    for i in range(n):
        H, W = gs_list[i].shape
        d[i].H, d[i].W, d[i].alpha = H, W, float(alphas[i])
        for k, (lst, name) in enumerate(((gs_list, "gs"), (go_list, "go"), (f_list, "f"))):
            t = lst[i]
            if t.stride(1) != 1:
                raise ValueError("slices must have unit column stride")
            diff = t.data_ptr() - bases[k]
            if diff % t.element_size():
                raise ValueError("misaligned slice buffer")
            setattr(d[i], "off_" + name, diff // t.element_size())
            setattr(d[i], "pitch_" + name, t.stride(0))
    return d, bases


def solve_slices(g_s, g_o, alpha, bc="neumann", tol=1e-6, precision="fp32", out_dtype=None,
                 nu=0, max_vcycles=0, use_graph=False, tile_rows=0, inner_cycles=0,
                 launch_mode=0, autotune=False, fine_sweeps=0, coarse_sweeps=0, allow_noconv=False, sor=False):
    """Eq. (1) per slice.  g_s, g_o: [S, H, W] tensors or lists of 2D tensors
    (uneven batch).  alpha: scalar or per-slice sequence.  Returns (f, report)
    with f shaped like the input (a list for list input)."""
    torch = _torch()
    as_list = isinstance(g_s, (list, tuple))
    gs_list = list(g_s) if as_list else list(g_s.unbind(0))
    go_list = list(g_o) if as_list else list(g_o.unbind(0))
    n = len(gs_list)
    if len(go_list) != n:
        raise ValueError("g_s and g_o must have the same number of slices")
    if not as_list and g_s.shape != g_o.shape:
        raise ValueError("g_s and g_o shapes differ")
    for a, b in zip(gs_list, go_list):
        if a.shape != b.shape or a.dim() != 2:
            raise ValueError("each slice pair must be 2D with equal shapes")
    _require_cuda(*gs_list, *go_list)
    gdt = {gs_list[0].dtype}
    if len({t.dtype for t in gs_list}) != 1 or len({t.dtype for t in go_list}) != 1:
        raise ValueError("all g_s slices (and all g_o slices) must share a dtype")
    alphas = [float(alpha)] * n if not hasattr(alpha, "__len__") else [float(a) for a in alpha]
    o = make_opts(precision, max_vcycles, nu, out_dtype, use_graph, tile_rows, inner_cycles,
                  launch_mode, autotune, fine_sweeps, coarse_sweeps, sor)
    od = o.out_dtype or (DTYPE_F32 if o.precision == 0 else DTYPE_F64)
    fdt = torch.float64 if od == DTYPE_F64 else torch.float32
    dev = gs_list[0].device
    if as_list:
        tot = sum(t.numel() for t in gs_list)
        flat = torch.empty(tot, dtype=fdt, device=dev)
        f_list, off = [], 0
        for t in gs_list:
            f_list.append(flat[off:off + t.numel()].view(t.shape))
            off += t.numel()
    else:
        f_all = torch.empty(g_s.shape, dtype=fdt, device=dev)
        f_list = list(f_all.unbind(0))
    d, bases = _descs(gs_list, go_list, f_list, alphas)
    L = lib()
    ws = L.gdf_solve_workspace_size(n, d, ctypes.byref(o))
    if ws == 0:
        raise GdfError(GDF_EINVAL, last_error())
    work = torch.empty(ws, dtype=torch.uint8, device=dev)
    rep = (SliceReport * n)()
    if use_graph:
        st = _on_side_stream(dev, lambda: L.solve_slices(n, d, _dtype_code(gs_list[0]), bases[0],
                                                         _dtype_code(go_list[0]), bases[1], BC[bc], float(tol),
                                                         bases[2], ctypes.byref(o), work.data_ptr(), ws, rep,
                                                         _stream(dev)),
                             [work, *gs_list, *go_list, *f_list])
    else:
        st = L.solve_slices(n, d, _dtype_code(gs_list[0]), bases[0], _dtype_code(go_list[0]),
                            bases[1], BC[bc], float(tol), bases[2], ctypes.byref(o),
                            work.data_ptr(), ws, rep, _stream(dev))
    _check(st, allow_noconv)
    del gdt
    return (f_list if as_list else f_all), _report_list(rep, n)


def solve_slices_backward(grad_f, f, g_s, alpha, bc="neumann", tol=1e-6, precision=None, nu=0,
                          max_vcycles=0, need=(True, True, True), tile_rows=0, launch_mode=0,
                          autotune=False, fine_sweeps=0, coarse_sweeps=0, allow_noconv=False,
                          alpha_sum=False):
    """Adjoint of Eq. (1): returns (dL/dg_s, dL/dg_o, dL/dalpha, report) for
    grad_f = dL/df.  Tensors are [S, H, W] of one float dtype.  dL/dalpha is a
    float64 CPU tensor of the per-slice terms, or with alpha_sum=True a float64
    device tensor holding their sum (formed by the library on the device: the
    gradient of one alpha shared by every slice)."""
    torch = _torch()
    _require_cuda(grad_f, f, g_s)
    if not (grad_f.shape == f.shape == g_s.shape) or grad_f.dim() != 3:
        raise ValueError("grad_f, f and g_s must be [S, H, W] of equal shapes")
    dt = grad_f.dtype
    if f.dtype != dt or g_s.dtype != dt or dt not in (torch.float32, torch.float64):
        raise ValueError("grad_f, f and g_s must share float32 or float64 dtype")
    grad_f, f, g_s = grad_f.contiguous(), f.contiguous(), g_s.contiguous()
    S, H, W = grad_f.shape
    prec = precision or ("fp64" if dt == torch.float64 else "fp32")
    alphas = [float(alpha)] * S if not hasattr(alpha, "__len__") else [float(a) for a in alpha]
    d = (SliceDesc * S)()
    for i in range(S):
        d[i].H, d[i].W, d[i].alpha = H, W, alphas[i]
        d[i].off_gs = d[i].off_go = d[i].off_f = i * H * W
        d[i].pitch_gs = d[i].pitch_go = d[i].pitch_f = W
    o = make_opts(prec, max_vcycles, nu, None, False, tile_rows, 0, launch_mode, autotune, fine_sweeps,
                  coarse_sweeps)
    L = lib()
    ws = L.gdf_backward_workspace_size(S, d, ctypes.byref(o))
    if ws == 0:
        raise GdfError(GDF_EINVAL, last_error())
    work = torch.empty(ws, dtype=torch.uint8, device=grad_f.device)
    ggs = torch.empty_like(grad_f) if need[0] else None
    ggo = torch.empty_like(grad_f) if need[1] else None
    ga = (ctypes.c_double * S)()
    gsum = torch.empty((), dtype=torch.float64, device=grad_f.device) if (need[2] and alpha_sum) else None
    rep = (SliceReport * S)()
    st = L.solve_slices_backward(S, d, _dtype_code(grad_f), grad_f.data_ptr(), f.data_ptr(),
                                 g_s.data_ptr(), BC[bc], float(tol),
                                 ggs.data_ptr() if ggs is not None else None,
                                 ggo.data_ptr() if ggo is not None else None,
                                 ga if (need[2] and not alpha_sum) else None,
                                 gsum.data_ptr() if gsum is not None else None, ctypes.byref(o),
                                 work.data_ptr(), ws, rep, _stream(grad_f.device))
    _check(st, allow_noconv)
    if gsum is not None:
        galpha = gsum
    else:
        galpha = torch.tensor([ga[i] for i in range(S)], dtype=torch.float64) if need[2] else None
    return ggs, ggo, galpha, _report_list(rep, S)


def smooth_transpose(grad, sigma_xy=1.0, sigma_z=3.0, add=None):
    """Transpose of the smoothing: dLoss/dstack for grad = dLoss/d(smoothed
    stack), FP32 [S, H, W] (see smooth_transpose in include/gdf.h).  add: an
    FP32 [S, H, W] tensor the library adds to the result in place (it is
    returned)."""
    torch = _torch()
    _require_cuda(grad)
    if grad.dim() != 3:
        raise ValueError("grad must be [S, H, W]")
    g = grad.to(torch.float32).contiguous()
    S, H, W = g.shape
    L = lib()
    ws = L.gdf_smooth_transpose_workspace_size(S, H, W)
    if ws == 0:
        raise GdfError(GDF_EINVAL, "S, H, W must be >= 1")
    work = torch.empty(ws, dtype=torch.uint8, device=g.device)
    if add is not None:
        if add.dtype != torch.float32 or tuple(add.shape) != (S, H, W) or not add.is_contiguous():
            raise ValueError("add must be a contiguous float32 [S, H, W] tensor")
        out = add
    else:
        out = torch.empty_like(g)
    st = L.smooth_transpose(g.data_ptr(), S, H, W, float(sigma_xy), float(sigma_z), out.data_ptr(),
                            out.data_ptr() if add is not None else None, work.data_ptr(), ws, _stream(g.device))
    _check(st)
    return out


def fuse_stack_backward(grad_f, f, stack, alpha, sigma_xy=1.0, sigma_z=3.0, tol=1e-6, **kw):
    """Gradient of a loss through fuse_stack with respect to the stack, the stack
    taken as real-valued: dLoss/dstack = smooth_transpose(dLoss/dg_s) + dLoss/dg_o,
    with dLoss/dg_s and dLoss/dg_o from the adjoint solve (solve_slices_backward).
    grad_f, f: FP32 [S, H, W]; returns (dLoss/dstack FP32, report)."""
    torch = _torch()
    g32 = grad_f.to(torch.float32).contiguous()
    f32 = f.to(torch.float32).contiguous()
    # (g_s only enters dLoss/dalpha, which is not asked for); the library adds
    # the transposed smoothing of dLoss/dg_s into dLoss/dg_o in place
    ggs, ggo, _, rep = solve_slices_backward(g32, f32, f32, alpha, tol=tol, need=(True, True, False), **kw)
    return smooth_transpose(ggs, sigma_xy, sigma_z, add=ggo), rep


def fuse_color(color, grey, alpha, tol=1e-6, **kw):
    """Fusion of a low-frequency colour image with a high-frequency grey one
    ("Extensions and Applications"): each channel c solves Eq. (1) with the
    channel as the value constraint and the grey image's gradients,
    (alpha I + L) f_c = alpha color_c + L grey, as one batch of solve_slices.
    color: [C, H, W], grey: [H, W] (float32 or float64, on the GPU); returns
    (f [C, H, W], report)."""
    torch = _torch()
    _require_cuda(color, grey)
    if color.dim() != 3 or grey.dim() != 2 or tuple(color.shape[1:]) != tuple(grey.shape):
        raise ValueError("color must be [C, H, W] and grey [H, W] of the same H, W")
    C = color.shape[0]
    go = grey.to(color.dtype).contiguous()
    return solve_slices([color[c] for c in range(C)], [go] * C, alpha, tol=tol, **kw)


def fuse_stack_streamed(stack, alpha, chunk=32, out=None, sigma_xy=1.0, sigma_z=3.0, tol=1e-6, **kw):
    """fuse_stack for stacks kept in host memory (larger than HBM).

    stack: uint8 [S, H, W] CPU tensor (pinned, for overlapped uploads).  Slices
    are processed `chunk` at a time; each chunk is uploaded with the
    floor(3 sigma_z) slices on either side that its smoothing reads, so every
    slice's result equals the whole-stack one (the solve is per slice; the
    slices on either side only enter the windows: z_range).  The next chunk's upload runs on a side
    stream while the current chunk computes, and each chunk's result goes back
    on a third stream while the next one computes.  Returns (f float32 [S, H, W] in
    pinned host memory, or `out`; the per-slice reports)."""
    torch = _torch()
    if stack.device.type != "cpu" or stack.dtype != torch.uint8 or stack.dim() != 3:
        raise ValueError("stack must be a uint8 [S, H, W] tensor in host memory")
    if chunk < 1:
        raise ValueError("chunk must be >= 1")
    if kw.get("return_smooth"):
        raise ValueError("fuse_stack_streamed does not return the smoothed stack")
    S, H, W = stack.shape
    rz = int(np.floor(3.0 * sigma_z)) if sigma_z > 0 else 0
    dev = torch.device("cuda", torch.cuda.current_device())
    if out is None:
        out = torch.empty((S, H, W), dtype=torch.float32, pin_memory=True)
    span = min(S, chunk + 2 * rz)
    bufs = [torch.empty((span, H, W), dtype=torch.uint8, device=dev) for _ in range(2)]
    freed = [torch.cuda.Event(), torch.cuda.Event()]   # chunk done with a buffer
    ready = [torch.cuda.Event(), torch.cuda.Event()]   # upload landed
    copy = torch.cuda.Stream(device=dev)               # uploads (default priority)
    down = torch.cuda.Stream(device=dev)               # downloads (default priority)
    main = torch.cuda.current_stream(dev)
    starts = list(range(0, S, chunk))
    reports = []

    def upload(c):
        z0 = starts[c]
        lo, hi = max(z0 - rz, 0), min(z0 + chunk + rz, S)
        b = c % 2
        with torch.cuda.stream(copy):
            if c >= 2:
                copy.wait_event(freed[b])
            bufs[b][:hi - lo].copy_(stack[lo:hi], non_blocking=True)
            ready[b].record(copy)

    upload(0)
    for c, z0 in enumerate(starts):
        if c + 1 < len(starts):
            upload(c + 1)
        b = c % 2
        z1 = min(z0 + chunk, S)
        lo, hi = max(z0 - rz, 0), min(z0 + chunk + rz, S)
        main.wait_event(ready[b])
        f, rep = fuse_stack(bufs[b][:hi - lo], alpha, tol=tol, sigma_xy=sigma_xy, sigma_z=sigma_z,
                            z_range=(z0 - lo, z1 - lo), **kw)
        freed[b].record(main)
        down.wait_stream(main)
        with torch.cuda.stream(down):
            out[z0:z1].copy_(f, non_blocking=True)
        f.record_stream(down)      # the allocator keeps f until the download ends
        reports += rep
    torch.cuda.synchronize(dev)
    return out, reports


def _make_autograd():
    torch = _torch()

    class ScreenedPoissonSolve(torch.autograd.Function):
        """f = solve of Eq. (1) per slice, differentiable in g_s, g_o and alpha.

        apply(g_s, g_o, alpha, tol=1e-6): g_s, g_o float tensors [S, H, W] on the
        GPU (same dtype; float64 runs the FP64 solver); alpha a scalar tensor
        (shared by all slices) or a 1D tensor of per-slice weights.
        """

        @staticmethod
        def forward(ctx, g_s, g_o, alpha, tol=1e-6):
            prec = "fp64" if g_s.dtype == torch.float64 else "fp32"
            a = alpha.detach().double().cpu()
            al = a.tolist() if a.dim() else float(a)
            f, _ = solve_slices(g_s.detach(), g_o.detach(), al, tol=tol, precision=prec,
                                out_dtype=DTYPE_F64 if prec == "fp64" else DTYPE_F32)
            ctx.save_for_backward(g_s, f, alpha)
            ctx.al = al
            ctx.tol = tol
            return f

        @staticmethod
        def backward(ctx, grad_f):
            g_s, f, alpha = ctx.saved_tensors
            need = ctx.needs_input_grad
            # a scalar alpha's gradient is the library's device sum over the slices
            ggs, ggo, ga, _ = solve_slices_backward(grad_f.contiguous().to(f.dtype), f, g_s.detach(),
                                                    ctx.al, tol=ctx.tol,
                                                    need=(need[0], need[1], need[2]),
                                                    alpha_sum=alpha.dim() == 0)
            galpha = None
            if need[2]:
                galpha = ga.to(dtype=alpha.dtype, device=alpha.device)
            return ggs, ggo, galpha, None

    return ScreenedPoissonSolve


class _Lazy:
    _cls = None

    def __get__(self, obj, owner):
        if _Lazy._cls is None:
            _Lazy._cls = _make_autograd()
        return _Lazy._cls


class _Namespace:
    ScreenedPoissonSolve = _Lazy()


def __getattr__(name):
    if name == "ScreenedPoissonSolve":
        return _Namespace.ScreenedPoissonSolve
    raise AttributeError(name)


# ------------------------------------------------------------------ profiling

def profile_enable(on=True, fine_only=False):
    """Time kernel classes with HIP events (fine_only: only "vcycle_fine")."""
    lib().gdf_profile_enable(0 if not on else (2 if fine_only else 1))


def profile_reset():
    lib().gdf_profile_reset()


def profile_read(kernel_class):
    """(launches, total_ms, algorithmic_bytes) recorded for a kernel class."""
    ms = ctypes.c_double(0.0)
    by = ctypes.c_double(0.0)
    n = lib().gdf_profile_read(kernel_class.encode(), ctypes.byref(ms), ctypes.byref(by))
    return n, ms.value, by.value
