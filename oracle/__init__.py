"""FP64 CPU oracle (test infrastructure only).

A plain, slow, obviously correct implementation of what the fusion path
computes, in double precision: the truncated, renormalised anisotropic
Gaussian smoothing (Section III-A and the Implementation subsection) and the
per-slice screened-Poisson solve of Eq. (1) by unpreconditioned conjugate
gradients, plus the relative residual and the adjoint.  The arithmetic lives
in ``oracle.c`` (built with gcc into ``liboracle.so``); this module only
marshals numpy arrays.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU
library.  Every function is pinned by the CPU tests against closed forms,
brute force or invariants (tests/test_oracle_*.py); none is "parity
unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BC_NEUMANN = 0
BC_PERIODIC = 1
_BC = {"neumann": BC_NEUMANN, "periodic": BC_PERIODIC}

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (OpenMP, no fast-math) into liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        L = ctypes.c_longlong
        lib.oracle_threads.argtypes = []
        lib.oracle_threads.restype = I
        lib.oracle_smooth_voxel.argtypes = [P, I, I, I, D, D, I, I, I]
        lib.oracle_smooth_voxel.restype = D
        lib.oracle_smooth.argtypes = [P, I, I, I, D, D, P]
        lib.oracle_smooth.restype = None
        lib.oracle_smooth_points.argtypes = [P, I, I, I, D, D, P, L, P]
        lib.oracle_smooth_points.restype = None
        lib.oracle_smooth_robust_points.argtypes = [P, I, I, I, D, D, P, L, P]
        lib.oracle_smooth_robust_points.restype = None
        lib.oracle_smooth_robust.argtypes = [P, I, I, I, D, D, P]
        lib.oracle_smooth_robust.restype = None
        lib.oracle_smooth_transpose.argtypes = [P, I, I, I, D, D, P]
        lib.oracle_smooth_transpose.restype = None
        lib.oracle_laplacian.argtypes = [P, I, I, I, P]
        lib.oracle_laplacian.restype = None
        lib.oracle_apply_A.argtypes = [P, I, I, D, I, P]
        lib.oracle_apply_A.restype = None
        lib.oracle_rhs.argtypes = [P, P, I, I, D, I, P]
        lib.oracle_rhs.restype = None
        lib.oracle_cg.argtypes = [P, I, I, D, I, D, I, P, P]
        lib.oracle_cg.restype = I
        lib.oracle_solve.argtypes = [P, P, I, I, D, I, D, I, P, P]
        lib.oracle_solve.restype = I
        lib.oracle_relres.argtypes = [P, P, P, I, I, D, I]
        lib.oracle_relres.restype = D
        lib.oracle_adjoint.argtypes = [P, P, P, I, I, D, I, D, I, P, P, P]
        lib.oracle_adjoint.restype = I
        _lib = lib
    return _lib


def threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(_load().oracle_threads())


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _bc(bc) -> int:
    return _BC[bc] if isinstance(bc, str) else int(bc)


# ------------------------------------------------------------------ smoothing

def smooth(stack: np.ndarray, sigma_xy: float = 1.0, sigma_z: float = 3.0) -> np.ndarray:
    """I1 = I0 * G (truncated at 3 sigma per axis, renormalised), float64 [S][H][W]."""
    st = np.ascontiguousarray(stack, dtype=np.uint8)
    S, H, W = st.shape
    out = np.empty((S, H, W), dtype=np.float64)
    _load().oracle_smooth(_ptr(st), S, H, W, float(sigma_xy), float(sigma_z), _ptr(out))
    return out


def smooth_points(stack: np.ndarray, zyx: np.ndarray, sigma_xy: float = 1.0,
                  sigma_z: float = 3.0) -> np.ndarray:
    """I1 at the given (z, y, x) voxels."""
    st = np.ascontiguousarray(stack, dtype=np.uint8)
    S, H, W = st.shape
    pts = np.ascontiguousarray(zyx, dtype=np.int32).reshape(-1, 3)
    out = np.empty(len(pts), dtype=np.float64)
    _load().oracle_smooth_points(_ptr(st), S, H, W, float(sigma_xy), float(sigma_z), _ptr(pts),
                                 len(pts), _ptr(out))
    return out


# ---------------------------------------------------------------- operators

def laplacian(v: np.ndarray, bc="neumann") -> np.ndarray:
    v = _f64(v)
    H, W = v.shape
    out = np.empty_like(v)
    _load().oracle_laplacian(_ptr(v), H, W, _bc(bc), _ptr(out))
    return out


def apply_A(v: np.ndarray, alpha: float, bc="neumann") -> np.ndarray:
    v = _f64(v)
    H, W = v.shape
    out = np.empty_like(v)
    _load().oracle_apply_A(_ptr(v), H, W, float(alpha), _bc(bc), _ptr(out))
    return out


def rhs(gs: np.ndarray, go: np.ndarray, alpha: float, bc="neumann") -> np.ndarray:
    gs, go = _f64(gs), _f64(go)
    H, W = gs.shape
    out = np.empty_like(gs)
    _load().oracle_rhs(_ptr(gs), _ptr(go), H, W, float(alpha), _bc(bc), _ptr(out))
    return out


# -------------------------------------------------------------------- solves

def cg(b: np.ndarray, alpha: float, bc="neumann", tol: float = 1e-12, maxit: int = 200000):
    b = _f64(b)
    H, W = b.shape
    x = np.empty_like(b)
    rel = ctypes.c_double(0.0)
    it = _load().oracle_cg(_ptr(b), H, W, float(alpha), _bc(bc), float(tol), int(maxit), _ptr(x),
                           ctypes.byref(rel))
    if it < 0:
        raise RuntimeError("oracle CG did not reach tol=%g (rel=%g)" % (tol, rel.value))
    return x


def solve(gs: np.ndarray, go: np.ndarray, alpha: float, bc="neumann", tol: float = 1e-12,
          maxit: int = 200000) -> np.ndarray:
    """One slice of Eq. (1): (alpha I + L) f = alpha g_s + L g_o."""
    gs, go = _f64(gs), _f64(go)
    H, W = gs.shape
    f = np.empty_like(gs)
    rel = ctypes.c_double(0.0)
    it = _load().oracle_solve(_ptr(gs), _ptr(go), H, W, float(alpha), _bc(bc), float(tol),
                              int(maxit), _ptr(f), ctypes.byref(rel))
    if it < 0:
        raise RuntimeError("oracle solve did not reach tol=%g (rel=%g)" % (tol, rel.value))
    return f


def solve_stack(gs: np.ndarray, go: np.ndarray, alpha, bc="neumann", tol: float = 1e-12):
    """Eq. (1) for every slice j of [S][H][W] inputs; alpha scalar or per slice."""
    S = gs.shape[0]
    al = np.broadcast_to(np.asarray(alpha, dtype=np.float64), (S,))
    return np.stack([solve(gs[j], go[j], al[j], bc, tol) for j in range(S)])


def relres(f: np.ndarray, gs: np.ndarray, go: np.ndarray, alpha: float, bc="neumann") -> float:
    """||b - A f|| / ||b||, b = alpha g_s + L g_o, in FP64."""
    f, gs, go = _f64(f), _f64(gs), _f64(go)
    H, W = f.shape
    return float(_load().oracle_relres(_ptr(f), _ptr(gs), _ptr(go), H, W, float(alpha), _bc(bc)))


def adjoint(gbar: np.ndarray, gs: np.ndarray, f: np.ndarray, alpha: float, bc="neumann",
            tol: float = 1e-12, maxit: int = 200000):
    """(dL/dg_s, dL/dg_o, dL/dalpha) for one slice, given gbar = dL/df."""
    gbar, gs, f = _f64(gbar), _f64(gs), _f64(f)
    H, W = gbar.shape
    dgs = np.empty_like(gbar)
    dgo = np.empty_like(gbar)
    da = ctypes.c_double(0.0)
    it = _load().oracle_adjoint(_ptr(gbar), _ptr(gs), _ptr(f), H, W, float(alpha), _bc(bc),
                                float(tol), int(maxit), _ptr(dgs), _ptr(dgo), ctypes.byref(da))
    if it < 0:
        raise RuntimeError("oracle adjoint solve did not converge")
    return dgs, dgo, da.value


def smooth_robust(stack: np.ndarray, sigma_xy: float = 1.0, sigma_z: float = 3.0) -> np.ndarray:
    """Robust cross-slice averaging ("Extensions and Applications"): the average
    across slices of the in-plane smoothed values keeps only those within two
    weighted standard deviations of the window's weighted mean (one pass).
    float64 [S][H][W]."""
    if sigma_z > 0 and int(np.floor(3.0 * sigma_z)) > 31:
        raise ValueError("smooth_robust: cross-slice windows wider than 63 taps are not supported")
    st = np.ascontiguousarray(stack, dtype=np.uint8)
    S, H, W = st.shape
    out = np.empty((S, H, W), dtype=np.float64)
    _load().oracle_smooth_robust(_ptr(st), S, H, W, float(sigma_xy), float(sigma_z), _ptr(out))
    return out


def smooth_robust_points(stack: np.ndarray, zyx: np.ndarray, sigma_xy: float = 1.0,
                         sigma_z: float = 3.0) -> np.ndarray:
    """smooth_robust at the given (z, y, x) voxels."""
    if sigma_z > 0 and int(np.floor(3.0 * sigma_z)) > 31:
        raise ValueError("smooth_robust: cross-slice windows wider than 63 taps are not supported")
    st = np.ascontiguousarray(stack, dtype=np.uint8)
    S, H, W = st.shape
    pts = np.ascontiguousarray(zyx, dtype=np.int32).reshape(-1, 3)
    out = np.empty(len(pts), dtype=np.float64)
    _load().oracle_smooth_robust_points(_ptr(st), S, H, W, float(sigma_xy), float(sigma_z), _ptr(pts),
                                        len(pts), _ptr(out))
    return out


def smooth_transpose(g: np.ndarray, sigma_xy: float = 1.0, sigma_z: float = 3.0) -> np.ndarray:
    """The transpose of smooth (as a linear map of the stack): the gradient of a
    loss on the smoothed stack with respect to the stack.  float64 [S][H][W]."""
    gg = np.ascontiguousarray(g, dtype=np.float64)
    S, H, W = gg.shape
    out = np.empty((S, H, W), dtype=np.float64)
    _load().oracle_smooth_transpose(_ptr(gg), S, H, W, float(sigma_xy), float(sigma_z), _ptr(out))
    return out


def fuse_stack(stack: np.ndarray, alpha: float, sigma_xy: float = 1.0, sigma_z: float = 3.0,
               bc="neumann", tol: float = 1e-12, robust: bool = False):
    """The whole method: smooth across slices, then blend each slice (Eq. (1)).
    robust: the robust cross-slice average of smooth_robust.

    Returns (f, g_s) as float64 [S][H][W].
    """
    gs = smooth_robust(stack, sigma_xy, sigma_z) if robust else smooth(stack, sigma_xy, sigma_z)
    go = np.asarray(stack, dtype=np.float64)
    return solve_stack(gs, go, alpha, bc, tol), gs
