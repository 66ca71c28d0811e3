"""Oracle values on a crop of a stack too large for the CPU oracle.

The screened operator's Green's function decays like exp(-sqrt(alpha) r)
(pixel units), so solving Eq. (1) on the crop padded by a halo of
ceil(40 / sqrt(alpha)) pixels (clipped at the true slice edges, where the true
Neumann condition applies) changes the crop's values by a factor of about
exp(-40) of the boundary mismatch: far below any tolerance used here.  The
smoothing of the padded region needs 3 more pixels of raw data (its in-plane
radius) except at true edges.  Pinned by tests/test_oracle_crop.py against the
full oracle solve.  Test infrastructure, like the rest of the oracle."""
import math

import numpy as np

import oracle
import synth


def crop_halo(alpha: float) -> int:
    return int(math.ceil(40.0 / math.sqrt(alpha)))


def crop_region(H: int, W: int, alpha: float, y0: int, y1: int, x0: int, x1: int):
    """((padded region), (raw region)) of a crop: rows and columns
    (lo, hi, lo, hi) of the halo-padded solve and of the raw data its
    smoothing reads."""
    h = crop_halo(alpha)
    py0, py1, px0, px1 = max(0, y0 - h), min(H, y1 + h), max(0, x0 - h), min(W, x1 + h)
    return (py0, py1, px0, px1), (max(0, py0 - 3), min(H, py1 + 3), max(0, px0 - 3), min(W, px1 + 3))


def fuse_crop(seed: int, S: int, H: int, W: int, alpha: float, y0: int, y1: int, x0: int, x1: int,
              z_list, ramp: bool = False, raw=None, tol: float = 1e-12):
    """Oracle f on slices z_list, rows [y0, y1), cols [x0, x1) of the seeded
    S x H x W stack (generated crop-wise); returns (f [len(z)][y1-y0][x1-x0],
    raw uint8 region used, region origin)."""
    (py0, py1, px0, px1), (my0, my1, mx0, mx1) = crop_region(H, W, alpha, y0, y1, x0, x1)
    if raw is None:
        raw = synth.make_stack(S, H, W, seed, ramp=ramp, y0=my0, y1=my1, x0=mx0, x1=mx1)
    yy, xx = np.mgrid[py0 - my0:py1 - my0, px0 - mx0:px1 - mx0]
    out = []
    for z in z_list:
        pts = np.stack([np.full(yy.size, z), yy.ravel(), xx.ravel()], axis=1)
        gs = oracle.smooth_points(raw, pts).reshape(yy.shape)
        go = raw[z, py0 - my0:py1 - my0, px0 - mx0:px1 - mx0].astype(np.float64)
        f = oracle.solve(gs, go, alpha, tol=tol)
        out.append(f[y0 - py0:y1 - py0, x0 - px0:x1 - px0])
    return np.stack(out), raw, (my0, mx0)
