"""Seeded synthetic EM-like image stacks (input generation only).

This module produces the inputs shared by the GPU path, the CPU oracle, the
tests and the benchmark.  It holds none of the fusion method's arithmetic: no
anisotropic smoothing as the paper defines it, no Poisson operator.  The
paper's datasets (Kasthuri11, Cardona; Results section, Scalability
subsection) are not available, so these stacks stand in for them.

Recipe (per stack, all draws seeded):

* base texture B (shared by every slice of a stack): 40 Gaussian blobs, each
  with centre uniform over the slice, width sigma_b ~ U(3, 20) px and
  amplitude ~ U(20, 120), value A exp(-r^2 / 2 sigma_b^2); plus band-limited
  noise of standard deviation 8: white Gaussian noise filtered with a
  Gaussian of width 1.5 px (truncated at 3 widths, reflecting edges).  The
  white noise is counter-based, keyed by (seed, y, x), so any crop can be
  regenerated without producing the whole slice.
* slice j: clip(rint(gain_j B + offset_j [+ ramp_j]), 0, 255) as uint8 with
  gain_j ~ U(0.8, 1.2), offset_j ~ U(-20, 20) and, when requested, a linear
  illumination ramp sx_j (x - W/2) + sy_j (y - H/2), sx_j, sy_j ~ U(-0.01, 0.01).
  These per-slice gain/offset/ramp changes are the low-xy-frequency,
  high-z-frequency artifacts the method removes (EM Image Processing section).
"""
from __future__ import annotations

import numpy as np
from scipy.ndimage import gaussian_filter

NOISE_SIGMA = 1.5
NOISE_TRUNC = 3.0
NOISE_STD = 8.0
_NOISE_R = int(NOISE_TRUNC * NOISE_SIGMA + 0.5)  # scipy's own radius rule

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _splitmix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea, Flood 2014) on uint64 arrays."""
    with np.errstate(over="ignore"):
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def white_noise(seed: int, y0: int, y1: int, x0: int, x1: int) -> np.ndarray:
    """Standard-normal noise on rows [y0,y1) x cols [x0,x1), keyed by (seed, y, x).

    Box-Muller on two 32-bit uniforms taken from one SplitMix64 output.
    """
    ys = np.arange(y0, y1, dtype=np.uint64)[:, None]
    xs = np.arange(x0, x1, dtype=np.uint64)[None, :]
    key = _splitmix64(np.full(1, seed, dtype=np.uint64))[0]
    with np.errstate(over="ignore"):
        h = _splitmix64((ys << np.uint64(32)) + xs + key)
    u1 = ((h >> np.uint64(32)).astype(np.float64) + 0.5) / 4294967296.0
    u2 = ((h & np.uint64(0xFFFFFFFF)).astype(np.float64) + 0.5) / 4294967296.0
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def _noise_gain() -> float:
    """Standard deviation of unit white noise after the (2D, separable)
    band-limiting filter: sqrt(sum of squared 2D taps) = sum of squared 1D taps."""
    imp = np.zeros(4 * _NOISE_R + 1)
    imp[2 * _NOISE_R] = 1.0
    k = gaussian_filter(imp, NOISE_SIGMA, truncate=NOISE_TRUNC, mode="constant")
    return float(np.sum(k * k))


def band_noise(seed: int, H: int, W: int, y0: int = 0, y1: int | None = None,
               x0: int = 0, x1: int | None = None) -> np.ndarray:
    """Band-limited noise (std 8) on a crop of an H x W slice."""
    y1 = H if y1 is None else y1
    x1 = W if x1 is None else x1
    r = _NOISE_R
    ya, yb = max(0, y0 - r), min(H, y1 + r)
    xa, xb = max(0, x0 - r), min(W, x1 + r)
    n = white_noise(seed, ya, yb, xa, xb)
    n = gaussian_filter(n, NOISE_SIGMA, truncate=NOISE_TRUNC, mode="reflect")
    n *= NOISE_STD / _noise_gain()
    return n[y0 - ya:y1 - ya, x0 - xa:x1 - xa]


def _blob_params(rng: np.random.Generator, H: int, W: int, n_blobs: int):
    cx = rng.uniform(0.0, W, n_blobs)
    cy = rng.uniform(0.0, H, n_blobs)
    sb = rng.uniform(3.0, 20.0, n_blobs)
    amp = rng.uniform(20.0, 120.0, n_blobs)
    return cx, cy, sb, amp


def base_texture(seed: int, H: int, W: int, y0: int = 0, y1: int | None = None,
                 x0: int = 0, x1: int | None = None, n_blobs: int = 40) -> np.ndarray:
    """Base texture B on a crop [y0,y1) x [x0,x1) of an H x W slice (float64)."""
    y1 = H if y1 is None else y1
    x1 = W if x1 is None else x1
    rng = np.random.Generator(np.random.PCG64(seed))
    cx, cy, sb, amp = _blob_params(rng, H, W, n_blobs)
    B = band_noise(seed, H, W, y0, y1, x0, x1).copy()
    for i in range(n_blobs):
        rad = int(np.ceil(6.0 * sb[i]))
        ya, yb = max(y0, int(cy[i]) - rad), min(y1, int(cy[i]) + rad + 1)
        xa, xb = max(x0, int(cx[i]) - rad), min(x1, int(cx[i]) + rad + 1)
        if ya >= yb or xa >= xb:
            continue
        yy = np.arange(ya, yb, dtype=np.float64)[:, None] - cy[i]
        xx = np.arange(xa, xb, dtype=np.float64)[None, :] - cx[i]
        B[ya - y0:yb - y0, xa - x0:xb - x0] += amp[i] * np.exp(-(yy * yy + xx * xx) / (2.0 * sb[i] ** 2))
    return B


def slice_params(seed: int, S: int):
    """Per-slice gain, offset and ramp slopes (sx, sy)."""
    rng = np.random.Generator(np.random.PCG64([seed, 7]))
    gain = rng.uniform(0.8, 1.2, S)
    off = rng.uniform(-20.0, 20.0, S)
    sx = rng.uniform(-0.01, 0.01, S)
    sy = rng.uniform(-0.01, 0.01, S)
    return gain, off, sx, sy


def make_stack(S: int, H: int, W: int, seed: int, ramp: bool = False,
               y0: int = 0, y1: int | None = None, x0: int = 0, x1: int | None = None,
               band_rows: int = 2048) -> np.ndarray:
    """uint8 stack [S][y1-y0][x1-x0] (a crop of the full S x H x W stack)."""
    y1 = H if y1 is None else y1
    x1 = W if x1 is None else x1
    gain, off, sx, sy = slice_params(seed, S)
    out = np.empty((S, y1 - y0, x1 - x0), dtype=np.uint8)
    xx = np.arange(x0, x1, dtype=np.float64)[None, :] - W / 2.0
    for ya in range(y0, y1, band_rows):
        yb = min(y1, ya + band_rows)
        B = base_texture(seed, H, W, ya, yb, x0, x1)
        yy = np.arange(ya, yb, dtype=np.float64)[:, None] - H / 2.0
        for j in range(S):
            v = gain[j] * B + off[j]
            if ramp:
                v = v + sx[j] * xx + sy[j] * yy
            out[j, ya - y0:yb - y0] = np.clip(np.rint(v), 0, 255).astype(np.uint8)
    return out


def uneven_batch(n: int, seed: int, sizes=tuple(range(512, 4097, 256)),
                 alpha_range=(0.001, 0.1), max_side: int | None = None):
    """Descriptors of an uneven batch: list of (H, W, alpha, slice_seed)."""
    rng = np.random.Generator(np.random.PCG64([seed, 11]))
    sizes = np.asarray(sizes)
    if max_side is not None:
        sizes = sizes[sizes <= max_side]
    Hs = rng.choice(sizes, n)
    Ws = rng.choice(sizes, n)
    al = rng.uniform(alpha_range[0], alpha_range[1], n)
    return [(int(Hs[i]), int(Ws[i]), float(al[i]), seed * 100003 + i) for i in range(n)]


def batch_slice(H: int, W: int, slice_seed: int):
    """One slice of an uneven batch: (g_orig uint8 [H][W], g_smooth float32 [H][W]).

    g_orig is a generator slice (gain/offset applied); g_smooth is the clipped
    base texture blurred in-plane (width 1 px), a stand-in for the corrected,
    low-frequency target of that slice.
    """
    g_o = make_stack(1, H, W, slice_seed)[0]
    B = np.clip(np.rint(base_texture(slice_seed, H, W)), 0, 255)
    g_s = gaussian_filter(B, 1.0, truncate=3.0, mode="nearest").astype(np.float32)
    return g_o, g_s


CONFIG_SEED = {0: 1000, 1: 1001, 2: 1002, 3: 1003, 4: 1004}


# ------------------------------------------------------------------------
# The same recipe evaluated with torch, on any device.  The benchmark's large
# workloads (thousands of megapixels) are generated on the GPU this way; the
# numpy functions above stay the definition, and the two agree to rounding
# (checked on small slices on the CPU).

def _s64(c: int) -> int:
    """uint64 constant as the int64 with the same bits."""
    return c - (1 << 64) if c >= (1 << 63) else c


def _lsr(z, k: int):
    """Logical right shift of an int64 tensor holding uint64 bits."""
    return (z >> k) & ((1 << (64 - k)) - 1)


def _splitmix64_t(z):
    z = z + _s64(0x9E3779B97F4A7C15)
    z = (z ^ _lsr(z, 30)) * _s64(0xBF58476D1CE4E5B9)
    z = (z ^ _lsr(z, 27)) * _s64(0x94D049BB133111EB)
    return z ^ _lsr(z, 31)


def white_noise_t(seed: int, y0: int, y1: int, x0: int, x1: int, device):
    import torch
    key = _s64(int(_splitmix64(np.full(1, seed, dtype=np.uint64))[0]))
    ys = torch.arange(y0, y1, dtype=torch.int64, device=device)[:, None]
    xs = torch.arange(x0, x1, dtype=torch.int64, device=device)[None, :]
    h = _splitmix64_t((ys << 32) + xs + key)
    u1 = (_lsr(h, 32).double() + 0.5) / 4294967296.0
    u2 = ((h & 0xFFFFFFFF).double() + 0.5) / 4294967296.0
    return torch.sqrt(-2.0 * torch.log(u1)) * torch.cos(2.0 * np.pi * u2)


def _gauss_taps(sigma: float, truncate: float):
    r = int(truncate * sigma + 0.5)
    x = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-0.5 * x * x / (sigma * sigma))
    return w / w.sum(), r


def _filter_axis_t(a, sigma: float, truncate: float, axis: int, mode: str):
    """1D Gaussian correlation along axis (0 or 1) of a 2D tensor; mode
    'reflect' (half-sample symmetric) or 'nearest' (edge replicate), as scipy."""
    import torch
    w, r = _gauss_taps(sigma, truncate)
    if axis == 0:
        a = a.t()
    n = a.shape[1]
    if mode == "reflect":
        if n < r:
            raise ValueError("axis shorter than the filter radius")
        left, right = a[:, :r].flip(1), a[:, n - r:].flip(1)
    else:
        left, right = a[:, :1].expand(-1, r), a[:, n - 1:].expand(-1, r)
    p = torch.cat([left, a, right], dim=1)
    out = torch.zeros_like(a)
    for k in range(2 * r + 1):
        out += float(w[k]) * p[:, k:k + n]
    return out.t().contiguous() if axis == 0 else out


def band_noise_t(seed: int, H: int, W: int, y0: int, y1: int, x0: int, x1: int, device):
    r = _NOISE_R
    ya, yb = max(0, y0 - r), min(H, y1 + r)
    xa, xb = max(0, x0 - r), min(W, x1 + r)
    n = white_noise_t(seed, ya, yb, xa, xb, device)
    n = _filter_axis_t(n, NOISE_SIGMA, NOISE_TRUNC, 0, "reflect")
    n = _filter_axis_t(n, NOISE_SIGMA, NOISE_TRUNC, 1, "reflect")
    n *= NOISE_STD / _noise_gain()
    return n[y0 - ya:y1 - ya, x0 - xa:x1 - xa]


def base_texture_t(seed: int, H: int, W: int, y0: int, y1: int, x0: int, x1: int, device,
                   n_blobs: int = 40):
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    cx, cy, sb, amp = _blob_params(rng, H, W, n_blobs)
    B = band_noise_t(seed, H, W, y0, y1, x0, x1, device).contiguous()
    for i in range(n_blobs):
        rad = int(np.ceil(6.0 * sb[i]))
        ya, yb = max(y0, int(cy[i]) - rad), min(y1, int(cy[i]) + rad + 1)
        xa, xb = max(x0, int(cx[i]) - rad), min(x1, int(cx[i]) + rad + 1)
        if ya >= yb or xa >= xb:
            continue
        yy = torch.arange(ya, yb, dtype=torch.float64, device=device)[:, None] - cy[i]
        xx = torch.arange(xa, xb, dtype=torch.float64, device=device)[None, :] - cx[i]
        B[ya - y0:yb - y0, xa - x0:xb - x0] += amp[i] * torch.exp(-(yy * yy + xx * xx) / (2.0 * sb[i] ** 2))
    return B


def make_stack_t(S: int, H: int, W: int, seed: int, device, ramp: bool = False,
                 band_rows: int = 2048):
    """make_stack evaluated with torch on `device` (uint8 tensor [S][H][W])."""
    import torch
    gain, off, sx, sy = slice_params(seed, S)
    out = torch.empty((S, H, W), dtype=torch.uint8, device=device)
    xx = torch.arange(0, W, dtype=torch.float64, device=device)[None, :] - W / 2.0
    for ya in range(0, H, band_rows):
        yb = min(H, ya + band_rows)
        B = base_texture_t(seed, H, W, ya, yb, 0, W, device)
        yy = torch.arange(ya, yb, dtype=torch.float64, device=device)[:, None] - H / 2.0
        for j in range(S):
            v = float(gain[j]) * B + float(off[j])
            if ramp:
                v = v + float(sx[j]) * xx + float(sy[j]) * yy
            out[j, ya:yb] = torch.clamp(torch.round(v), 0, 255).to(torch.uint8)
    return out


def batch_slice_t(H: int, W: int, slice_seed: int, device):
    """batch_slice evaluated with torch on `device`: (g_orig uint8, g_smooth float32)."""
    import torch
    g_o = make_stack_t(1, H, W, slice_seed, device)[0]
    B = torch.clamp(torch.round(base_texture_t(slice_seed, H, W, 0, H, 0, W, device)), 0, 255)
    g_s = _filter_axis_t(B, 1.0, 3.0, 0, "nearest")
    g_s = _filter_axis_t(g_s, 1.0, 3.0, 1, "nearest")
    return g_o, g_s.to(torch.float32)
