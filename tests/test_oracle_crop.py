"""The crop oracle equals the full oracle inside the crop (pins oracle.crop)."""
import numpy as np

import oracle
import synth
from oracle.crop import crop_halo, fuse_crop


def test_crop_matches_full_solve():
    S, H, W, alpha, seed = 3, 640, 700, 0.05, 77
    assert crop_halo(alpha) == 179
    stack = synth.make_stack(S, H, W, seed, ramp=True)
    gs = oracle.smooth(stack)
    for (y0, y1, x0, x1) in ((200, 328, 250, 380), (0, 96, 600, 700)):   # interior, corner
        fc, _, _ = fuse_crop(seed, S, H, W, alpha, y0, y1, x0, x1, [1], ramp=True)
        ff = oracle.solve(gs[1], stack[1].astype(np.float64), alpha, tol=1e-12)
        assert np.abs(fc[0] - ff[y0:y1, x0:x1]).max() < 1e-8
