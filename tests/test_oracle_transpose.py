"""Pins for the oracle's transpose of the smoothing (the gradient through it).

The smoothing is linear in the stack, so its transpose is fixed by the
dot-product identity <smooth(x), y> = <x, smooth_transpose(y)> for every x and
y; smooth itself is pinned against scipy's N-d correlation elsewhere.  A
constant gradient also has a closed form away from the stack's borders (the
weights of every window sum to its normaliser there).
"""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("shape,sxy,sz", [((6, 9, 11), 1.0, 3.0), ((3, 14, 5), 0.7, 0.0), ((9, 8, 8), 2.0, 1.5),
                                          ((1, 1, 7), 1.0, 3.0)])
def test_dot_product_identity(shape, sxy, sz):
    rng = np.random.default_rng(sum(shape))
    x = rng.integers(0, 256, shape).astype(np.uint8)
    y = rng.standard_normal(shape)
    lhs = float((oracle.smooth(x, sxy, sz) * y).sum())
    rhs = float((x.astype(np.float64) * oracle.smooth_transpose(y, sxy, sz)).sum())
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs)) * 1e3


def test_constant_gradient_interior():
    # voxels at least two radii from every border: every voxel of their window
    # has a full window, so D is the full weight sum throughout and the
    # transpose of a constant c is c
    g = np.full((40, 20, 20), 3.5)
    out = oracle.smooth_transpose(g, 1.0, 3.0)
    np.testing.assert_allclose(out[18:22, 6:14, 6:14], 3.5, rtol=1e-12)
    assert abs(out[0, 0, 0] - 3.5) > 1e-3   # near the borders it is not
