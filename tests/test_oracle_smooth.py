"""Pins for the oracle's anisotropic smoothing (Section III-A; 3-sigma support
from the Implementation subsection).

The oracle sums the truncated 3D Gaussian tap by tap.  These tests check it
against an independent construction (scipy's N-d correlation of the stack
and of an all-ones stack with an explicitly built kernel), and against
properties any weighted average of this kind must have.
"""
import json
import os

import numpy as np
import pytest
from scipy.ndimage import correlate

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")


def _kernel(sxy, sz):
    rxy = int(np.floor(3 * sxy)) if sxy > 0 else 0
    rz = int(np.floor(3 * sz)) if sz > 0 else 0
    dz, dy, dx = np.meshgrid(np.arange(-rz, rz + 1), np.arange(-rxy, rxy + 1),
                             np.arange(-rxy, rxy + 1), indexing="ij")
    k = np.ones(dz.shape)
    if sxy > 0:
        k *= np.exp(-(dx ** 2 + dy ** 2) / (2 * sxy ** 2))
    if sz > 0:
        k *= np.exp(-dz ** 2 / (2 * sz ** 2))
    return k


def _scipy_smooth(st, sxy, sz):
    k = _kernel(sxy, sz)
    num = correlate(st.astype(np.float64), k, mode="constant", cval=0.0)
    den = correlate(np.ones(st.shape), k, mode="constant", cval=0.0)
    return num / den


@pytest.mark.parametrize("shape,sxy,sz", [
    ((5, 7, 9), 1.0, 3.0),
    ((12, 6, 5), 1.0, 3.0),
    ((23, 4, 4), 1.0, 3.0),
    ((1, 8, 11), 1.0, 3.0),
    ((9, 1, 13), 1.0, 3.0),
    ((7, 9, 6), 0.7, 1.5),
    ((6, 5, 5), 0.0, 2.0),
    ((6, 5, 5), 1.3, 0.0),
])
def test_matches_independent_correlation(shape, sxy, sz):
    rng = np.random.default_rng(hash(shape) % 2 ** 32)
    st = rng.integers(0, 256, size=shape, dtype=np.uint8)
    got = oracle.smooth(st, sxy, sz)
    ref = _scipy_smooth(st, sxy, sz)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-11)


def test_points_match_full():
    rng = np.random.default_rng(3)
    st = rng.integers(0, 256, size=(11, 13, 17), dtype=np.uint8)
    full = oracle.smooth(st)
    pts = np.stack([rng.integers(0, n, 40) for n in st.shape], axis=1)
    got = oracle.smooth_points(st, pts)
    np.testing.assert_array_equal(got, full[pts[:, 0], pts[:, 1], pts[:, 2]])


def test_constant_stack_unchanged():
    st = np.full((10, 9, 8), 77, dtype=np.uint8)
    np.testing.assert_allclose(oracle.smooth(st), 77.0, rtol=0, atol=1e-12)


def test_single_slice_is_inplane_only():
    rng = np.random.default_rng(5)
    st = rng.integers(0, 256, size=(1, 12, 10), dtype=np.uint8)
    np.testing.assert_allclose(oracle.smooth(st, 1.0, 3.0), oracle.smooth(st, 1.0, 0.0), atol=1e-12)


def test_convex_combination_bounds():
    rng = np.random.default_rng(6)
    st = rng.integers(30, 200, size=(8, 10, 10), dtype=np.uint8)
    out = oracle.smooth(st)
    assert out.min() >= st.min() - 1e-12 and out.max() <= st.max() + 1e-12


def test_interior_impulse_response_is_the_gaussian():
    # An interior impulse (no tap reaches an edge) returns the normalised,
    # truncated, separable Gaussian: exp(-(dx^2+dy^2)/2) exp(-dz^2/18) / sum.
    # (every output the impulse reaches has its whole window inside the stack)
    S, H, W = 37, 13, 13
    st = np.zeros((S, H, W), dtype=np.uint8)
    st[18, 6, 6] = 255
    out = oracle.smooth(st, 1.0, 3.0)
    wx = np.exp(-np.arange(-3, 4) ** 2 / 2.0)
    wz = np.exp(-np.arange(-9, 10) ** 2 / 18.0)
    k = wz[:, None, None] * wx[None, :, None] * wx[None, None, :]
    ref = np.zeros((S, H, W))
    ref[9:28, 3:10, 3:10] = 255 * k / k.sum()
    np.testing.assert_allclose(out, ref, atol=1e-12)
    # symmetric under every axis flip
    np.testing.assert_allclose(out, out[::-1, ::-1, ::-1], atol=1e-12)


def test_paper_parameters_give_radii_3_and_9():
    p = json.load(open(GOLDEN))
    k = _kernel(p["sigma_xy_px"], p["sigma_z_px"])
    assert k.shape == (19, 7, 7)
    # the slice window of the distributed scheme: |j - k| <= 3 sigma_z
    assert (k.shape[0] - 1) // 2 == int(p["truncation_sigmas"] * p["sigma_z_px"])
