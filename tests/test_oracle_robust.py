"""Pins for the oracle's robust cross-slice averaging ("Extensions and
Applications": only colour values within two standard deviations are
averaged across slices).

Reading (also in the design notes): at each voxel the values averaged across
slices are the in-plane smoothed values of the slices in the cross-slice
window, with the cross-slice Gaussian weights; values whose squared distance
from the window's weighted mean exceeds four times the weighted variance are
left out, once.  The pins below follow from that definition by hand, not from
the code.  A window with one value v0 of weight share p against a common value
v1 has mean p v0 + (1 - p) v1 and variance p (1 - p) (v0 - v1)^2, so v0 is left
out exactly when p < 1/5 (and v1 when p > 4/5).  Hence a zeroed interior slice
of a constant stack is left out wherever its share stays below 1/5 (sigma_z =
3: at most w_0 / sum w = 0.133), two-slice windows leave nothing out when both
shares lie in [1/5, 4/5] (sigma_z >= 0.6), a symmetric linear ramp loses its
two tails symmetrically, and any result is a convex combination of the
window's values.
"""
import ctypes

import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("sigma_xy,sigma_z", [(1.0, 3.0), (0.5, 3.0), (2.0, 4.0)])
def test_zeroed_slices_are_left_out(sigma_xy, sigma_z):
    # a constant stack with corrupt (all-zero) interior slices farther apart
    # than a window: each window holds at most one, with a share below 1/5
    st = np.full((48, 11, 9), 137, np.uint8)
    for z in (13, 39):
        st[z] = 0
    rob = oracle.smooth_robust(st, sigma_xy, sigma_z)
    plain = oracle.smooth(st, sigma_xy, sigma_z)
    assert np.abs(rob - 137).max() <= 1e-9
    assert plain[13].max() < 137 - 10   # the naive average is pulled down


def test_share_threshold():
    # sigma_z = 1: the centre's share is 1 / (1 + 2 (e^-1/2 + e^-2 + e^-9/2)) = 0.40,
    # above 1/5, so a zeroed interior slice is kept at its own position
    st = np.full((20, 5, 5), 90, np.uint8)
    st[10] = 0
    rob = oracle.smooth_robust(st, 0.0, 1.0)
    np.testing.assert_allclose(rob[10], oracle.smooth(st, 0.0, 1.0)[10], rtol=0, atol=1e-10)
    assert rob[10].max() < 90 - 30


def test_two_slices_never_leave_out():
    rng = np.random.default_rng(5)
    st = rng.integers(0, 256, (2, 13, 17)).astype(np.uint8)
    for sxy, sz in [(1.0, 3.0), (0.0, 1.0), (1.5, 0.7)]:
        np.testing.assert_allclose(oracle.smooth_robust(st, sxy, sz), oracle.smooth(st, sxy, sz),
                                   rtol=0, atol=1e-10)


def test_linear_ramp_interior_is_unchanged():
    # v_z = 10 + 5 z: the tails beyond two standard deviations are cut on both
    # sides by the same weights, so the interior average stays at the centre
    z = np.arange(40, dtype=np.float64)
    st = np.broadcast_to((10 + 5 * z)[:, None, None], (40, 6, 7)).astype(np.uint8)
    rob = oracle.smooth_robust(st, 1.0, 3.0)
    for zz in range(9, 31):
        np.testing.assert_allclose(rob[zz], 10 + 5 * zz, rtol=0, atol=1e-9)


def test_convex_combination():
    rng = np.random.default_rng(8)
    st = rng.integers(0, 256, (15, 10, 12)).astype(np.uint8)
    rob = oracle.smooth_robust(st, 0.0, 3.0)   # no in-plane blur: window values are raw voxels
    for z in range(15):
        lo = st[max(0, z - 9):z + 10].min(axis=0)
        hi = st[max(0, z - 9):z + 10].max(axis=0)
        assert (rob[z] >= lo - 1e-9).all() and (rob[z] <= hi + 1e-9).all()


def test_window_wider_than_the_oracle_holds_is_refused():
    # the oracle keeps a window of at most 63 taps (radius 31); a wider window
    # (sigma_z >= 32/3) is refused, in the wrapper and in the C routine, rather
    # than silently cut short
    st = np.full((3, 4, 5), 7, np.uint8)
    with pytest.raises(ValueError):
        oracle.smooth_robust(st, 1.0, 11.0)
    v = oracle._load().oracle_smooth_robust_voxel
    v.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                  ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    v.restype = ctypes.c_double
    assert np.isnan(v(st.ctypes.data_as(ctypes.c_void_p), 3, 4, 5, 1.0, 11.0, 1, 1, 1))
    assert abs(oracle.smooth_robust(st, 1.0, 10.0)[1, 1, 1] - 7.0) <= 1e-12   # radius 30: within the window


def test_points_equal_whole_stack():
    # the point form evaluates the same voxel routine as the whole-stack form
    rng = np.random.default_rng(4)
    st = rng.integers(0, 256, (12, 9, 11)).astype(np.uint8)
    st[5] = 0
    full = oracle.smooth_robust(st, 1.0, 3.0)
    pts = np.stack([rng.integers(0, n, 50) for n in st.shape], axis=1)
    np.testing.assert_array_equal(oracle.smooth_robust_points(st, pts, 1.0, 3.0), full[tuple(pts.T)])
