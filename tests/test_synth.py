"""The input generator: seeded, crop-consistent, and of the stated statistics."""
import numpy as np
import pytest

import synth


def test_deterministic_and_crop_consistent():
    a = synth.make_stack(3, 200, 170, seed=5, ramp=True)
    b = synth.make_stack(3, 200, 170, seed=5, ramp=True)
    np.testing.assert_array_equal(a, b)
    c = synth.make_stack(3, 200, 170, seed=5, ramp=True, y0=37, y1=150, x0=11, x1=120)
    np.testing.assert_array_equal(c, a[:, 37:150, 11:120])
    d = synth.make_stack(3, 200, 170, seed=5, ramp=True, band_rows=64)
    np.testing.assert_array_equal(d, a)


def test_noise_statistics():
    n = synth.band_noise(3, 512, 512)
    assert abs(n.std() - 8.0) < 0.3
    assert abs(n.mean()) < 0.3


def test_uneven_batch_sizes():
    d = synth.uneven_batch(64, seed=2)
    for H, W, a, _ in d:
        assert H % 256 == 0 and W % 256 == 0 and 512 <= H <= 4096 and 512 <= W <= 4096
        assert 0.001 <= a <= 0.1


@pytest.mark.parametrize("H,W,seed", [(64, 80, 3), (300, 257, 11), (130, 700, 5)])
def test_torch_generator_matches_numpy(H, W, seed):
    # the device-side generator is the same recipe: equal on the CPU to rounding
    o, s = synth.batch_slice(H, W, seed)
    ot, st = synth.batch_slice_t(H, W, seed, "cpu")
    assert (o != ot.numpy()).sum() <= 2
    assert np.abs(s - st.numpy()).max() <= 1e-4
    a = synth.make_stack(3, H, W, seed, ramp=True, band_rows=64)
    b = synth.make_stack_t(3, H, W, seed, "cpu", ramp=True, band_rows=64).numpy()
    assert (a != b).sum() <= 2 and np.abs(a.astype(int) - b).max() <= 1
