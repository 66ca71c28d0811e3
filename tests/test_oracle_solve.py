"""Pins for the oracle's screened-Poisson solve (Section III-B: the energy,
Eq. (1) and its frequency-space form).

* Neumann: the DCT-II diagonalises the grid Laplacian with reflecting edges,
  so Eq. (1) has the closed form of the frequency-space blend with the
  discrete eigenvalues 4 sin^2(pi k / 2W) + 4 sin^2(pi l / 2H).
* Periodic: the same with the DFT and 4 sin^2(pi k / W) + 4 sin^2(pi l / H),
  i.e. the paper's Fourier formula on the pixel lattice.
* The minimiser of the discrete energy itself, by a dense solve of its
  Hessian obtained from energy evaluations only (no stencil code).
* Invariants of the problem.
"""
import numpy as np
import pytest
from scipy.fft import dctn, fft2, idctn, ifft2

import oracle


def _data(H, W, seed):
    rng = np.random.default_rng(seed)
    go = rng.integers(0, 256, size=(H, W)).astype(np.float64)
    gs = go + rng.normal(0, 20, size=(H, W))
    return gs, go


def dct_blend(gs, go, alpha):
    H, W = gs.shape
    lam = (4 * np.sin(np.pi * np.arange(H) / (2 * H)) ** 2)[:, None] + \
          (4 * np.sin(np.pi * np.arange(W) / (2 * W)) ** 2)[None, :]
    Gs = dctn(gs, type=2, norm="ortho")
    Go = dctn(go, type=2, norm="ortho")
    return idctn((alpha * Gs + lam * Go) / (alpha + lam), type=2, norm="ortho")


def fft_blend(gs, go, alpha):
    H, W = gs.shape
    lam = (4 * np.sin(np.pi * np.arange(H) / H) ** 2)[:, None] + \
          (4 * np.sin(np.pi * np.arange(W) / W) ** 2)[None, :]
    return np.real(ifft2((alpha * fft2(gs) + lam * fft2(go)) / (alpha + lam)))


@pytest.mark.parametrize("H,W,alpha", [(16, 16, 0.01), (17, 23, 0.01), (32, 9, 0.1),
                                       (40, 40, 0.001), (1, 31, 0.05), (64, 48, 1.0)])
def test_neumann_matches_dct_closed_form(H, W, alpha):
    gs, go = _data(H, W, H * 131 + W)
    f = oracle.solve(gs, go, alpha, "neumann", tol=1e-13)
    np.testing.assert_allclose(f, dct_blend(gs, go, alpha), rtol=0, atol=1e-9)


@pytest.mark.parametrize("H,W,alpha", [(16, 16, 0.01), (18, 10, 0.05), (2, 7, 0.3), (33, 27, 0.002)])
def test_periodic_matches_fourier_closed_form(H, W, alpha):
    gs, go = _data(H, W, H * 7 + W)
    f = oracle.solve(gs, go, alpha, "periodic", tol=1e-13)
    np.testing.assert_allclose(f, fft_blend(gs, go, alpha), rtol=0, atol=1e-9)


def _energy(f, gs, go, alpha):
    """Discrete form of the paper's energy: alpha (f - g_s)^2 summed over
    pixels plus the squared difference of f's and g_o's forward differences
    over every pixel pair sharing an edge inside the slice."""
    e = alpha * np.sum((f - gs) ** 2)
    e += np.sum(((f[:, 1:] - f[:, :-1]) - (go[:, 1:] - go[:, :-1])) ** 2)
    e += np.sum(((f[1:, :] - f[:-1, :]) - (go[1:, :] - go[:-1, :])) ** 2)
    return e


@pytest.mark.parametrize("H,W", [(4, 5), (1, 7), (6, 6), (3, 1), (1, 1)])
def test_matches_dense_energy_minimiser(H, W):
    alpha = 0.03
    gs, go = _data(H, W, 17 * H + W)
    n = H * W
    # The energy is quadratic: E(f) = 1/2 f^T Q f - c^T f + E(0).  Recover Q
    # and c from energy values only (exact second / first differences), then
    # solve the dense system.  Q does not depend on the data, so it is taken
    # with zero data (small, exactly representable energies); c uses steps of
    # size s so that rounding of the large data-dependent energies stays small.
    z = np.zeros((H, W))
    e = np.eye(n).reshape(n, H, W)
    Ez = np.array([_energy(e[i], z, z, alpha) for i in range(n)])
    Q = np.empty((n, n))
    for i in range(n):
        for j in range(n):
            Q[i, j] = _energy(e[i] + e[j], z, z, alpha) - Ez[i] - Ez[j]
    s = 1e3
    c = np.array([(_energy(-s * e[i], gs, go, alpha) - _energy(s * e[i], gs, go, alpha)) / (2 * s)
                  for i in range(n)])
    f_dense = np.linalg.solve(Q, c).reshape(H, W)
    f = oracle.solve(gs, go, alpha, tol=1e-14)
    np.testing.assert_allclose(f, f_dense, rtol=0, atol=1e-8)


def test_energy_is_minimal_at_solution():
    gs, go = _data(12, 10, 4)
    alpha = 0.02
    f = oracle.solve(gs, go, alpha, tol=1e-14)
    E = _energy(f, gs, go, alpha)
    rng = np.random.default_rng(0)
    for _ in range(10):
        d = rng.normal(size=f.shape) * 1e-3
        assert _energy(f + d, gs, go, alpha) > E


def test_identical_inputs_return_input():
    gs, go = _data(20, 30, 1)
    f = oracle.solve(go, go, 0.01, tol=1e-14)
    np.testing.assert_allclose(f, go, atol=1e-9)


def test_large_alpha_returns_smooth_input():
    gs, go = _data(20, 30, 2)
    f = oracle.solve(gs, go, 1e9, tol=1e-14)
    np.testing.assert_allclose(f, gs, atol=1e-6)


def test_small_alpha_returns_detail_plus_mean():
    gs, go = _data(12, 14, 3)
    alpha = 1e-9
    f = oracle.solve(gs, go, alpha, tol=1e-14)
    np.testing.assert_allclose(f, go + gs.mean() - go.mean(), atol=1e-5)


@pytest.mark.parametrize("alpha", [0.001, 0.01, 0.5])
def test_neumann_mean_preserved(alpha):
    gs, go = _data(25, 19, 5)
    f = oracle.solve(gs, go, alpha, tol=1e-14)
    assert abs(f.mean() - gs.mean()) < 1e-8


def test_offset_invariances():
    gs, go = _data(15, 22, 6)
    a = 0.01
    f = oracle.solve(gs, go, a, tol=1e-14)
    np.testing.assert_allclose(oracle.solve(gs, go + 13.0, a, tol=1e-14), f, atol=1e-8)
    np.testing.assert_allclose(oracle.solve(gs + 7.5, go, a, tol=1e-14), f + 7.5, atol=1e-8)


def test_linearity():
    g1s, g1o = _data(14, 11, 7)
    g2s, g2o = _data(14, 11, 8)
    a = 0.05
    f1 = oracle.solve(g1s, g1o, a, tol=1e-14)
    f2 = oracle.solve(g2s, g2o, a, tol=1e-14)
    f12 = oracle.solve(2 * g1s - g2s, 2 * g1o - g2o, a, tol=1e-14)
    np.testing.assert_allclose(f12, 2 * f1 - f2, atol=1e-8)


def test_single_pixel_slice():
    f = oracle.solve(np.array([[42.0]]), np.array([[7.0]]), 0.01)
    assert abs(f[0, 0] - 42.0) < 1e-12


def test_operator_symmetric():
    rng = np.random.default_rng(9)
    x, y = rng.normal(size=(2, 13, 17))
    for bc in ("neumann", "periodic"):
        assert abs(np.sum(oracle.apply_A(x, 0.3, bc) * y) - np.sum(x * oracle.apply_A(y, 0.3, bc))) < 1e-10


def test_relres_closed_form_for_constant_error():
    # A constant error c has A c = alpha c (constants span L's null space
    # under Neumann), so the residual norm is alpha |c| sqrt(N).
    gs, go = _data(16, 20, 10)
    a = 0.01
    f = oracle.solve(gs, go, a, tol=1e-14)
    b = oracle.rhs(gs, go, a)
    rel = oracle.relres(f + 0.25, gs, go, a)
    assert abs(rel - a * 0.25 * np.sqrt(f.size) / np.linalg.norm(b)) < 1e-12
    assert oracle.relres(f, gs, go, a) < 1e-13


def test_rhs_definition():
    # b = alpha g_s - Delta g_o with the 5-point Laplacian and reflected ghosts
    gs, go = _data(6, 7, 11)
    a = 0.2
    pad = np.pad(go, 1, mode="edge")
    lap5 = pad[:-2, 1:-1] + pad[2:, 1:-1] + pad[1:-1, :-2] + pad[1:-1, 2:] - 4 * go
    np.testing.assert_allclose(oracle.rhs(gs, go, a), a * gs - lap5, atol=1e-12)
