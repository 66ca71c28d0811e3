"""Pins for the oracle's adjoint of Eq. (1).

For a loss of f, the gradients follow from differentiating
(alpha I + L) f = alpha g_s + L g_o.  Central finite differences are exact
(up to rounding) in g_s and g_o because f is affine in them; in alpha they
carry an O(eps^2) term.  The DCT closed form gives a second, independent
check of the whole gradient field.
"""
import numpy as np
from scipy.fft import dctn, idctn

import oracle


def _setup(H=9, W=11, seed=0):
    rng = np.random.default_rng(seed)
    go = rng.integers(0, 256, size=(H, W)).astype(np.float64)
    gs = go + rng.normal(0, 15, size=(H, W))
    t = rng.uniform(0, 255, size=(H, W))
    return gs, go, t


def _loss(gs, go, a, t):
    f = oracle.solve(gs, go, a, tol=1e-14)
    return np.sum((f - t) ** 2), f


def test_adjoint_matches_central_differences():
    gs, go, t = _setup()
    a = 0.02
    L0, f = _loss(gs, go, a, t)
    dgs, dgo, da = oracle.adjoint(2 * (f - t), gs, f, a, tol=1e-14)
    rng = np.random.default_rng(1)
    eps = 1e-3
    for _ in range(6):
        y, x = rng.integers(0, gs.shape[0]), rng.integers(0, gs.shape[1])
        for arr, grad in ((gs, dgs), (go, dgo)):
            p = arr.copy(); p[y, x] += eps
            m = arr.copy(); m[y, x] -= eps
            if arr is gs:
                fp = oracle.solve(p, go, a, tol=1e-14); fm = oracle.solve(m, go, a, tol=1e-14)
            else:
                fp = oracle.solve(gs, p, a, tol=1e-14); fm = oracle.solve(gs, m, a, tol=1e-14)
            # elementwise form of L(+) - L(-) avoids cancelling the large totals
            fd = np.sum((fp - fm) * (fp + fm - 2 * t)) / (2 * eps)
            assert abs(fd - grad[y, x]) <= 1e-6 * max(1.0, abs(grad[y, x]))
    fp = oracle.solve(gs, go, a + 1e-6, tol=1e-14)
    fm = oracle.solve(gs, go, a - 1e-6, tol=1e-14)
    fd = np.sum((fp - fm) * (fp + fm - 2 * t)) / 2e-6
    assert abs(fd - da) <= 1e-5 * abs(da)


def test_adjoint_matches_dct_closed_form():
    gs, go, t = _setup(12, 8, 2)
    a = 0.05
    H, W = gs.shape
    f = oracle.solve(gs, go, a, tol=1e-14)
    gbar = 2 * (f - t)
    lam_k = (4 * np.sin(np.pi * np.arange(H) / (2 * H)) ** 2)[:, None] + \
            (4 * np.sin(np.pi * np.arange(W) / (2 * W)) ** 2)[None, :]
    G = dctn(gbar, type=2, norm="ortho")
    lam = idctn(G / (a + lam_k), type=2, norm="ortho")
    dgo_ref = idctn(G * lam_k / (a + lam_k), type=2, norm="ortho")
    dgs, dgo, da = oracle.adjoint(gbar, gs, f, a, tol=1e-14)
    np.testing.assert_allclose(dgs, a * lam, atol=1e-9)
    np.testing.assert_allclose(dgo, dgo_ref, atol=1e-9)
    assert abs(da - np.sum(lam * (gs - f))) < 1e-7 * max(1, abs(da))


def test_gradients_of_invariances():
    # f is unchanged by g_o + c (Neumann), so dL/dg_o sums to zero; and
    # g_s + c shifts f by c, so sum(dL/dg_s) = sum(dL/df).
    gs, go, t = _setup(10, 10, 3)
    a = 0.01
    f = oracle.solve(gs, go, a, tol=1e-14)
    gbar = 2 * (f - t)
    dgs, dgo, _ = oracle.adjoint(gbar, gs, f, a, tol=1e-14)
    assert abs(dgo.sum()) < 1e-7 * np.abs(gbar).sum()
    assert abs(dgs.sum() - gbar.sum()) < 1e-7 * np.abs(gbar).sum()
