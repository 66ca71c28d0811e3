"""GPU parity at the full sizes of the batched, mixed-precision and adjoint
workloads, with the settings bench.py times.  Whole batches are checked by a
property that holds at any size (the FP64 relative residual, recomputed here
with plain torch float64 operations, not the library's kernels), and sampled
outputs against the oracle: the smallest slices of the batch, 1024 x 1024
crops of the 21504 x 26624 slices (crop oracle: halo ceil(40/sqrt(alpha)) px),
and gradients on two full slices plus central differences on 32 voxels."""
import numpy as np
import pytest
import torch

import oracle
import paper_1506_02079_amd as gdf
import synth
from crop_oracle import fuse_crop

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _lap(v):
    out = torch.zeros_like(v)
    d = v[:, 1:] - v[:, :-1]
    out[:, 1:] += d
    out[:, :-1] -= d
    d = v[1:, :] - v[:-1, :]
    out[1:, :] += d
    out[:-1, :] -= d
    return out


def _relres_torch(f, gs, go, alpha):
    f, gs, go = f.double(), gs.double(), go.double()
    b = alpha * gs + _lap(go)
    r = b - (alpha * f + _lap(f))
    return float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(b))


def test_batched_full_size_512_uneven_slices():
    desc = synth.uneven_batch(512, seed=synth.CONFIG_SEED[2])
    go, gs = [], []
    for H, W, _, sd in desc:
        o, s = synth.batch_slice_t(H, W, sd, DEV)
        go.append(o)
        gs.append(s)
    al = [a for _, _, a, _ in desc]
    print("batch generated: %.3f Gpx" % (sum(H * W for H, W, _, _ in desc) / 1e9), flush=True)
    f32, rep32 = gdf.solve_slices(gs, go, al, tol=1e-6, use_graph=True, autotune=True)   # the benchmark's call
    tuned = gdf.autotune_last()
    print("tuned", tuned, flush=True)
    # the same iteration with the output formed in FP64 (before rounding)
    f64, rep = gdf.solve_slices(gs, go, al, tol=1e-6, use_graph=True, out_dtype=gdf.DTYPE_F64, **tuned)
    assert all(r["status"] == gdf.GDF_OK and r["rel_residual"] <= 1e-6 for r in rep)
    assert [r["rel_residual"] for r in rep] == [r["rel_residual"] for r in rep32]
    worst = 0.0
    for i in range(len(desc)):
        # the FP32 output is the FP64 one rounded
        assert torch.equal(f32[i], f64[i].float())
        worst = max(worst, _relres_torch(f64[i], gs[i], go[i], al[i]))
    print("worst recomputed rel. residual %.3e" % worst, flush=True)
    assert worst <= 1e-6 * (1 + 1e-6)
    # the three smallest slices, and the two smallest alphas among slices of at
    # most 1 Mpx (the largest error per unit of residual)
    small = sorted(range(len(desc)), key=lambda k: desc[k][0] * desc[k][1])[:3]
    low_a = sorted((k for k in range(len(desc)) if desc[k][0] * desc[k][1] <= 1 << 20),
                   key=lambda k: desc[k][2])[:2]
    for i in small + low_a:
        H, W, a, sd = desc[i]
        o, s = synth.batch_slice(H, W, sd)
        assert np.array_equal(o, go[i].cpu().numpy()) and np.abs(s - gs[i].cpu().numpy()).max() <= 1e-4
        fr = oracle.solve(s, o.astype(np.float64), a, tol=1e-11)
        err = np.abs(f32[i].cpu().numpy() - fr).max()
        print("slice", i, (H, W, a), "max abs err vs oracle %.2e" % err, flush=True)
        assert err <= 1e-3


def test_mixed_full_size_crops():
    S, H, W, alpha = 4, 21504, 26624, 0.01
    seed = synth.CONFIG_SEED[3]
    st = synth.make_stack_t(S, H, W, seed, DEV)
    print("stack generated", flush=True)
    f, rep = gdf.fuse_stack(st, alpha, tol=1e-8, precision="mixed")
    print([r["rel_residual"] for r in rep], flush=True)
    assert all(r["status"] == gdf.GDF_OK and r["rel_residual"] <= 1e-8 for r in rep)
    zs = [0, 3]
    for (y0, x0) in ((0, 0), (10240, 12800), (H - 1024, W - 1024)):
        fc, raw, (my0, mx0) = fuse_crop(seed, S, H, W, alpha, y0, y0 + 1024, x0, x0 + 1024, zs)
        dev_raw = st[:, my0:my0 + raw.shape[1], mx0:mx0 + raw.shape[2]].cpu().numpy()
        assert np.array_equal(raw, dev_raw)   # the oracle sees the GPU's input
        got = f[zs, y0:y0 + 1024, x0:x0 + 1024].cpu().numpy()
        err = np.abs(got - fc).max()
        print("crop", (y0, x0), "max abs err vs oracle %.2e" % err, flush=True)
        assert err <= 1e-4


def test_adjoint_full_size():
    S, H, W, alpha = 16, 1024, 1024, 0.01
    seed = synth.CONFIG_SEED[4]
    stack = synth.make_stack(S, H, W, seed)
    gs = oracle.smooth(stack)
    go = stack.astype(np.float64)
    t = np.random.default_rng(seed).uniform(0.0, 255.0, size=go.shape)
    G = lambda a, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dt)
    # FP32 autograd (the benchmark's configuration) against the oracle on two slices
    gs32 = G(gs, torch.float32).requires_grad_()
    go32 = G(go, torch.float32).requires_grad_()
    al = torch.tensor(alpha, device=DEV, requires_grad=True)
    f = gdf.ScreenedPoissonSolve.apply(gs32, go32, al)
    ((f - G(t, torch.float32)) ** 2).sum().backward()
    for j in (0, 11):
        fj = oracle.solve(gs[j], go[j], alpha, tol=1e-12)
        r_gs, r_go, r_a = oracle.adjoint(2.0 * (fj - t[j]), gs[j], fj, alpha)
        e_gs = np.abs(gs32.grad[j].cpu().numpy() - r_gs).max() / np.abs(r_gs).max()
        e_go = np.abs(go32.grad[j].cpu().numpy() - r_go).max() / np.abs(r_go).max()
        print("slice", j, "rel err dL/dg_s %.2e dL/dg_o %.2e" % (e_gs, e_go), flush=True)
        assert e_gs <= 2e-3 and e_go <= 2e-3
    # FP64 adjoint against central differences (eps 1e-3) on 32 voxels; the
    # loss is quadratic in g_s and g_o, so the differences are exact up to
    # rounding, and only the perturbed slice changes
    f64, _ = gdf.solve_slices(G(gs), G(go), alpha, tol=1e-13, precision="fp64", max_vcycles=200)
    f64 = f64.cpu().numpy()
    dgs, dgo, da, _ = gdf.solve_slices_backward(G(2.0 * (f64 - t)), G(f64), G(gs), alpha, tol=1e-12)
    dgs, dgo = dgs.cpu().numpy(), dgo.cpu().numpy()
    rng = np.random.default_rng(seed + 1)
    eps = 1e-3
    for _ in range(32):
        j, y, x = int(rng.integers(0, S)), int(rng.integers(0, H)), int(rng.integers(0, W))
        for which, grad in (("gs", dgs), ("go", dgo)):
            out = []
            for sgn in (1.0, -1.0):
                a_gs, a_go = gs[j].copy(), go[j].copy()
                (a_gs if which == "gs" else a_go)[y, x] += sgn * eps
                fj, _ = gdf.solve_slices(G(a_gs[None]), G(a_go[None]), alpha, tol=1e-13, precision="fp64",
                                         max_vcycles=200)
                out.append(fj[0].cpu().numpy())
            fd = np.sum((out[0] - out[1]) * (out[0] + out[1] - 2.0 * t[j])) / (2.0 * eps)
            assert abs(fd - grad[j, y, x]) <= 1e-5 * max(1.0, abs(grad[j, y, x])), (which, j, y, x, fd, grad[j, y, x])
