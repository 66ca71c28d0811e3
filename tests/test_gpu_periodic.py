"""GPU parity of the periodic (wrap-around) boundary, the paper's Fourier basis
(Section III-B, frequency-space interpretation), against the oracle's
periodic solve (pinned on the CPU by the FFT closed form): small, odd, prime
and one- and two-pixel sides (a two-pixel side couples its pixels across both
faces), uneven batches with and without graph capture, the whole method on a
stack, mixed precision, and the adjoint."""
import numpy as np
import pytest
import torch

import oracle
import paper_1506_02079_amd as gdf
import synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _pair(H, W, seed):
    """EM-like slices (generator); small ones can clip to a constant, so the
    small shapes below take _rand_pair."""
    o, s = synth.batch_slice(H, W, seed)
    return o.astype(np.float64), s.astype(np.float64)


def _rand_pair(H, W, seed):
    """Random intensities g_o and a target g_s = g_o + noise (never constant)."""
    rng = np.random.default_rng(seed)
    o = rng.integers(0, 256, size=(H, W)).astype(np.float64)
    return o, o + rng.normal(0, 20, size=(H, W))


SHAPES = [(16, 16), (17, 23), (33, 27), (2, 7), (1, 31), (64, 48), (129, 257), (3, 3), (1, 1), (2, 2), (300, 5)]


@pytest.mark.parametrize("H,W", SHAPES)
def test_periodic_fp64_matches_oracle(H, W):
    o, s = _rand_pair(H, W, 500 + H * 7 + W)
    for alpha in (0.01, 0.3):
        print("periodic fp64", (H, W), alpha, flush=True)
        f, rep = gdf.solve_slices(torch.from_numpy(s[None]).to(DEV), torch.from_numpy(o[None]).to(DEV), alpha,
                                  bc="periodic", tol=1e-11, precision="fp64", max_vcycles=200)
        fr = oracle.solve(s, o, alpha, "periodic", tol=1e-13)
        err = np.abs(f[0].cpu().numpy() - fr).max()
        rel = oracle.relres(f[0].cpu().numpy(), s, o, alpha, "periodic")
        print("err %.2e rel %.2e" % (err, rel), rep[0], flush=True)
        assert rep[0]["status"] == gdf.GDF_OK and rel <= 1.01e-11
        assert rep[0]["rel_residual_init"] > 0.0   # a nontrivial system
        assert abs(rep[0]["rel_residual"] - rel) <= 1e-2 * rel + 1e-14
        assert err <= 1e-6


@pytest.mark.parametrize("use_graph", [False, True])
def test_periodic_fp32_uneven_batch(use_graph):
    sizes = [(256, 256), (77, 130), (1, 50), (33, 1), (129, 257), (512, 96), (3, 3), (2, 64)]
    rng = np.random.default_rng(8)
    pairs = [_rand_pair(H, W, 700 + i) for i, (H, W) in enumerate(sizes)]
    al = [float(rng.uniform(0.001, 0.1)) for _ in sizes]
    tg = [torch.from_numpy(s.astype(np.float32)).to(DEV) for _, s in pairs]
    to = [torch.from_numpy(o.astype(np.float32)).to(DEV) for o, _ in pairs]
    for rep_i in range(2 if use_graph else 1):
        print("periodic fp32 batch, graph", use_graph, "call", rep_i, flush=True)
        f, rep = gdf.solve_slices(tg, to, al, bc="periodic", tol=1e-6, use_graph=use_graph,
                                  out_dtype=gdf.DTYPE_F64)
        for i, (H, W) in enumerate(sizes):
            o, s = pairs[i]
            s32 = s.astype(np.float32).astype(np.float64)
            fr = oracle.solve(s32, o, al[i], "periodic", tol=1e-12)
            fi = f[i].cpu().numpy()
            err = np.abs(fi - fr).max()
            rel = oracle.relres(fi, s32, o, al[i], "periodic")
            # (random intensities make ||L g_o|| large, so a relative residual of
            # 1e-6 allows errors above 1e-3 there; the bound that holds is
            # ||f - f*|| <= ||r|| / alpha, lambda_min(A) = alpha)
            bound = max(1e-3, 1.01 * rel * np.linalg.norm(oracle.rhs(s32, o, al[i], "periodic")) / al[i])
            print((H, W), al[i], "err %.2e (bound %.2e) rel %.2e" % (err, bound, rel), rep[i], flush=True)
            assert err <= bound
            assert rel <= 1.01e-6
            assert rep[i]["status"] == gdf.GDF_OK
            # the reported residual is the one recomputed here (of the unrounded f)
            assert abs(rep[i]["rel_residual"] - rel) <= 1e-3 * rel + 1e-12


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-6), ("mixed", 1e-8), ("fp64", 1e-10)])
def test_periodic_fuse_stack_matches_oracle(precision, tol):
    # the smoothing is the same for either boundary (renormalised at the stack's
    # edges); the blend wraps
    stack = synth.make_stack(6, 96, 131, seed=811, ramp=True)
    print("periodic fuse_stack", precision, flush=True)
    f, rep, gsm = gdf.fuse_stack(torch.from_numpy(stack).to(DEV), 0.005, bc="periodic", tol=tol,
                                 precision=precision, return_smooth=True, out_dtype=gdf.DTYPE_F64)
    f2, rep2 = gdf.fuse_stack(torch.from_numpy(stack).to(DEV), 0.005, bc="periodic", tol=tol, precision=precision)
    torch.cuda.synchronize()
    gs = gsm.cpu().numpy().astype(np.float64)
    assert np.abs(gs - oracle.smooth(stack)).max() <= (1e-9 if precision == "fp64" else 2e-4)
    f = f.cpu().numpy()
    for z in range(stack.shape[0]):
        fr = oracle.solve(gs[z], stack[z].astype(np.float64), 0.005, "periodic", tol=1e-13)
        err = np.abs(f[z] - fr).max()
        rel = oracle.relres(f[z], gs[z], stack[z].astype(np.float64), 0.005, "periodic")
        print("slice", z, "err %.2e rel %.2e" % (err, rel), rep[z], flush=True)
        assert err <= (1e-4 if precision != "fp32" else 1e-3)
        assert rel <= tol * 1.01
        assert np.abs(f2[z].cpu().numpy().astype(np.float64) - fr).max() <= 1e-3
    assert all(r["status"] == gdf.GDF_OK for r in rep + rep2)


@pytest.mark.parametrize("dtype,tol,rtol", [(torch.float64, 1e-11, 1e-7), (torch.float32, 1e-6, 2e-3)])
def test_periodic_adjoint_matches_oracle(dtype, tol, rtol):
    rng = np.random.default_rng(12)
    stack = synth.make_stack(3, 70, 91, seed=813)
    go = stack.astype(np.float64)
    gs = oracle.smooth(stack)
    t = rng.uniform(0, 255, size=go.shape)
    alpha = 0.02
    f = oracle.solve_stack(gs, go, alpha, "periodic", tol=1e-13)
    gbar = 2 * (f - t)
    T = lambda a: torch.from_numpy(a).to(DEV, dtype)
    print("periodic adjoint", dtype, flush=True)
    dgs, dgo, da, rep = gdf.solve_slices_backward(T(gbar), T(f), T(gs), alpha, bc="periodic", tol=tol)
    for j in range(3):
        r_gs, r_go, r_a = oracle.adjoint(gbar[j], gs[j], f[j], alpha, "periodic", tol=1e-13)
        e_gs = np.abs(dgs[j].cpu().numpy() - r_gs).max() / np.abs(r_gs).max()
        e_go = np.abs(dgo[j].cpu().numpy() - r_go).max() / np.abs(r_go).max()
        print("slice", j, "rel err %.2e %.2e" % (e_gs, e_go), float(da[j]), r_a, flush=True)
        assert e_gs <= rtol and e_go <= rtol
        assert abs(float(da[j]) - r_a) <= rtol * abs(r_a) * 10
        assert rep[j]["rel_residual"] <= tol


def test_periodic_many_levels_low_alpha():
    # alpha 0.001 on 512 x 700: six levels, odd coarse sides (700 -> 350 -> 175
    # -> 88 ...), FP32 to 1e-6
    o, s = _pair(512, 700, 907)
    print("periodic 512 x 700 alpha 0.001", flush=True)
    f, rep = gdf.solve_slices(torch.from_numpy(s.astype(np.float32)[None]).to(DEV),
                              torch.from_numpy(o.astype(np.float32)[None]).to(DEV), 0.001, bc="periodic",
                              tol=1e-6, out_dtype=gdf.DTYPE_F64)
    s32 = s.astype(np.float32).astype(np.float64)
    fr = oracle.solve(s32, o, 0.001, "periodic", tol=1e-12)
    err = np.abs(f[0].cpu().numpy() - fr).max()
    print("err %.2e" % err, rep[0], flush=True)
    assert rep[0]["status"] == gdf.GDF_OK and rep[0]["vcycles"] <= 20
    assert err <= 1e-3
