"""GPU parity at the extremes of the input sizes: the widest slice the library
takes (4194304 columns), a 100000-row slice three columns wide, and a batch
of 3000 tiny uneven slices (1 to 40 pixels a side) in one captured launch."""
import numpy as np
import pytest
import torch

import oracle
import paper_1506_02079_amd as gdf
import synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
W_MAX = 4194304


def _rand_pair(H, W, seed):
    rng = np.random.default_rng(seed)
    o = rng.integers(0, 256, size=(H, W)).astype(np.float64)
    return o, np.clip(o + rng.normal(0, 30, size=(H, W)), 0, 255)


@pytest.mark.parametrize("H,W", [(1, W_MAX), (2, W_MAX), (100000, 3)])
def test_extreme_shapes_match_oracle(H, W):
    o, s = _rand_pair(H, W, H + 7)
    print("extreme shape", (H, W), flush=True)
    f, rep = gdf.solve_slices(torch.from_numpy(s.astype(np.float32)[None]).to(DEV),
                              torch.from_numpy(o.astype(np.float32)[None]).to(DEV), 0.01, tol=1e-6,
                              out_dtype=gdf.DTYPE_F64)
    s32 = s.astype(np.float32).astype(np.float64)
    fr = oracle.solve(s32, o, 0.01, tol=1e-12)
    fg = f[0].cpu().numpy()
    err = np.abs(fg - fr).max()
    rel = oracle.relres(fg, s32, o, 0.01)
    # (random intensities make ||L g_o|| large, so a relative residual of 1e-6
    # allows errors above 1e-3; the bound that holds is ||f - f*|| <= ||r|| / alpha)
    bound = max(1e-3, 1.01 * rel * np.linalg.norm(oracle.rhs(s32, o, 0.01)) / 0.01)
    print("err %.2e (bound %.2e) rel %.2e" % (err, bound, rel), rep[0], flush=True)
    assert rep[0]["status"] == gdf.GDF_OK and rel <= 1.01e-6
    assert err <= bound


def test_widest_stack_smoothing_sampled():
    """fuse_stack on 3 slices of 2 x 4194304: smoothing at sampled voxels and
    one slice's solve against the oracle."""
    S, H, W = 3, 2, W_MAX
    rng = np.random.default_rng(5)
    stack = rng.integers(0, 256, size=(S, H, W), dtype=np.uint8)
    print("widest stack", (S, H, W), flush=True)
    f, rep, gsm = gdf.fuse_stack(torch.from_numpy(stack).to(DEV), 0.01, tol=1e-6, return_smooth=True,
                                 out_dtype=gdf.DTYPE_F64)
    pts = np.stack([rng.integers(0, S, 3000), rng.integers(0, H, 3000), rng.integers(0, W, 3000)], axis=1)
    pts[:6] = [[0, 0, 0], [2, 1, W - 1], [1, 0, W - 1], [1, 1, 0], [0, 1, W // 2], [2, 0, 63]]
    ref = oracle.smooth_points(stack, pts.astype(np.int32))
    g = gsm.cpu().numpy()[pts[:, 0], pts[:, 1], pts[:, 2]].astype(np.float64)
    assert np.abs(g - ref).max() <= 2e-4
    z = 1
    gs = gsm[z].cpu().numpy().astype(np.float64)
    fr = oracle.solve(gs, stack[z].astype(np.float64), 0.01, tol=1e-12)
    fz = f[z].cpu().numpy()
    go = stack[z].astype(np.float64)
    err = np.abs(fz - fr).max()
    rel = oracle.relres(fz, gs, go, 0.01)
    bound = max(1e-3, 1.01 * rel * np.linalg.norm(oracle.rhs(gs, go, 0.01)) / 0.01)   # (random data, as above)
    print("slice", z, "err %.2e (bound %.2e) rel %.2e" % (err, bound, rel), rep[z], flush=True)
    assert err <= bound and rel <= 1.01e-6 and all(r["status"] == gdf.GDF_OK for r in rep)


def test_many_tiny_slices_one_graph():
    rng = np.random.default_rng(3000)
    n = 3000
    sizes = [(int(rng.integers(1, 41)), int(rng.integers(1, 41))) for _ in range(n)]
    al = [float(rng.uniform(0.001, 0.5)) for _ in range(n)]
    pairs = [_rand_pair(H, W, 20000 + i) for i, (H, W) in enumerate(sizes)]
    tg = [torch.from_numpy(s.astype(np.float32)).to(DEV) for _, s in pairs]
    to = [torch.from_numpy(o.astype(np.float32)).to(DEV) for o, _ in pairs]
    print("tiny slices", n, flush=True)
    for rep_i in range(2):   # capture, then replay
        f, rep = gdf.solve_slices(tg, to, al, tol=1e-6, use_graph=True, max_vcycles=30, out_dtype=gdf.DTYPE_F64)
        worst = 0.0
        for i in range(0, n, 7):   # every seventh slice against the oracle (bound as above)
            o, s = pairs[i]
            s32 = s.astype(np.float32).astype(np.float64)
            fr = oracle.solve(s32, o, al[i], tol=1e-13)
            fi = f[i].cpu().numpy()
            rel = oracle.relres(fi, s32, o, al[i])
            bound = max(1e-3, 1.01 * rel * np.linalg.norm(oracle.rhs(s32, o, al[i])) / al[i])
            worst = max(worst, np.abs(fi - fr).max() / bound)
        print("replay", rep_i, "worst err / bound %.2f" % worst, flush=True)
        assert worst <= 1.0
        assert all(r["status"] == gdf.GDF_OK and r["rel_residual"] <= 1e-6 for r in rep)
