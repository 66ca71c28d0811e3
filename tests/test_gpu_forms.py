"""GPU checks of the three solver forms beside the plain solve -- FP64
iterative refinement around FP32 V-cycles, the adjoint solve behind the
autograd function, graph-captured uneven batches -- and of the plain solve at
the full 64 x 2048 x 2048 benchmark size (sampled against the oracle)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1506_02079_amd as gdf
import synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


# ------------------------------------------------------------------ mixed

@pytest.mark.parametrize("shape,alpha", [((4, 300, 257), 0.001), ((3, 256, 256), 0.01)])
def test_mixed_precision_reaches_1e8(shape, alpha):
    stack = synth.make_stack(*shape, seed=21 + shape[1], ramp=True)
    print("mixed", shape, alpha, flush=True)
    f, rep, gsm = gdf.fuse_stack(torch.from_numpy(stack).to(DEV), alpha, tol=1e-8,
                                 precision="mixed", return_smooth=True)
    f = f.cpu().numpy()
    assert f.dtype == np.float64
    gsm = gsm.cpu().numpy().astype(np.float64)
    f_ref = oracle.solve_stack(gsm, stack.astype(np.float64), alpha, tol=1e-13)
    err = np.abs(f - f_ref).max()
    rel = [oracle.relres(f[j], gsm[j], stack[j].astype(np.float64), alpha) for j in range(shape[0])]
    print("err", err, "rel", max(rel), [r["vcycles"] for r in rep])
    assert max(rel) <= 1e-8 * 1.01
    assert all(r["rel_residual"] <= 1e-8 for r in rep)
    assert err <= 1e-4


def test_mixed_solve_slices_float_inputs():
    gs, go = zip(*[(s, o.astype(np.float32)) for o, s in
                   (synth.batch_slice(H, W, 40 + H) for H, W in ((200, 300), (64, 64)))])
    tg = [torch.from_numpy(a).to(DEV) for a in gs]
    to = [torch.from_numpy(a).to(DEV) for a in go]
    f, rep = gdf.solve_slices(tg, to, [0.005, 0.05], tol=1e-9, precision="mixed")
    for i, a in enumerate((0.005, 0.05)):
        fr = oracle.solve(gs[i], go[i], a, tol=1e-13)
        assert np.abs(f[i].cpu().numpy() - fr).max() <= 1e-5
        assert oracle.relres(f[i].cpu().numpy(), gs[i], go[i], a) <= 1.01e-9


# ---------------------------------------------------------------- adjoint

def _adj_data(S, H, W, seed):
    stack = synth.make_stack(S, H, W, seed=seed)
    go = stack.astype(np.float64)
    gs = oracle.smooth(stack)
    t = np.random.default_rng(seed).uniform(0, 255, size=go.shape)
    return gs, go, t


@pytest.mark.parametrize("dtype,tol,rtol", [(torch.float64, 1e-11, 1e-7), (torch.float32, 1e-6, 2e-3)])
def test_adjoint_matches_oracle(dtype, tol, rtol):
    gs, go, t = _adj_data(3, 96, 130, 5)
    alpha = 0.01
    f = oracle.solve_stack(gs, go, alpha, tol=1e-13)
    gbar = 2 * (f - t)
    T = lambda a: torch.from_numpy(a).to(DEV, dtype)
    dgs, dgo, da, rep = gdf.solve_slices_backward(T(gbar), T(f), T(gs), alpha, tol=tol)
    for j in range(3):
        r_gs, r_go, r_a = oracle.adjoint(gbar[j], gs[j], f[j], alpha, tol=1e-13)
        scale = np.abs(r_gs).max()
        assert np.abs(dgs[j].cpu().numpy() - r_gs).max() <= rtol * scale
        assert np.abs(dgo[j].cpu().numpy() - r_go).max() <= rtol * np.abs(r_go).max()
        assert abs(float(da[j]) - r_a) <= rtol * abs(r_a) * 10
        assert rep[j]["rel_residual"] <= tol


def test_adjoint_central_differences():
    # loss = sum (f - t)^2 with the GPU FP64 solve; eps = 1e-3 at 32 voxels.
    # f is affine in g_s and g_o, so central differences are exact up to rounding.
    gs, go, t = _adj_data(2, 64, 80, 9)
    alpha = 0.01
    G = lambda a: torch.from_numpy(a).to(DEV)
    solve = lambda s, o: gdf.solve_slices(G(s), G(o), alpha, tol=1e-13, precision="fp64",
                                          max_vcycles=200)[0].cpu().numpy()
    f = solve(gs, go)
    dgs, dgo, da, _ = gdf.solve_slices_backward(G(2 * (f - t)), G(f), G(gs), alpha, tol=1e-12)
    dgs, dgo = dgs.cpu().numpy(), dgo.cpu().numpy()
    rng = np.random.default_rng(3)
    eps = 1e-3
    for _ in range(32):
        j, y, x = rng.integers(0, 2), rng.integers(0, 64), rng.integers(0, 80)
        for which, grad in (("gs", dgs), ("go", dgo)):
            p, m = (gs.copy(), gs.copy()) if which == "gs" else (go.copy(), go.copy())
            p[j, y, x] += eps
            m[j, y, x] -= eps
            fp = solve(p, go) if which == "gs" else solve(gs, p)
            fm = solve(m, go) if which == "gs" else solve(gs, m)
            fd = np.sum((fp - fm) * (fp + fm - 2 * t)) / (2 * eps)
            assert abs(fd - grad[j, y, x]) <= 1e-5 * max(1.0, abs(grad[j, y, x])), (which, fd, grad[j, y, x])


def test_autograd_gradcheck():
    torch.manual_seed(0)
    gs = (torch.rand(2, 8, 8, dtype=torch.float64, device=DEV) * 255).requires_grad_()
    go = (torch.rand(2, 8, 8, dtype=torch.float64, device=DEV) * 255).requires_grad_()
    alpha = torch.tensor(0.05, dtype=torch.float64, device=DEV, requires_grad=True)
    fn = lambda a, b, c: gdf.ScreenedPoissonSolve.apply(a, b, c, 1e-13)
    assert torch.autograd.gradcheck(fn, (gs, go, alpha), eps=1e-4, atol=1e-6, rtol=1e-5)


def test_autograd_loss_backward_fp32():
    stack = synth.make_stack(4, 128, 96, seed=77)
    gs = torch.from_numpy(oracle.smooth(stack).astype(np.float32)).to(DEV).requires_grad_()
    go = torch.from_numpy(stack.astype(np.float32)).to(DEV).requires_grad_()
    alpha = torch.tensor(0.01, device=DEV, requires_grad=True)
    tgt = torch.rand(4, 128, 96, device=DEV) * 255
    f = gdf.ScreenedPoissonSolve.apply(gs, go, alpha)
    ((f - tgt) ** 2).sum().backward()
    f64 = oracle.solve_stack(gs.detach().cpu().double().numpy(), stack.astype(np.float64), 0.01,
                             tol=1e-13)
    gbar = 2 * (f64 - tgt.cpu().double().numpy())
    da = 0.0
    for j in range(4):
        r_gs, r_go, r_a = oracle.adjoint(gbar[j], gs.detach().cpu().double().numpy()[j], f64[j], 0.01)
        assert np.abs(gs.grad[j].cpu().numpy() - r_gs).max() <= 2e-3 * np.abs(r_gs).max()
        assert np.abs(go.grad[j].cpu().numpy() - r_go).max() <= 2e-3 * np.abs(r_go).max()
        da += r_a
    assert abs(float(alpha.grad) - da) <= 5e-3 * abs(da)


# ----------------------------------------------------------- uneven batch

def test_graph_uneven_batch_moderate():
    desc = synth.uneven_batch(24, seed=2, max_side=1536)
    pairs = [synth.batch_slice(H, W, sd) for H, W, _, sd in desc]
    al = [a for _, _, a, _ in desc]
    tg = [torch.from_numpy(s).to(DEV) for _, s in pairs]
    to = [torch.from_numpy(o).to(DEV) for o, _ in pairs]
    f1, rep1 = gdf.solve_slices(tg, to, al, tol=1e-6, use_graph=True, max_vcycles=16)
    f2, rep2 = gdf.solve_slices(tg, to, al, tol=1e-6, use_graph=True, max_vcycles=16)   # replay
    f3, rep3 = gdf.solve_slices(tg, to, al, tol=1e-6, use_graph=False, max_vcycles=16)
    for i in range(len(desc)):
        assert torch.equal(f1[i], f2[i])
        assert torch.equal(f1[i], f3[i])
        assert rep1[i]["rel_residual"] <= 1e-6 and rep1[i]["status"] == gdf.GDF_OK
    for i in (0, 7, 23):
        o, s = pairs[i]
        fr = oracle.solve(s, o.astype(np.float64), al[i], tol=1e-11)
        err = np.abs(f1[i].cpu().numpy() - fr).max()
        print(desc[i], "err", err)
        assert err <= 1e-3


# ------------------------------------------------------ full benchmark size

def test_full_size_plain_fp32_sampled():
    S, H, W, alpha = 64, 2048, 2048, 0.01
    stack = synth.make_stack(S, H, W, seed=1001, ramp=True)
    print("generated", flush=True)
    f, rep, gsm = gdf.fuse_stack(torch.from_numpy(stack).to(DEV), alpha, tol=1e-6,
                                 return_smooth=True)
    assert all(r["status"] == gdf.GDF_OK and r["rel_residual"] <= 1e-6 for r in rep)
    rng = np.random.default_rng(0)
    # smoothing at sampled voxels, edges and corners included
    pts = np.stack([rng.integers(0, n, 4000) for n in (S, H, W)], axis=1)
    pts[:8] = [[0, 0, 0], [S - 1, H - 1, W - 1], [0, H - 1, 0], [S - 1, 0, W - 1],
               [5, 0, 100], [60, 2047, 5], [30, 1000, 0], [31, 7, 2047]]
    ref = oracle.smooth_points(stack, pts)
    got = gsm.cpu().numpy()[pts[:, 0], pts[:, 1], pts[:, 2]]
    assert np.abs(got - ref).max() <= 2e-4
    # whole slices through the oracle (edge slice and a middle one)
    for z in (0, 37):
        yy, xx = np.mgrid[0:H, 0:W]
        p = np.stack([np.full(H * W, z), yy.ravel(), xx.ravel()], axis=1)
        gs_z = oracle.smooth_points(stack, p).reshape(H, W)
        fz = oracle.solve(gs_z, stack[z].astype(np.float64), alpha, tol=1e-10)
        err = np.abs(f[z].cpu().numpy().astype(np.float64) - fz).max()
        print("slice", z, "max abs err", err, rep[z], flush=True)
        assert err <= 1e-3


# ----------------------------------------------- launch modes and autotuning

def test_persistent_launch_matches_grid():
    # 16-row items: several times more work items than the waves resident on
    # the chip, so the persistent grid really loops
    stack = synth.make_stack(8, 1024, 1024, seed=31, ramp=True)
    st = torch.from_numpy(stack).to(DEV)
    print("persistent vs grid", flush=True)
    f1, r1 = gdf.fuse_stack(st, 0.01, tile_rows=16, launch_mode="grid")
    f2, r2 = gdf.fuse_stack(st, 0.01, tile_rows=16, launch_mode="persistent")
    assert torch.equal(f1, f2)
    assert [r["vcycles"] for r in r1] == [r["vcycles"] for r in r2]
    assert all(r["rel_residual"] <= 1e-6 for r in r2)


def test_autotuned_uneven_batch_graph():
    desc = synth.uneven_batch(10, seed=4, max_side=1024)
    pairs = [synth.batch_slice(H, W, sd) for H, W, _, sd in desc]
    al = [a for _, _, a, _ in desc]
    tg = [torch.from_numpy(s).to(DEV) for _, s in pairs]
    to = [torch.from_numpy(o).to(DEV) for o, _ in pairs]
    print("autotune", [(H, W) for H, W, _, _ in desc], flush=True)
    f1, rep1 = gdf.solve_slices(tg, to, al, tol=1e-6, use_graph=True, autotune=True)
    t = gdf.autotune_last()
    print("tuned", t, flush=True)
    assert t["nu"] in (1, 2) and t["tile_rows"] in (0, 32, 64, 128, 256) and t["launch_mode"] in (1, 2)
    assert t["fine_sweeps"] in (0, 2 * t["nu"] + 1, 2 * t["nu"] + 2)
    assert t["coarse_sweeps"] in (0, t["nu"])
    assert all(r["rel_residual"] <= 1e-6 and r["status"] == gdf.GDF_OK for r in rep1)
    # cached choice: the same settings given explicitly reproduce the result
    f2, rep2 = gdf.solve_slices(tg, to, al, tol=1e-6, use_graph=True, **t)
    for a, b in zip(f1, f2):
        assert torch.equal(a, b)
    i = min(range(len(desc)), key=lambda k: desc[k][0] * desc[k][1])
    o, s = pairs[i]
    fr = oracle.solve(s, o.astype(np.float64), al[i], tol=1e-11)
    assert np.abs(f1[i].cpu().numpy() - fr).max() <= 1e-3


def test_fp32_floor_slice_escalates_to_refinement():
    # slice 56 of the seeded 512-slice uneven batch: 93% of it clips to 0, so
    # ||b|| is small against the correction and FP32 iterates stall near
    # 1.2e-6; the solver detects the stall and re-solves the slice with FP32
    # V-cycles inside FP64 refinement
    H, W, a, sd = synth.uneven_batch(512, seed=1002)[56]
    o, s = synth.batch_slice(H, W, sd)
    print("floor slice", H, W, a, flush=True)
    for graph in (False, True):
        f, rep = gdf.solve_slices([torch.from_numpy(s).to(DEV)], [torch.from_numpy(o).to(DEV)], [a],
                                  tol=1e-6, use_graph=graph)
        print(rep, flush=True)
        assert rep[0]["status"] == gdf.GDF_OK and rep[0]["rel_residual"] <= 1e-6
        assert rep[0]["vcycles"] < 40
        fr = oracle.solve(s, o.astype(np.float64), a, tol=1e-12)
        assert np.abs(f[0].cpu().numpy() - fr).max() <= 1e-3


def test_output_pass_row_and_quad_agree():
    # widths that are multiples of 4 with aligned outputs take the row-marching
    # output pass; a leading 3 x 3 slice shifts every later output off the
    # four-element grid and sends the whole call through the quad pass
    shapes = [(200, 260), (96, 512), (37, 4)]
    al = [0.01, 0.003, 0.05]
    pairs = [synth.batch_slice(H, W, 70 + i) for i, (H, W) in enumerate(shapes)]
    tg = [torch.from_numpy(s).to(DEV) for _, s in pairs]
    to = [torch.from_numpy(o).to(DEV) for o, _ in pairs]
    print("row vs quad output pass", shapes, flush=True)
    f1, r1 = gdf.solve_slices(tg, to, al, tol=1e-6)
    o3, s3 = synth.batch_slice(3, 3, 79)
    f2, r2 = gdf.solve_slices([torch.from_numpy(s3).to(DEV)] + tg, [torch.from_numpy(o3).to(DEV)] + to,
                              [0.02] + al, tol=1e-6)
    for i in range(len(shapes)):
        assert torch.equal(f1[i], f2[i + 1])
        assert r1[i]["vcycles"] == r2[i + 1]["vcycles"]
        assert abs(r1[i]["rel_residual"] - r2[i + 1]["rel_residual"]) <= 1e-9 * r1[i]["rel_residual"]
        assert r1[i]["rel_residual"] <= 1e-6 and r1[i]["status"] == gdf.GDF_OK
        o, s = pairs[i]
        fr = oracle.solve(s, o.astype(np.float64), al[i], tol=1e-11)
        assert np.abs(f1[i].cpu().numpy() - fr).max() <= 1e-3


@pytest.mark.parametrize("coarse_sweeps", [1, 2, 3])
def test_coarse_sweep_counts(coarse_sweeps):
    # sweeps on the coarse levels: same solution; three take no more cycles than two
    stack = synth.make_stack(4, 300, 412, seed=63, ramp=True)
    st = torch.from_numpy(stack).to(DEV)
    f2, r2 = gdf.fuse_stack(st, 0.003, tol=1e-6, coarse_sweeps=2)
    f1, r1, gsm = gdf.fuse_stack(st, 0.003, tol=1e-6, coarse_sweeps=coarse_sweeps, return_smooth=True)
    print(coarse_sweeps, [r["vcycles"] for r in r2], [r["vcycles"] for r in r1], flush=True)
    assert all(r["rel_residual"] <= 1e-6 and r["status"] == gdf.GDF_OK for r in r1)
    if coarse_sweeps == 3:
        assert sum(r["vcycles"] for r in r1) <= sum(r["vcycles"] for r in r2)
    g = gsm.cpu().numpy().astype(np.float64)
    for j in (0, 3):
        fr = oracle.solve(g[j], stack[j].astype(np.float64), 0.003, tol=1e-11)
        assert np.abs(f1[j].cpu().numpy() - fr).max() <= 1e-3


def test_default_coarse_sweeps_follow_screening():
    # default coarse sweeps: nu + 1, and nu on levels whose alpha 4^l is at least
    # 0.05.  At alpha 0.1 every coarse level qualifies, so the default run is the
    # explicit two-sweep run bit for bit (and not the explicit three-sweep one:
    # the plans are cached apart); at alpha 0.001 only the deep levels do.
    stack = synth.make_stack(3, 300, 412, seed=67, ramp=True)
    st = torch.from_numpy(stack).to(DEV)
    fd, rd = gdf.fuse_stack(st, 0.1, tol=1e-6)
    f2, r2 = gdf.fuse_stack(st, 0.1, tol=1e-6, coarse_sweeps=2)
    f3, r3 = gdf.fuse_stack(st, 0.1, tol=1e-6, coarse_sweeps=3)
    assert torch.equal(fd, f2)
    assert [r["vcycles"] for r in rd] == [r["vcycles"] for r in r2]
    assert not torch.equal(fd, f3)
    for a in (0.1, 0.001):
        f1, r1, gsm = gdf.fuse_stack(st, a, tol=1e-6, return_smooth=True)
        assert all(r["rel_residual"] <= 1e-6 and r["status"] == gdf.GDF_OK for r in r1)
        g = gsm.cpu().numpy().astype(np.float64)
        for j in (0, 2):
            fr = oracle.solve(g[j], stack[j].astype(np.float64), a, tol=1e-11)
            assert np.abs(f1[j].cpu().numpy() - fr).max() <= 1e-3


@pytest.mark.parametrize("nu,fine_sweeps", [(2, 5), (2, 6), (1, 3), (1, 4)])
def test_fused_pass_sweep_counts(nu, fine_sweeps):
    # more sweeps in the fused finest pass: same solution, fewer or equal cycles
    stack = synth.make_stack(5, 333, 270, seed=61, ramp=True)
    st = torch.from_numpy(stack).to(DEV)
    f0, r0 = gdf.fuse_stack(st, 0.01, tol=1e-6, nu=nu)
    f1, r1, gsm = gdf.fuse_stack(st, 0.01, tol=1e-6, nu=nu, fine_sweeps=fine_sweeps, return_smooth=True)
    print(nu, fine_sweeps, [r["vcycles"] for r in r0], [r["vcycles"] for r in r1], flush=True)
    assert all(r["rel_residual"] <= 1e-6 and r["status"] == gdf.GDF_OK for r in r1)
    assert sum(r["vcycles"] for r in r1) <= sum(r["vcycles"] for r in r0)
    g = gsm.cpu().numpy().astype(np.float64)
    for j in (0, 4):
        fr = oracle.solve(g[j], stack[j].astype(np.float64), 0.01, tol=1e-11)
        assert np.abs(f1[j].cpu().numpy() - fr).max() <= 1e-3


def test_robust_averaging_restores_corrupt_slices():
    # "Extensions and Applications": a constant stack with zeroed (missing)
    # interior slices.  Robust averaging leaves the zeros out of every window
    # (their weight share is below 1/5), so the low-frequency target stays
    # constant and the blend restores the missing slices; plain averaging
    # pulls the target down around them.
    # (more than a window apart: a window holding two odd slices can keep the
    # milder one, its distance being small against the other's)
    st = np.full((48, 96, 128), 140, np.uint8)
    st[12] = 0
    st[34, 48:] = 0   # the lower half of a slice, as in the paper's figure
    t = torch.from_numpy(st).to(DEV)
    f, rep, gsm = gdf.fuse_stack(t, 0.01, tol=1e-6, robust=True, return_smooth=True, out_dtype=gdf.DTYPE_F64)
    # (plain averaging leaves a step in the target of the slices next to the
    # half-zeroed one while their g_o is flat: FP32 V-cycles stall a hair above
    # tol there, and those slices are re-solved by FP64 refinement)
    fp, rep_p, gsp = gdf.fuse_stack(t, 0.01, tol=1e-6, return_smooth=True, out_dtype=gdf.DTYPE_F64)
    torch.cuda.synchronize()
    assert all(r["status"] == gdf.GDF_OK and r["rel_residual"] <= 1e-6 for r in rep_p)
    assert np.abs(gsm.cpu().numpy() - 140).max() <= 1e-3
    assert gsp.cpu().numpy()[12].max() < 130
    f = f.cpu().numpy()
    assert np.abs(f[12] - 140).max() <= 1e-2   # g_o = 0 there: f is the constant target
    assert np.abs(fp.cpu().numpy()[12] - 140).max() > 5
    assert all(r["status"] == gdf.GDF_OK for r in rep)


@pytest.mark.parametrize("robust", [False, True])
def test_blank_slices_default_call_matches_oracle(robust):
    # The paper's bad-data case ("Extensions and Applications"): one blank and
    # one half-blank slice in an EM-like stack, through the default call (no
    # smoothed stack returned, FP32).  Slices next to the blank ones can stall
    # at the FP32 floor; they are re-solved by FP64 refinement from g_s
    # smoothed again inside the workspace, so every slice reaches tol.
    st = synth.make_stack(40, 96, 128, seed=91, ramp=True)
    st[13] = 0
    st[27, 40:] = 0
    t = torch.from_numpy(st).to(DEV)
    print("blank slices, robust =", robust, flush=True)
    f, rep = gdf.fuse_stack(t, 0.01, tol=1e-6, robust=robust)
    torch.cuda.synchronize()
    print([r["vcycles"] for r in rep], max(r["rel_residual"] for r in rep), flush=True)
    assert all(r["status"] == gdf.GDF_OK and r["rel_residual"] <= 1e-6 for r in rep)
    f = f.cpu().numpy().astype(np.float64)
    # the GPU's own g_s (the same deterministic smoothing, returned by a second
    # call) defines the system each slice solves; the plain smoothing is also
    # checked against the oracle's (robust decisions at the threshold are
    # FP32 on the GPU, FP64 in the oracle: covered by the robust parity test)
    _, _, gsm = gdf.fuse_stack(t, 0.01, tol=1e-6, robust=robust, return_smooth=True)
    gs = gsm.cpu().numpy().astype(np.float64)
    if not robust:
        assert np.abs(gs - oracle.smooth(st)).max() <= 2e-4
    # (the FP64 output: the residual of an FP32-rounded f can exceed tol by its rounding)
    f64, rep64 = gdf.fuse_stack(t, 0.01, tol=1e-6, robust=robust, out_dtype=gdf.DTYPE_F64)
    f64 = f64.cpu().numpy()
    assert all(r["status"] == gdf.GDF_OK for r in rep64)
    for z in (0, 12, 13, 14, 26, 27, 28, 39):
        fr = oracle.solve(gs[z], st[z].astype(np.float64), 0.01, tol=1e-12)
        err = np.abs(f[z] - fr).max()
        rel = oracle.relres(f64[z], gs[z], st[z].astype(np.float64), 0.01)
        print("slice", z, "err %.2e rel %.2e" % (err, rel), flush=True)
        assert err <= 1e-3
        assert rel <= 1.01e-6


def _robust_margin(st, z, y, x, sxy=1.0, sz=3.0):
    """The oracle's decision margin at voxel (z, y, x): the smallest
    |(p - mu)^2 - 4 var| over the in-stack taps of the cross-slice window (how
    far each value is from the two-standard-deviation threshold), and the
    largest |p - mu|; p are the in-plane smoothed values (the oracle's
    smoothing with no cross-slice blur), mu and var their weighted mean and
    variance with the cross-slice Gaussian weights."""
    S = st.shape[0]
    rz = int(np.floor(3 * sz))
    zs = [zz for zz in range(z - rz, z + rz + 1) if 0 <= zz < S]
    pts = np.array([[zz, y, x] for zz in zs], dtype=np.int32)
    p = oracle.smooth_points(st, pts, sxy, 0.0)
    w = np.exp(-(np.array(zs) - z) ** 2 / (2 * sz * sz))
    mu = np.sum(w * p) / np.sum(w)
    var = np.sum(w * (p - mu) ** 2) / np.sum(w)
    return np.min(np.abs((p - mu) ** 2 - 4 * var)), np.max(np.abs(p - mu))


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_robust_averaging_matches_oracle(precision):
    # EM-like stack with a corrupt slice.  Whether a value lies within two
    # standard deviations is decided in FP32 on the GPU and in FP64 in the
    # oracle, so a value right at the threshold can go either way.  Every
    # voxel that differs by more than the smoothing bar must be such a tie:
    # with in-plane values off by at most e (FP32 rounding of a 49-tap sum of
    # values <= 255: e = 1e-3), p - mu is off by at most 2e and var by at most
    # 4 e M + 4 e^2 (M = max |p - mu|), so (p - mu)^2 - 4 var moves by at most
    # 20 e M + 20 e^2; a decision can flip only where the oracle's margin is
    # within that.  At most one voxel in a thousand may be such a tie.  The
    # solve is then checked against the oracle on the GPU's own smoothed stack.
    st = synth.make_stack(24, 70, 90, seed=51, ramp=True)
    st[11, 20:] = 3
    t = torch.from_numpy(st).to(DEV)
    f, rep, gsm = gdf.fuse_stack(t, 0.01, tol=1e-6, robust=True, precision=precision, return_smooth=True,
                                 out_dtype=gdf.DTYPE_F64)
    torch.cuda.synchronize()
    gs = gsm.cpu().numpy().astype(np.float64)
    ref = oracle.smooth_robust(st)
    bad = np.abs(gs - ref) > 2e-4
    print(precision, "voxels off", int(bad.sum()), "of", bad.size, "max err", float(np.abs(gs - ref).max()))
    assert bad.mean() <= 1e-3
    e = 1e-3
    for z, y, x in zip(*np.nonzero(bad)):
        margin, M = _robust_margin(st, z, y, x)
        print("tie at", (z, y, x), "margin %.3e bound %.3e" % (margin, 20 * e * M + 20 * e * e))
        assert margin <= 20 * e * M + 20 * e * e
    fr = oracle.solve_stack(gs, st.astype(np.float64), 0.01, tol=1e-12)
    assert np.abs(f.cpu().numpy() - fr).max() <= 1e-3
    assert all(r["status"] == gdf.GDF_OK for r in rep)


@pytest.mark.parametrize("shape,sxy,sz", [((9, 37, 70), 1.0, 3.0), ((4, 20, 9), 2.0, 1.0), ((6, 33, 40), 0.0, 4.0),
                                          ((5, 30, 72), 1.0, 3.0), ((3, 17, 48), 2.0, 3.0), ((3, 9, 1104), 1.0, 1.0), ((2, 150, 32), 1.0, 1.0),
                                          ((2, 6, 8), 2.5, 0.5), ((7, 12, 9), 1.0, 3.0)])
def test_smooth_transpose_matches_oracle(shape, sxy, sz):
    """Widths of a multiple of 4 take the fused 4-column x-y pass (radii 0, 3,
    6 and 7, a row wider than one workgroup's 1024 voxels, heights that are
    not a multiple of the 64-row segment), planes of a multiple of 4 voxels
    the 4-column z pass (12 x 9); the others the one-voxel forms."""
    rng = np.random.default_rng(sum(shape))
    g = rng.standard_normal(shape)
    out = gdf.smooth_transpose(torch.from_numpy(g).to(DEV, torch.float32), sxy, sz)
    torch.cuda.synchronize()
    ref = oracle.smooth_transpose(g, sxy, sz)
    assert np.abs(out.cpu().numpy() - ref).max() <= 1e-5 * np.abs(ref).max() + 1e-6


def test_smooth_transpose_unaligned_buffers():
    """Buffers 4 bytes off a 16-byte boundary (W a multiple of 4) take the
    one-voxel passes through the C ABI; both agree with the oracle."""
    S, H, W = 5, 21, 64
    n = S * H * W
    g = np.random.default_rng(5).standard_normal((S, H, W))
    buf_g = torch.zeros(n + 4, dtype=torch.float32, device=DEV)
    buf_o = torch.zeros(n + 4, dtype=torch.float32, device=DEV)
    buf_g[1:1 + n] = torch.from_numpy(g.reshape(-1)).to(DEV, torch.float32)
    L = gdf.lib()
    ws = L.gdf_smooth_transpose_workspace_size(S, H, W)
    work = torch.empty(ws + 16, dtype=torch.uint8, device=DEV)
    print("unaligned transpose", (S, H, W), flush=True)
    st = L.smooth_transpose(buf_g.data_ptr() + 4, S, H, W, 1.0, 3.0, buf_o.data_ptr() + 4, None,
                            work.data_ptr() + 4, ws, gdf._stream(DEV))
    assert st == 0, gdf.last_error()
    torch.cuda.synchronize()
    out = buf_o[1:1 + n].cpu().numpy().reshape(S, H, W)
    ref = oracle.smooth_transpose(g, 1.0, 3.0)
    assert np.abs(out - ref).max() <= 1e-5 * np.abs(ref).max() + 1e-6
    assert float(buf_o[0]) == 0.0 and float(buf_o[1 + n]) == 0.0   # nothing written outside


def test_fuse_stack_backward_matches_oracle():
    # dLoss/dstack = S^T (alpha lambda) + L lambda, lambda = A^-1 dLoss/df per
    # slice; the oracle's adjoint and transposed smoothing are pinned separately
    stack = synth.make_stack(6, 48, 64, seed=61, ramp=True)
    t = torch.from_numpy(stack).to(DEV)
    f, rep = gdf.fuse_stack(t, 0.02, tol=1e-8, precision="mixed", out_dtype=gdf.DTYPE_F64)
    rng = np.random.default_rng(3)
    gf = rng.standard_normal(stack.shape)
    gst, rep_b = gdf.fuse_stack_backward(torch.from_numpy(gf).to(DEV, torch.float32), f.to(torch.float32), t, 0.02,
                                         tol=1e-7)
    torch.cuda.synchronize()
    f64 = f.cpu().numpy()
    gs = oracle.smooth(stack)
    dgs = np.empty_like(gf)
    dgo = np.empty_like(gf)
    for z in range(stack.shape[0]):
        a, b, _ = oracle.adjoint(gf[z], gs[z], f64[z], 0.02, tol=1e-12)
        dgs[z], dgo[z] = a, b
    ref = oracle.smooth_transpose(dgs) + dgo
    err = np.abs(gst.cpu().numpy() - ref).max()
    print("stack gradient max err", err, "scale", np.abs(ref).max())
    assert err <= 1e-3 * np.abs(ref).max()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fuse_color_matches_oracle(precision):
    # colour value constraints with grey gradients: each channel is Eq. (1)
    # with g_s the channel and g_o the grey image; FP64 to 1e-8, and FP32 (the
    # benchmark's form) to 1e-6 with the FP64 residual recomputed on the CPU
    rng = np.random.default_rng(17)
    H, W = 90, 130
    base, _ = synth.batch_slice(H, W, 5)
    grey = base.astype(np.float64)
    color = np.stack([grey * 0.6 + 40, grey * 0.9, 200 - grey * 0.5]) + rng.normal(0, 2, (3, H, W))
    blur = oracle.smooth(np.clip(color, 0, 255).astype(np.uint8), 4.0, 0.0)   # low-frequency colour
    dt = torch.float64 if precision == "fp64" else torch.float32
    tol = 1e-8 if precision == "fp64" else 1e-6
    blur_in, grey_in = blur.astype(np.float32 if precision == "fp32" else np.float64), grey
    f, rep = gdf.fuse_color(torch.from_numpy(blur_in).to(DEV, dt), torch.from_numpy(grey_in).to(DEV, dt), 0.01,
                            tol=tol, precision=precision, out_dtype=gdf.DTYPE_F64)
    torch.cuda.synchronize()
    for c in range(3):
        g_c = blur_in[c].astype(np.float64)
        ref = oracle.solve(g_c, grey, 0.01, tol=1e-12)
        err = np.abs(f[c].cpu().numpy() - ref).max()
        rel = oracle.relres(f[c].cpu().numpy(), g_c, grey, 0.01)
        print(precision, "channel", c, "err %.2e rel %.2e" % (err, rel), flush=True)
        assert err <= (1e-4 if precision == "fp64" else 1e-3)
        assert rel <= tol * 1.01
        assert rep[c]["status"] == gdf.GDF_OK


# ------------------------------------------------------- host-resident stacks

def test_streamed_stack_matches_whole():
    """Chunks of 16 slices with their smoothing halos give each slice the same
    result as the whole-stack call (the solve is per slice, Eq. (1))."""
    S, H, W = 37, 96, 130
    stack = synth.make_stack(S, H, W, seed=77)
    print("streamed", (S, H, W), flush=True)
    host = torch.from_numpy(stack).pin_memory()
    f_s, rep_s = gdf.fuse_stack_streamed(host, 0.01, chunk=16)
    f_w, rep_w = gdf.fuse_stack(torch.from_numpy(stack).to(DEV), 0.01)
    assert f_s.device.type == "cpu" and f_s.shape == (S, H, W) and len(rep_s) == S
    diff = np.abs(f_s.numpy() - f_w.cpu().numpy()).max()
    print("max diff vs whole stack", diff)
    assert diff <= 1e-3
    assert all(r["status"] == 0 and r["rel_residual"] <= 1e-6 for r in rep_s)
    # slices next to chunk edges against the oracle
    gs = oracle.smooth(stack)
    for j in (0, 15, 16, 31, 32, 36):
        fr = oracle.solve(gs[j], stack[j].astype(np.float64), 0.01, tol=1e-12)
        assert np.abs(f_s[j].numpy() - fr).max() <= 1e-3, j


@pytest.mark.parametrize("precision,z0,z1", [("fp32", 10, 20), ("fp32", 0, 5), ("fp32", 27, 32),
                                              ("fp32", 31, 32), ("fp32", 0, 32), ("fp64", 3, 29),
                                              ("mixed", 12, 13)])
def test_fuse_stack_slice_range(precision, z0, z1):
    """z_range solves slices z0 .. z1 - 1 only, the others entering their
    cross-slice windows: g_s is the whole-stack one bit for bit, f matches
    the whole-stack call and the oracle, the report has one entry per slice."""
    S, H, W = 32, 70, 150
    stack = synth.make_stack(S, H, W, seed=91, ramp=True)
    st = torch.from_numpy(stack).to(DEV)
    tol = {"fp32": 1e-6, "fp64": 1e-10, "mixed": 1e-8}[precision]
    print("slice range", precision, (z0, z1), flush=True)
    f_r, rep_r, gs_r = gdf.fuse_stack(st, 0.01, tol=tol, precision=precision, return_smooth=True, z_range=(z0, z1))
    f_w, rep_w, gs_w = gdf.fuse_stack(st, 0.01, tol=tol, precision=precision, return_smooth=True)
    f_n, rep_n = gdf.fuse_stack(st, 0.01, tol=tol, precision=precision, z_range=(z0, z1))   # no g_s output
    torch.cuda.synchronize()
    assert f_r.shape == (z1 - z0, H, W) and gs_r.shape == (z1 - z0, H, W) and len(rep_r) == z1 - z0
    assert torch.equal(gs_r, gs_w[z0:z1])
    bound = {"fp32": 1e-3, "fp64": 1e-6, "mixed": 1e-4}[precision]
    assert (f_r - f_w[z0:z1]).abs().max().item() <= bound
    assert (f_n - f_w[z0:z1]).abs().max().item() <= bound
    assert all(r["status"] == gdf.GDF_OK and r["rel_residual"] <= tol for r in rep_r + rep_n)
    gs = oracle.smooth(stack)
    for j in sorted({z0, z1 - 1}):
        fr = oracle.solve(gs[j], stack[j].astype(np.float64), 0.01, tol=1e-12)
        err = np.abs(f_r[j - z0].cpu().numpy().astype(np.float64) - fr).max()
        print("slice", j, "err %.2e" % err, flush=True)
        assert err <= bound


@pytest.mark.parametrize("precision,z_range", [("fp32", None), ("fp32", (4, 9)), ("mixed", None),
                                              ("fp64", (0, 3))])
def test_fuse_stack_graph_replays(precision, z_range):
    """use_graph: the captured schedule (smoothing, cycles, device-side
    convergence) replayed three times, with eager calls in between, gives the
    eager result each time."""
    S, H, W = 12, 90, 140
    stack = synth.make_stack(S, H, W, seed=93, ramp=True)
    st = torch.from_numpy(stack).to(DEV)
    tol = {"fp32": 1e-6, "fp64": 1e-10, "mixed": 1e-8}[precision]
    kw = dict(tol=tol, precision=precision, z_range=z_range, max_vcycles=12)
    f_e, rep_e = gdf.fuse_stack(st, 0.01, **kw)
    out = torch.empty_like(f_e)
    for i in range(3):
        print("graph replay", precision, z_range, i, flush=True)
        f_g, rep_g = gdf.fuse_stack(st, 0.01, use_graph=True, **kw)
        torch.cuda.synchronize()
        assert (f_g - f_e).abs().max().item() <= (1e-3 if precision == "fp32" else 1e-6)
        assert all(r["status"] == gdf.GDF_OK and r["rel_residual"] <= tol for r in rep_g)
        assert [r["vcycles"] for r in rep_g] == [r["vcycles"] for r in rep_e]
        out.copy_(gdf.fuse_stack(st, 0.02, tol=tol, precision=precision, z_range=z_range)[0])   # eager work between
    # asynchronous: no report, nothing waits; the caller's stream orders the result
    f_a, rep_a = gdf.fuse_stack(st, 0.01, use_graph=True, wait=False, **kw)
    assert rep_a is None
    assert (f_a - f_e).abs().max().item() <= (1e-3 if precision == "fp32" else 1e-6)
    with pytest.raises(ValueError):
        gdf.fuse_stack(st, 0.01, wait=False, **kw)


@pytest.mark.parametrize("shape", [(7, 33, 64), (5, 21, 37)])
def test_smooth_transpose_adds_in_place(shape):
    """out = K (G / D) + add with add = out (accumulate in place), on the
    four-column passes (W = 64) and the one-voxel passes (W = 37)."""
    rng = np.random.default_rng(sum(shape) + 1)
    g = rng.standard_normal(shape)
    base = rng.standard_normal(shape)
    acc = torch.from_numpy(base).to(DEV, torch.float32)
    out = gdf.smooth_transpose(torch.from_numpy(g).to(DEV, torch.float32), 1.0, 3.0, add=acc)
    torch.cuda.synchronize()
    assert out.data_ptr() == acc.data_ptr()
    ref = oracle.smooth_transpose(g, 1.0, 3.0) + base
    assert np.abs(out.cpu().numpy() - ref).max() <= 1e-5 * np.abs(ref).max() + 1e-6


def test_backward_alpha_sum_on_device():
    """The device total of dLoss/dalpha equals the sum of the per-slice terms
    (and the oracle's)."""
    gs, go, t = _adj_data(4, 64, 90, 15)
    alpha = 0.01
    f = oracle.solve_stack(gs, go, alpha, tol=1e-13)
    gbar = 2 * (f - t)
    T = lambda a: torch.from_numpy(a).to(DEV, torch.float64)
    _, _, per, _ = gdf.solve_slices_backward(T(gbar), T(f), T(gs), alpha, tol=1e-11, need=(False, False, True))
    _, _, tot, _ = gdf.solve_slices_backward(T(gbar), T(f), T(gs), alpha, tol=1e-11, need=(False, False, True),
                                             alpha_sum=True)
    assert tot.is_cuda and tot.dim() == 0
    ref = sum(oracle.adjoint(gbar[j], gs[j], f[j], alpha, tol=1e-13)[2] for j in range(4))
    assert abs(float(tot) - float(per.sum())) <= 1e-12 * abs(ref)
    assert abs(float(tot) - ref) <= 1e-7 * abs(ref)
