"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bars: max |f_gpu - f_oracle| <= 1e-3 on 0-255 intensities; FP64 relative
residual <= tol for every slice, both as reported by the library and as
recomputed here on the CPU from an FP64 copy of the output.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1506_02079_amd as gdf
import synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
ABS_TOL = 1e-3


def _relres_stack(f, gs, go, alpha):
    return [oracle.relres(f[j], gs[j], go[j], alpha) for j in range(f.shape[0])]


def _run_fuse(stack, alpha, precision, tol, **kw):
    print("fuse_stack", stack.shape, alpha, precision, tol, flush=True)
    t = torch.from_numpy(stack).to(DEV)
    f, rep, gsm = gdf.fuse_stack(t, alpha, tol=tol, precision=precision, return_smooth=True,
                                 out_dtype=gdf.DTYPE_F64, **kw)
    torch.cuda.synchronize()
    return f.cpu().numpy(), rep, gsm.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fuse_stack_small_config(precision):
    # 8 slices of 256 x 256, alpha = 0.01, Neumann, to 1e-6
    stack = synth.make_stack(8, 256, 256, seed=synth.CONFIG_SEED[0])
    alpha, tol = 0.01, 1e-6
    f, rep, gsm = _run_fuse(stack, alpha, precision, tol)
    f_ref, gs_ref = oracle.fuse_stack(stack, alpha, tol=1e-12)
    smooth_tol = 1e-10 if precision == "fp64" else 2e-4
    assert np.abs(gsm - gs_ref).max() <= smooth_tol
    err = np.abs(f - f_ref).max()
    print("max abs err", err, "vcycles", [r["vcycles"] for r in rep])
    assert err <= ABS_TOL
    for r in rep:
        assert r["status"] == gdf.GDF_OK and r["rel_residual"] <= tol
    # independent residual check on the CPU (against the GPU's own g_s)
    cpu_rel = _relres_stack(f, gsm, stack.astype(np.float64), alpha)
    for r, c in zip(rep, cpu_rel):
        assert c <= tol * 1.01
        assert abs(c - r["rel_residual"]) <= 1e-3 * tol + 1e-3 * c


@pytest.mark.parametrize("shape,alpha", [((12, 203, 331), 0.01), ((3, 77, 130), 0.001),
                                         ((1, 64, 300), 0.1), ((20, 33, 17), 0.05),
                                         ((5, 1, 97), 0.01), ((4, 129, 1), 0.01),
                                         ((2, 1, 1), 0.3), ((9, 250, 260), 5.0)])
def test_fuse_stack_ragged_fp32(shape, alpha):
    stack = synth.make_stack(*shape, seed=7 + shape[1], ramp=True)
    tol = 1e-6
    f, rep, gsm = _run_fuse(stack, alpha, "fp32", tol)
    f_ref, gs_ref = oracle.fuse_stack(stack, alpha, tol=1e-12)
    assert np.abs(gsm - gs_ref).max() <= 2e-4
    err = np.abs(f - f_ref).max()
    print("max abs err", err, "vcycles", [r["vcycles"] for r in rep])
    assert err <= ABS_TOL
    cpu_rel = _relres_stack(f, gsm, stack.astype(np.float64), alpha)
    assert max(cpu_rel) <= tol * 1.01
    assert all(r["status"] == gdf.GDF_OK for r in rep)


def _uneven(sizes, seed):
    """EM-like slices: g_o from the stack generator, g_s its in-plane-blurred base."""
    rng = np.random.default_rng(seed)
    gs, go, al = [], [], []
    for i, (H, W) in enumerate(sizes):
        o, s = synth.batch_slice(H, W, seed * 1000 + i)
        go.append(o.astype(np.float32))
        gs.append(s)
        al.append(float(rng.uniform(0.001, 0.1)))
    return gs, go, al


@pytest.mark.parametrize("use_graph", [False, True])
def test_solve_slices_uneven_batch(use_graph):
    sizes = [(256, 256), (77, 130), (1, 1), (1, 50), (33, 1), (129, 257), (512, 96), (3, 3)]
    gs, go, al = _uneven(sizes, 3)
    tg = [torch.from_numpy(a).to(DEV) for a in gs]
    to = [torch.from_numpy(a).to(DEV) for a in go]
    tol = 1e-6
    for rep_i in range(2 if use_graph else 1):
        f, rep = gdf.solve_slices(tg, to, al, tol=tol, use_graph=use_graph, max_vcycles=30,
                                  out_dtype=gdf.DTYPE_F64)
        torch.cuda.synchronize()
        for i in range(len(sizes)):
            fr = oracle.solve(gs[i], go[i], al[i], tol=1e-12)
            fi = f[i].cpu().numpy()
            err = np.abs(fi - fr).max()
            rel = oracle.relres(fi, gs[i], go[i], al[i])
            print(sizes[i], al[i], "err", err, "rel", rel, rep[i])
            assert err <= ABS_TOL
            assert rel <= tol * 1.01
            assert rep[i]["status"] == gdf.GDF_OK


def test_uint8_orig_and_fp64_solve():
    stack = synth.make_stack(4, 100, 120, seed=11)
    gs = oracle.smooth(stack)
    tg = torch.from_numpy(gs).to(DEV)
    to = torch.from_numpy(stack).to(DEV)
    f, rep = gdf.solve_slices(tg, to, 0.02, tol=1e-10, precision="fp64")
    ref = oracle.solve_stack(gs, stack.astype(np.float64), 0.02, tol=1e-13)
    assert np.abs(f.cpu().numpy() - ref).max() <= 1e-6
    assert all(r["rel_residual"] <= 1e-10 for r in rep)


def test_identical_inputs_give_input():
    stack = synth.make_stack(2, 90, 70, seed=12).astype(np.float32)
    t = torch.from_numpy(stack).to(DEV)
    f, rep = gdf.solve_slices(t, t, 0.01, tol=1e-6)
    assert np.abs(f.cpu().numpy() - stack).max() <= 1e-4


def test_deterministic():
    stack = synth.make_stack(4, 300, 200, seed=13, ramp=True)
    t = torch.from_numpy(stack).to(DEV)
    f1, r1 = gdf.fuse_stack(t, 0.01)
    f2, r2 = gdf.fuse_stack(t, 0.01)
    assert torch.equal(f1, f2)
    assert [r["rel_residual"] for r in r1] == [r["rel_residual"] for r in r2]


def test_noconv_reported():
    stack = synth.make_stack(2, 128, 128, seed=14)
    t = torch.from_numpy(stack).to(DEV)
    f, rep = gdf.fuse_stack(t, 0.01, tol=1e-9, max_vcycles=1, allow_noconv=True)
    assert all(r["status"] == gdf.GDF_ENOCONV and r["vcycles"] == 1 for r in rep)
    with pytest.raises(gdf.GdfError):
        gdf.fuse_stack(t, 0.01, tol=1e-9, max_vcycles=1)


@pytest.mark.parametrize("shape,alpha", [((6, 129, 257), 0.01), ((5, 200, 131), 0.003), ((3, 65, 33), 0.05)])
def test_fused_restriction_matches_restriction_pass(shape, alpha):
    # fuse_stack restricts the unshifted level-0 right-hand side inside the
    # smoothing pass and removes the mean's share (4 wx wy children) in the first
    # level-1 pass; solve_slices on the same g_s and g_o restricts the shifted one
    # in a pass of its own.  Odd sizes give partial last cells (wx, wy = 1/2), and
    # the illumination ramp a large mean.  Both solve the same system.  The
    # bfloat16 level-1 values differ by rounding (the unshifted sums are larger),
    # which can cost a slice right at tol one more cycle; a missing or wrong mean
    # correction would cost every slice one.
    stack = synth.make_stack(*shape, seed=29 + shape[2], ramp=True)
    t = torch.from_numpy(stack).to(DEV)
    f1, rep1, gsm = gdf.fuse_stack(t, alpha, tol=1e-6, return_smooth=True)
    go = t.to(torch.float32)
    f2, rep2 = gdf.solve_slices([gsm[z] for z in range(shape[0])], [go[z] for z in range(shape[0])], alpha,
                                tol=1e-6)
    torch.cuda.synchronize()
    c1 = [r["vcycles"] for r in rep1]
    c2 = [r["vcycles"] for r in rep2]
    print(shape, alpha, "cycles fused", c1, "separate", c2)
    assert sum(c1) <= sum(c2) + shape[0] // 2
    assert all(r["status"] == gdf.GDF_OK and r["rel_residual"] <= 1e-6 for r in rep1 + rep2)
    f2s = torch.stack([x for x in f2]).cpu().numpy()
    assert np.abs(f1.cpu().numpy() - f2s).max() <= ABS_TOL


@pytest.mark.parametrize("sigma_xy,sigma_z,precision", [(0.5, 1.0, "fp32"), (2.0, 0.0, "fp32"), (1.0, 4.0, "fp32"),
                                                         (0.0, 2.0, "fp32"), (2.3, 1.5, "fp64")])
def test_smoothing_radii(sigma_xy, sigma_z, precision):
    # other truncation radii than the default (3 in-plane, 9 across): the
    # in-plane radius selects the kernel instance (3 or up to 7), the cross-slice
    # radius another (0 to 12); odd sizes, stacks shallower than the cross-slice
    # reach, and the restriction into level 1 with an odd slice count per tile
    stack = synth.make_stack(7, 61, 75, seed=41, ramp=True)
    t = torch.from_numpy(stack).to(DEV)
    f, rep, gsm = gdf.fuse_stack(t, 0.02, tol=1e-6, sigma_xy=sigma_xy, sigma_z=sigma_z, precision=precision,
                                 return_smooth=True, out_dtype=gdf.DTYPE_F64)
    torch.cuda.synchronize()
    gs_ref = oracle.smooth(stack, sigma_xy, sigma_z)
    gerr = np.abs(gsm.cpu().numpy().astype(np.float64) - gs_ref).max()
    f_ref, _ = oracle.fuse_stack(stack, 0.02, sigma_xy=sigma_xy, sigma_z=sigma_z, tol=1e-12)
    ferr = np.abs(f.cpu().numpy() - f_ref).max()
    print(sigma_xy, sigma_z, precision, "smoothing err", gerr, "f err", ferr, [r["vcycles"] for r in rep])
    assert gerr <= (2e-4 if precision == "fp32" else 1e-9)
    assert ferr <= ABS_TOL
    assert all(r["status"] == gdf.GDF_OK and r["rel_residual"] <= 1e-6 for r in rep)


@pytest.mark.parametrize("S,H,W,Wp,extra_rows,precision", [(5, 70, 93, 101, 3, "fp32"), (6, 64, 128, 160, 5, "fp32"),
                                                            (4, 50, 77, 80, 2, "mixed")])
def test_fuse_stack_pitched_stack(S, H, W, Wp, extra_rows, precision):
    # a stack viewed inside a larger buffer: row pitch Wp > W and slice pitch
    # (H + extra_rows) Wp > H Wp, through fuse_stack's pitches.  An odd width
    # takes the smoothing's byte loads; W = 128 with a 160-byte pitch the
    # dword loads with a pitch; the output pass and the FP64 re-solve of the
    # mixed scheme read g_o at the pitched offsets.  The bytes between rows
    # and slices hold 255 and must not leak into the result.
    stack = synth.make_stack(S, H, W, seed=300 + W, ramp=True)
    big = torch.full((S, H + extra_rows, Wp), 255, dtype=torch.uint8, device=DEV)
    view = big[:, :H, :W]
    view.copy_(torch.from_numpy(stack).to(DEV))
    assert view.stride() == ((H + extra_rows) * Wp, Wp, 1)
    print("pitched", (S, H, W), "pitches", view.stride()[:2], precision, flush=True)
    f, rep, gsm = gdf.fuse_stack(view, 0.01, tol=1e-6, precision=precision, return_smooth=True,
                                 out_dtype=gdf.DTYPE_F64)
    f2, rep2 = gdf.fuse_stack(view, 0.01, tol=1e-6, precision=precision)   # no g_s output
    torch.cuda.synchronize()
    f_ref, gs_ref = oracle.fuse_stack(stack, 0.01, tol=1e-12)
    gerr = np.abs(gsm.cpu().numpy().astype(np.float64) - gs_ref).max()
    err = np.abs(f.cpu().numpy() - f_ref).max()
    err2 = np.abs(f2.cpu().numpy().astype(np.float64) - f_ref).max()
    print("smoothing err %.2e f err %.2e (without g_s %.2e)" % (gerr, err, err2), flush=True)
    assert gerr <= 2e-4
    assert err <= ABS_TOL and err2 <= ABS_TOL
    cpu_rel = _relres_stack(f.cpu().numpy(), gsm.cpu().numpy().astype(np.float64), stack.astype(np.float64), 0.01)
    assert max(cpu_rel) <= 1e-6 * 1.01
    assert all(r["status"] == gdf.GDF_OK for r in rep + rep2)
