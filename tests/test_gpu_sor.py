"""GPU parity of the over-relaxed fused finest passes (opts.sor): the same
problem, Eq. (1) per slice, solved with successive over-relaxation in the
level-0 red-black sweeps (a solver choice; the result is still the unique
solution, so the oracle is the same)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1506_02079_amd as gdf
import synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.mark.parametrize("shape,alpha,nu,fs", [((6, 128, 160), 0.01, 2, 4), ((5, 97, 203), 0.001, 2, 5),
                                               ((4, 300, 130), 0.1, 1, 4), ((3, 1, 700), 0.01, 2, 4),
                                               ((3, 257, 3), 0.05, 2, 5)])
def test_sor_fuse_stack_matches_oracle(shape, alpha, nu, fs):
    stack = synth.make_stack(*shape, seed=sum(shape) + 31, ramp=True)
    print("sor fuse_stack", shape, alpha, nu, fs, flush=True)
    # (FP64 output: the reported residual is that of the unrounded g_o + u)
    f, rep, gsm = gdf.fuse_stack(torch.from_numpy(stack).to(DEV), alpha, tol=1e-6, nu=nu, fine_sweeps=fs,
                                 sor=True, return_smooth=True, out_dtype=gdf.DTYPE_F64)
    gs = gsm.cpu().numpy().astype(np.float64)
    f = f.cpu().numpy()
    for z in range(shape[0]):
        fr = oracle.solve(gs[z], stack[z].astype(np.float64), alpha, tol=1e-12)
        err = np.abs(f[z] - fr).max()
        rel = oracle.relres(f[z].astype(np.float64), gs[z], stack[z].astype(np.float64), alpha)
        print("slice", z, "err %.2e rel %.2e" % (err, rel), rep[z], flush=True)
        assert err <= 1e-3 and rel <= 1.01e-6
        assert rep[z]["status"] == gdf.GDF_OK


@pytest.mark.parametrize("use_graph", [False, True])
def test_sor_uneven_batch_and_mixed(use_graph):
    rng = np.random.default_rng(77)
    sizes = [(256, 256), (77, 530), (1, 50), (513, 129), (64, 1200)]
    al = [float(rng.uniform(0.001, 0.1)) for _ in sizes]
    pairs = [synth.batch_slice(H, W, 900 + i) for i, (H, W) in enumerate(sizes)]
    tg = [torch.from_numpy(s.astype(np.float32)).to(DEV) for _, s in pairs]
    to = [torch.from_numpy(o.astype(np.float32)).to(DEV) for o, _ in pairs]
    print("sor batch, graph", use_graph, flush=True)
    f, rep = gdf.solve_slices(tg, to, al, tol=1e-6, sor=True, use_graph=use_graph, max_vcycles=30)
    fm, repm = gdf.solve_slices(tg, to, al, tol=1e-9, sor=True, precision="mixed", out_dtype=gdf.DTYPE_F64)
    for i, (o, s) in enumerate(pairs):
        s32 = s.astype(np.float32).astype(np.float64)
        o64 = o.astype(np.float64)
        fr = oracle.solve(s32, o64, al[i], tol=1e-13)
        e32 = np.abs(f[i].cpu().numpy() - fr).max()
        e64 = np.abs(fm[i].cpu().numpy() - fr).max()
        print(sizes[i], al[i], "err fp32 %.2e mixed %.2e" % (e32, e64), rep[i], repm[i], flush=True)
        assert rep[i]["status"] == gdf.GDF_OK and e32 <= 1e-3
        assert repm[i]["status"] == gdf.GDF_OK and repm[i]["rel_residual"] <= 1e-9 and e64 <= 1e-5


def test_sor_full_size_sampled():
    """The headline stack's shape with the over-relaxed passes: every slice to
    1e-6 (reported), two whole slices against the oracle."""
    S, H, W = 64, 2048, 2048
    stack = synth.make_stack(S, H, W, seed=synth.CONFIG_SEED[1], ramp=True)
    print("sor full size", flush=True)
    f, rep, gsm = gdf.fuse_stack(torch.from_numpy(stack).to(DEV), 0.01, tol=1e-6, nu=2, fine_sweeps=4, sor=True,
                                 return_smooth=True)
    assert all(r["status"] == gdf.GDF_OK and r["rel_residual"] <= 1e-6 for r in rep)
    for z in (0, 37):
        gs = gsm[z].cpu().numpy().astype(np.float64)
        fr = oracle.solve(gs, stack[z].astype(np.float64), 0.01, tol=1e-10)
        err = np.abs(f[z].cpu().numpy() - fr).max()
        print("slice", z, "err %.2e" % err, rep[z], flush=True)
        assert err <= 1e-3
