"""solve_slices_noalloc (the entry point backed by the library's static
device scratch) through the C ABI, against solve_slices with a caller
workspace on the same inputs, on two calls in a row (the second batch
smaller), and against the oracle."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_1506_02079_amd as gdf
import synth

DEV = torch.device("cuda:0")


def _call_noalloc(tg, to, al, tol):
    f_list = [torch.full_like(t, float("nan")) for t in tg]
    d, bases = gdf._descs(tg, to, f_list, al)
    n = len(tg)
    rep = (gdf.SliceReport * n)()
    o = gdf.make_opts()
    st = gdf.lib().solve_slices_noalloc(n, d, gdf.DTYPE_F32, bases[0], gdf.DTYPE_U8, bases[1], 0, float(tol),
                                        bases[2], ctypes.byref(o), rep, gdf._stream(DEV))
    return st, f_list, gdf._report_list(rep, n)


@pytest.mark.gpu
def test_noalloc_matches_workspace_entry_point():
    # first call: three uneven slices (odd sizes, one a single column); second
    # call: one smaller slice, so the scratch holds the first call's values
    for sizes, seed in (([(300, 257), (128, 512), (77, 1)], 5), ([(64, 96)], 6)):
        rng = np.random.default_rng(seed)
        pairs = [synth.batch_slice(H, W, seed * 100 + i) for i, (H, W) in enumerate(sizes)]
        al = [float(rng.uniform(0.003, 0.05)) for _ in sizes]
        tg = [torch.from_numpy(s).to(DEV) for _, s in pairs]
        to = [torch.from_numpy(o).to(DEV) for o, _ in pairs]
        print("noalloc", sizes, al, flush=True)
        st, f_new, rep_new = _call_noalloc(tg, to, al, 1e-6)
        assert st == gdf.GDF_OK, gdf.last_error()
        f_ref, rep_ref = gdf.solve_slices(tg, to, al, tol=1e-6)
        torch.cuda.synchronize()
        for i in range(len(sizes)):
            assert torch.equal(f_new[i], f_ref[i])
            assert rep_new[i] == rep_ref[i]
            o, s = pairs[i]
            fr = oracle.solve(s, o.astype(np.float64), al[i], tol=1e-12)
            err = np.abs(f_new[i].cpu().numpy() - fr).max()
            print(sizes[i], "max abs err vs oracle %.2e" % err, rep_new[i], flush=True)
            assert err <= 1e-3
            assert rep_new[i]["status"] == gdf.GDF_OK and rep_new[i]["rel_residual"] <= 1e-6
