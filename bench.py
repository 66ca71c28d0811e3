"""Benchmark: gradient-domain fusion of a synthetic EM stack on one MI355X.

Workload (the headline): 64 slices of 2048 x 2048 uint8 (EM-like texture,
per-slice gain/offset and a linear illumination ramp), anisotropic smoothing
(sigma_xy = 1, sigma_z = 3) then the screened-Poisson blend of Eq. (1) with
alpha = 0.01, Neumann boundaries, FP32 V-cycles, every slice to an FP64
relative residual of 1e-6.  One step = one fuse_stack call on the stack
already resident in HBM (smoothing, all V-cycles, output formation).

Prints one JSON line: throughput in Mvoxels/s, the roofline of the dominant
kernel (the fused finest-level V-cycle pass) from HIP events around its
launches, the other forms (batched, mixed precision, adjoint, FP64 small
stack, ...), and the oracle leg: the CPU oracle timed on a bounded sample of
the headline workload (cpu_baseline), and the maximum absolute error of every
form's result against the FP64 oracle on sampled slices, crops or voxels.
The oracle leg runs after every GPU measurement, so the two never overlap.
"""
import argparse
import hashlib
import json
import os
import re
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402  (seeded input generator)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
S, H, W = 64, 2048, 2048
ALPHA, TOL = 0.01, 1e-6
SEED = 1001
CHECK_SLICES = (0, 31, 32)   # headline slices the oracle solves: an edge slice and the two at a chunk edge
ORACLE_TOL = 1e-10           # oracle solves for the error checks (the GPU results are at 1e-6 or 1e-8)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def traffic_from_profile():
    """HBM bytes per launch of the fused finest pass from the committed
    rocprofv3 counter summary, or None if the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", "vcycle_fine_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if hashlib.sha256(open(MG_SRC, "rb").read()).hexdigest() != rec.get("mg_kernels_sha256"):
        return None
    return rec.get("hbm_bytes_per_launch")


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# the fused finest pass (FP32 level 0, bfloat16 coarse level): prolongation, no zero
# start, residual norm + restriction, unit stencil, plain or over-relaxed; one
# launch per pass
FINE_KERNEL_RE = r"strip_kernel<float, float, unsigned short, true, false, \d+, 3, false(, (true|false))?>"
MG_SRC = os.path.join(ROOT, "paper_1506_02079_amd", "csrc", "mg_kernels.hip")


def _counter_rows(d):
    import csv
    path = os.path.join(d, "run_counter_collection.csv")
    return list(csv.DictReader(open(path)))


def summarize_pmc(fetch_dir, write_dir, out_json, command):
    """HBM bytes per launch of the fused finest pass from two rocprofv3 --pmc
    runs of `bench.py --calib-copy` (FETCH_SIZE, then WRITE_SIZE; KiB per
    dispatch).  Each counter is scaled by what it reads for the plain 1 GiB
    device copies the run performs (3 copies of 2^30 bytes)."""
    res = {}
    for name, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = [r for r in _counter_rows(d) if r["Counter_Name"] == name]
        copy = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
        ratio = sum(copy) / (3.0 * (1 << 30) / 1024.0)   # counter KiB per KiB copied
        fine = [r for r in rows if re.search(FINE_KERNEL_RE, r["Kernel_Name"])]
        vals = [float(r["Counter_Value"]) for r in fine]
        passes = len(vals)
        kib = sum(vals) / max(1, passes)
        res[name] = {"kib_per_pass": kib, "passes": passes, "copy_counter_ratio": ratio,
                     "bytes_per_pass": kib * 1024.0 / ratio if ratio > 0 else None}
    rd, wr = res["FETCH_SIZE"]["bytes_per_pass"], res["WRITE_SIZE"]["bytes_per_pass"]
    rec = {"kernel": "vcycle_fine (strip_kernel SK_FINE, FP32 with bfloat16 coarse level, over-relaxed "
                     "sweeps as the bench runs it; one launch per pass)",
           "workload": "fuse_stack 64 x 2048 x 2048, alpha 0.01, tol 1e-6",
           "mg_kernels_sha256": hashlib.sha256(open(MG_SRC, "rb").read()).hexdigest(),
           "hbm_read_bytes_per_launch": rd, "hbm_write_bytes_per_launch": wr,
           "hbm_bytes_per_launch": (rd + wr) if rd and wr else None,
           "counters": res, "command": command}
    with open(out_json, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))


def _timed(torch, fn, steps, warmup):
    # (the previous call's outputs are dropped before the next call, so that
    # large forms do not hold two sets of outputs and workspaces at once)
    out = None
    for _ in range(warmup):
        out = None
        out = fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = None
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps, out


def _maxerr(a, b):
    return float(np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)).max())


# Each form returns (result, check): `check` is None or a function run in the
# oracle leg, after every GPU measurement, returning the keys it adds to the
# result (max_abs_err_vs_oracle and what it was measured on).  A check only
# holds host copies of the GPU's inputs and outputs.

def bench_plain_fp64_small(gdf, torch, dev, steps):
    """The plain method in FP64 on 8 x 256 x 256 (alpha 0.01, tol 1e-6), the
    oracle timed on the same stack."""
    S0, H0, W0 = 8, 256, 256
    stack = synth.make_stack(S0, H0, W0, seed=synth.CONFIG_SEED[0])
    st = torch.from_numpy(stack).to(dev)
    log("fp64 small stack: timing")
    ms, (f, rep) = _timed(torch, lambda: gdf.fuse_stack(st, ALPHA, tol=TOL, precision="fp64"), steps, 2)
    f = f.cpu().numpy()
    vox = S0 * H0 * W0
    res = {"value": vox / (ms * 1e-3) / 1e6, "unit": "Mvoxels/s", "ms_per_step": ms, "steps": steps,
           "workload": "fuse_stack FP64: 8 x 256 x 256 uint8 (no ramp), sigma_xy=1, sigma_z=3, alpha=0.01, "
                       "Neumann, FP64 V-cycles to rel. residual 1e-6",
           "worst_rel_residual": max(r["rel_residual"] for r in rep),
           "vcycles_min_max": [min(r["vcycles"] for r in rep), max(r["vcycles"] for r in rep)]}

    def check():
        import oracle
        t0 = time.perf_counter()
        oracle.fuse_stack(stack, ALPHA, tol=TOL)   # the oracle on the same work: smoothing + CG to 1e-6
        t_or = time.perf_counter() - t0
        f_ref, _ = oracle.fuse_stack(stack, ALPHA, tol=1e-12)
        return {"max_abs_err_vs_oracle": _maxerr(f, f_ref), "err_measured_on": "all 8 slices",
                "oracle_Mvoxels_s": vox / t_or / 1e6, "oracle_threads": oracle.threads()}
    return res, check


def bench_batched(gdf, torch, dev, steps):
    """512 uneven slices (sides 512..4096 step 256, alpha ~ U(0.001, 0.1)) in one
    graph-captured solve_slices call, settings autotuned on the first call."""
    desc = synth.uneven_batch(512, seed=synth.CONFIG_SEED[2])
    log("batched: generating %d slices" % len(desc))
    go, gs, al = [], [], []
    for H_, W_, a, sd in desc:
        o, s = synth.batch_slice_t(H_, W_, sd, dev)
        go.append(o)
        gs.append(s)
        al.append(a)
    px = float(sum(H_ * W_ for H_, W_, _, _ in desc))
    kw = dict(tol=TOL, use_graph=True, autotune=True)
    log("batched: autotuning")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gdf.solve_slices(gs, go, al, **kw)
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t0
    tuned = gdf.autotune_last()
    log("batched: tuned %s in %.1f s; timing" % (tuned, t_tune))
    ms, (f, rep) = _timed(torch, lambda: gdf.solve_slices(gs, go, al, **kw), steps, 1)
    vc = [r["vcycles"] for r in rep]
    res = {"value": px / (ms * 1e-3) / 1e6, "unit": "Mvoxels/s", "ms_per_step": ms, "steps": steps,
           "workload": "solve_slices: 512 uneven slices (H, W uniform on 512..4096 step 256, %.3f Gpx), "
                       "alpha per slice U(0.001, 0.1), FP32, tol 1e-6, one captured graph per call" % (px / 1e9),
           "autotuned": tuned, "autotune_s": t_tune,
           "worst_rel_residual": max(r["rel_residual"] for r in rep), "vcycles_min_max": [min(vc), max(vc)]}
    # the oracle subset: the two smallest and two largest slices, the two lowest
    # and two highest alphas (the test suite checks 16 and every residual)
    n = len(desc)
    pick = []
    for k in (sorted(range(n), key=lambda i: desc[i][0] * desc[i][1])[:2] +
              sorted(range(n), key=lambda i: -desc[i][0] * desc[i][1])[:2] +
              sorted(range(n), key=lambda i: desc[i][2])[:2] + sorted(range(n), key=lambda i: -desc[i][2])[:2]):
        if k not in pick:
            pick.append(k)
    held = [(i, gs[i].cpu().numpy(), go[i].cpu().numpy(), f[i].cpu().numpy()) for i in pick]

    def check():
        import oracle
        errs = []
        for i, s, o, fi in held:
            fr = oracle.solve(s, o.astype(np.float64), desc[i][2], tol=ORACLE_TOL)
            errs.append(_maxerr(fi, fr))
        return {"max_abs_err_vs_oracle": max(errs),
                "err_measured_on": "%d whole slices: the 2 smallest, 2 largest (4096 x 4096 among them), 2 lowest "
                                   "and 2 highest alphas; (H, W, alpha, err) = %s" %
                                   (len(held), [(desc[i][0], desc[i][1], round(desc[i][2], 5), float("%.3g" % e))
                                                for (i, _, _, _), e in zip(held, errs)])}
    return res, check


MIXED_SHAPE = (4, 21504, 26624)
MIXED_CROP = {0.001: ((0, 0), 1), 0.01: ((21504 - 1024, 26624 - 1024), 2)}   # 1024^2 crop corner, slice


def bench_mixed(gdf, torch, dev, steps, alpha):
    """4 slices of 21504 x 26624: FP32 V-cycles inside FP64 refinement to 1e-8."""
    S3, H3, W3 = MIXED_SHAPE
    log("mixed: generating %dx%dx%d" % (S3, H3, W3))
    st = synth.make_stack_t(S3, H3, W3, synth.CONFIG_SEED[3], dev)
    run = lambda: gdf.fuse_stack(st, alpha, tol=1e-8, precision="mixed")
    log("mixed alpha=%g: timing" % alpha)
    ms, (f, rep) = _timed(torch, run, steps, 1)
    vc = [r["vcycles"] for r in rep]
    res = {"value": S3 * H3 * W3 / (ms * 1e-3) / 1e6, "unit": "Mvoxels/s", "ms_per_step": ms, "steps": steps,
           "workload": "fuse_stack mixed: 4 x 21504 x 26624 uint8, sigma_xy=1, sigma_z=3, alpha=%g, FP32 "
                       "V-cycles (3 per refinement step) + FP64 residual/update to FP64 rel. residual 1e-8"
                       % alpha,
           "worst_rel_residual": max(r["rel_residual"] for r in rep), "inner_vcycles_min_max": [min(vc), max(vc)]}
    (y0, x0), z = MIXED_CROP[alpha]
    fc = f[z, y0:y0 + 1024, x0:x0 + 1024].cpu().numpy()
    del f, st

    def check():
        # (the crop oracle regenerates the crop's raw data from the generator's
        # numpy definition)
        from oracle.crop import fuse_crop
        ref, _, _ = fuse_crop(synth.CONFIG_SEED[3], S3, H3, W3, alpha, y0, y0 + 1024, x0, x0 + 1024, [z],
                              tol=1e-11)
        return {"max_abs_err_vs_oracle": _maxerr(fc, ref[0]),
                "err_measured_on": "1024 x 1024 crop at (%d, %d) of slice %d (crop oracle, halo %d px)" %
                                   (y0, x0, z, int(np.ceil(40 / np.sqrt(alpha))))}
    return res, check


def bench_robust(gdf, torch, dev, stack, kw, steps):
    """The headline stack with robust cross-slice averaging ("Extensions and Applications")."""
    st = torch.from_numpy(stack).to(dev)
    run = lambda: gdf.fuse_stack(st, ALPHA, robust=True, **kw)
    log("robust: timing")
    ms, (f, rep) = _timed(torch, run, steps, 1)
    fz = f[32].cpu().numpy()
    del f
    _, _, gsm = gdf.fuse_stack(st, ALPHA, robust=True, return_smooth=True, **kw)   # the GPU's robust g_s
    gsz = gsm[32].cpu().numpy().astype(np.float64)
    del gsm
    gdf.profile_reset()
    gdf.profile_enable(True)
    gdf.fuse_stack(st, ALPHA, robust=True, **kw)
    torch.cuda.synchronize()
    gdf.profile_enable(False)
    n, sm, _ = gdf.profile_read("smooth")
    S_, H_, W_ = stack.shape
    vc = [r["vcycles"] for r in rep]
    res = {"value": S_ * H_ * W_ / (ms * 1e-3) / 1e6, "unit": "Mvoxels/s", "ms_per_step": ms, "steps": steps,
           "workload": "fuse_stack on the headline stack with robust cross-slice averaging (values beyond two "
                       "weighted standard deviations of the window mean left out), FP32, tol 1e-6",
           "smooth_ms": sm / max(1, n), "worst_rel_residual": max(r["rel_residual"] for r in rep),
           "vcycles_min_max": [min(vc), max(vc)]}

    def check():
        # end to end against the oracle's robust smoothing and solve; then the
        # solve alone (the oracle on the GPU's own g_s), and the voxels whose
        # robust average differs: each must be a threshold tie, a value whose
        # squared distance from the window mean is within the FP32 rounding
        # bound 20 e M + 20 e^2 (e = 1e-3) of four times the variance
        import oracle
        yy, xx = np.mgrid[0:H_, 0:W_]
        pts = np.stack([np.full(H_ * W_, 32), yy.ravel(), xx.ravel()], axis=1)
        gsr = oracle.smooth_robust_points(stack, pts).reshape(H_, W_)
        go = stack[32].astype(np.float64)
        fr = oracle.solve(gsr, go, ALPHA, tol=ORACLE_TOL)
        fg = oracle.solve(gsz, go, ALPHA, tol=ORACLE_TOL)
        off = np.argwhere(np.abs(gsz - gsr) > 2e-4)
        non_ties = 0
        zs = np.arange(32 - 9, 32 + 10)
        w = np.exp(-(zs - 32) ** 2 / 18.0)
        for y, x in off:
            p = oracle.smooth_points(stack, np.stack([zs, np.full(19, y), np.full(19, x)], axis=1), 1.0, 0.0)
            mu = np.sum(w * p) / np.sum(w)
            var = np.sum(w * (p - mu) ** 2) / np.sum(w)
            M = np.max(np.abs(p - mu))
            if np.min(np.abs((p - mu) ** 2 - 4 * var)) > 20e-3 * M + 20e-6:
                non_ties += 1
        return {"max_abs_err_vs_oracle": _maxerr(fz, fr), "solve_err_on_gpu_g_s": _maxerr(fz, fg),
                "g_s_voxels_off": int(len(off)), "g_s_voxels_off_not_threshold_ties": non_ties,
                "err_measured_on": "slice 32: end to end against the oracle's robust smoothing and solve; "
                                   "solve_err_on_gpu_g_s is the oracle's solve of the GPU's own g_s"}
    return res, check


def bench_stack_gradient(gdf, torch, dev, shape, steps):
    """The transpose of the smoothing (the gradient through it) on an FP32
    gradient of the headline stack's shape: a fused in-plane pass and a
    cross-slice pass, each reading and writing 4 bytes per voxel."""
    g = torch.randn(shape, device=dev, dtype=torch.float32)
    log("stack gradient: timing")
    ms, out = _timed(torch, lambda: gdf.smooth_transpose(g, 1.0, 3.0), steps, 1)
    n = g.numel()
    del out, g
    # the error check runs the same call on a smaller gradient (the oracle's
    # transpose is a plain sum over every voxel's window)
    gs_small = np.random.default_rng(5).standard_normal((19, 256, 256))
    out_small = gdf.smooth_transpose(torch.from_numpy(gs_small).to(dev, torch.float32), 1.0, 3.0).cpu().numpy()
    res = {"value": n / (ms * 1e-3) / 1e6, "unit": "Mvoxels/s", "ms_per_step": ms, "steps": steps,
           "workload": "smooth_transpose (dLoss/dstack through the smoothing) on a %d x %d x %d FP32 gradient, "
                       "sigma_xy=1, sigma_z=3" % tuple(shape),
           "algo_GBps": 2 * 2 * 4 * n / (ms * 1e-3) / 1e9}

    def check():
        import oracle
        ref = oracle.smooth_transpose(gs_small, 1.0, 3.0)
        return {"max_abs_err_vs_oracle": _maxerr(out_small, ref), "err_scale": float(np.abs(ref).max()),
                "err_measured_on": "a 19 x 256 x 256 standard-normal gradient through the same entry point"}
    return res, check


def bench_host_streamed(gdf, torch, stack, steps):
    """The headline stack held in pinned host memory and solved 32 slices at a
    time with their smoothing halos; the rate includes the PCIe uploads and the
    FP32 result's download."""
    CHUNK = 32
    host = torch.from_numpy(np.ascontiguousarray(stack)).pin_memory()
    out = torch.empty(tuple(stack.shape), dtype=torch.float32, pin_memory=True)
    log("host streamed: timing")
    ms, (_, rep) = _timed(torch, lambda: gdf.fuse_stack_streamed(host, ALPHA, chunk=CHUNK, out=out, tol=TOL),
                          steps, 1)
    held = {z: out[z].numpy().copy() for z in (31, 32)}   # the two slices either side of the chunk edge
    dev_out = torch.empty_like(out, device="cuda")   # (the download timing below overwrites out)
    d2h_ms, _ = _timed(torch, lambda: out.copy_(dev_out, non_blocking=True), 3, 1)
    del dev_out
    S_, H_, W_ = stack.shape
    vc = [r["vcycles"] for r in rep]
    res = {"value": S_ * H_ * W_ / (ms * 1e-3) / 1e6, "unit": "Mvoxels/s", "ms_per_step": ms, "steps": steps,
           "result_download_ms": d2h_ms, "d2h_GBps": out.numel() * 4 / (d2h_ms * 1e-3) / 1e9,
           "workload": "fuse_stack_streamed: the headline stack in pinned host memory, chunks of %d slices " % CHUNK +
                       "(+9 halo slices each side), FP32 result back to pinned host memory, tol 1e-6",
           "worst_rel_residual": max(r["rel_residual"] for r in rep), "vcycles_min_max": [min(vc), max(vc)]}
    return res, held


def bench_color(gdf, torch, dev, steps):
    """Colour fusion: 3 channels of 4096 x 4096 (low-frequency colour) with one
    grey image's gradients, FP32 to 1e-6, one batch."""
    C, H_, W_ = 3, 4096, 4096
    grey, _ = synth.batch_slice_t(H_, W_, 7, dev)
    grey = grey.to(torch.float32)
    color = torch.stack([grey * 0.6 + 40.0, grey * 0.9, 200.0 - 0.5 * grey])
    color = torch.nn.functional.avg_pool2d(color[None], 9, stride=1, padding=4, count_include_pad=False)[0]
    color = color.contiguous()
    log("color: timing")
    ms, (f, rep) = _timed(torch, lambda: gdf.fuse_color(color, grey, 0.01, tol=1e-6), steps, 1)
    vc = [r["vcycles"] for r in rep]
    res = {"value": C * H_ * W_ / (ms * 1e-3) / 1e6, "unit": "Mpixels/s (all channels)", "ms_per_step": ms,
           "steps": steps, "workload": "fuse_color: 3 x 4096 x 4096 FP32 colour target with the gradients of "
                                       "one grey image, alpha 0.01, tol 1e-6",
           "worst_rel_residual": max(r["rel_residual"] for r in rep), "vcycles_min_max": [min(vc), max(vc)]}
    c0, g0, f0 = color[0].cpu().numpy(), grey.cpu().numpy(), f[0].cpu().numpy()
    del f

    def check():
        import oracle
        fr = oracle.solve(c0, g0.astype(np.float64), 0.01, tol=ORACLE_TOL)
        return {"max_abs_err_vs_oracle": _maxerr(f0, fr), "err_measured_on": "channel 0 (whole 4096 x 4096 image)"}
    return res, check


def bench_adjoint(gdf, torch, dev, steps):
    """16 x 1024 x 1024 FP32: loss = sum (f - t)^2 through the autograd function."""
    S4, H4, W4 = 16, 1024, 1024
    stack_np = synth.make_stack(S4, H4, W4, synth.CONFIG_SEED[4])
    stack = torch.from_numpy(stack_np).to(dev)
    _, _, gsm = gdf.fuse_stack(stack, ALPHA, return_smooth=True)
    gen = torch.Generator(device=dev)
    gen.manual_seed(synth.CONFIG_SEED[4])
    tgt = torch.rand((S4, H4, W4), generator=gen, device=dev) * 255.0
    gs = gsm.clone().requires_grad_()
    go = stack.float().requires_grad_()
    alpha = torch.tensor(ALPHA, device=dev, requires_grad=True)

    def fwd():
        return gdf.ScreenedPoissonSolve.apply(gs, go, alpha)

    def fwd_bwd():
        gs.grad = go.grad = alpha.grad = None
        loss = ((fwd() - tgt) ** 2).sum()
        loss.backward()
        return loss

    log("adjoint: timing")
    ms_f, _ = _timed(torch, fwd, steps, 1)
    ms_fb, _ = _timed(torch, fwd_bwd, steps, 1)
    vox = S4 * H4 * W4
    res = {"value": vox / (ms_fb * 1e-3) / 1e6, "unit": "Mvoxels/s (forward + backward)",
           "ms_per_step": ms_fb, "steps": steps, "forward_ms": ms_f, "backward_ms": ms_fb - ms_f,
           "backward_Mvoxels_s": vox / ((ms_fb - ms_f) * 1e-3) / 1e6,
           "workload": "ScreenedPoissonSolve on 16 x 1024 x 1024 FP32 (g_s = the method's smoothing), "
                       "alpha=0.01, loss sum (f - t)^2; backward = adjoint solve (FP32 V-cycles in FP64 "
                       "refinement) to 1e-6 + gradient assembly"}
    zs = (0, 11)
    held = {z: (gs.grad[z].cpu().numpy(), go.grad[z].cpu().numpy()) for z in zs}
    t_np = tgt.cpu().numpy()
    ga = float(alpha.grad)

    def check():
        import oracle
        e_gs = e_go = 0.0
        for z in zs:
            pts = np.stack([np.full(H4 * W4, z)] + [a.ravel() for a in np.mgrid[0:H4, 0:W4]], axis=1)
            gsz = oracle.smooth_points(stack_np, pts).reshape(H4, W4)
            goz = stack_np[z].astype(np.float64)
            fz = oracle.solve(gsz, goz, ALPHA, tol=ORACLE_TOL)
            r_gs, r_go, _ = oracle.adjoint(2.0 * (fz - t_np[z]), gsz, fz, ALPHA, tol=ORACLE_TOL)
            e_gs = max(e_gs, _maxerr(held[z][0], r_gs) / float(np.abs(r_gs).max()))
            e_go = max(e_go, _maxerr(held[z][1], r_go) / float(np.abs(r_go).max()))
        return {"max_abs_err_vs_oracle": {"dL_dg_s_rel_to_max": e_gs, "dL_dg_o_rel_to_max": e_go},
                "dL_dalpha_gpu": ga,
                "err_measured_on": "slices 0 and 11: the oracle's own smoothing, solve and adjoint; errors relative "
                                   "to the largest gradient entry"}
    return res, check


def cpu_baseline(stack, f_gpu):
    """The oracle as it stands on a bounded sample of the headline workload:
    for each of three slices, FP64 tap-by-tap smoothing of every voxel of the
    slice (over the full stack) plus its CG solve to the same 1e-6 relative
    residual; the median of the three rates.  The smoothed slices are kept for
    the headline's error check (CG to 1e-10 against the GPU's f)."""
    import oracle
    oracle.build(force=False)
    rates, parts, gsz = [], [], {}
    yy, xx = np.mgrid[0:H, 0:W]
    for z in CHECK_SLICES:
        pts = np.stack([np.full(H * W, z), yy.ravel(), xx.ravel()], axis=1).astype(np.int32)
        t0 = time.perf_counter()
        gs = oracle.smooth_points(stack, pts).reshape(H, W)
        t1 = time.perf_counter()
        oracle.solve(gs, stack[z].astype(np.float64), ALPHA, tol=TOL)
        t2 = time.perf_counter()
        rates.append(H * W / (t2 - t0) / 1e6)
        parts.append("slice %d: smoothing %.1f s + CG %.1f s" % (z, t1 - t0, t2 - t1))
        gsz[z] = gs
    base = {"value": statistics.median(rates), "unit": "Mvoxels/s", "cores": oracle.threads(), "kind": "oracle",
            "host_cpu": host_cpu_model(),
            "sample": "median of 3 slices (%s) of the 64 x 2048 x 2048 stack: FP64 tap-by-tap smoothing of every "
                      "voxel of the slice + unpreconditioned CG to rel. residual 1e-6; %s" %
                      (", ".join(str(z) for z in CHECK_SLICES), "; ".join(parts)),
            "rates": rates}
    errs, refs = {}, {}
    for z in CHECK_SLICES:
        refs[z] = oracle.solve(gsz[z], stack[z].astype(np.float64), ALPHA, tol=ORACLE_TOL)
        errs[z] = _maxerr(f_gpu[z], refs[z])
    return base, errs, refs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg (CPU baseline and error checks)")
    # defaults: the fastest settings measured for this workload on MI355X (a
    # sweep over nu, fine and coarse sweeps, band height and over-relaxation;
    # --autotune runs the library's tuner instead, inside the untimed warm-up)
    ap.add_argument("--nu", type=int, default=2)
    ap.add_argument("--fine-sweeps", type=int, default=4)
    ap.add_argument("--sor", type=int, default=1, choices=[0, 1],
                    help="over-relaxed sweeps in the fused finest passes (opts.sor)")
    ap.add_argument("--coarse-sweeps", type=int, default=0,
                    help="0: the library default (nu + 1, nu on strongly screened levels)")
    ap.add_argument("--tile-rows", type=int, default=0,
                    help="rows per level-0 work item; 0: the library default (80, fewer for small batches)")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the batched, mixed-precision, adjoint and other forms")
    ap.add_argument("--forms", default="", help="comma-separated subset of the forms to run (default: all)")
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--launch", default="grid", choices=["default", "grid", "persistent"])
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run plain 1 GiB device copies (HBM counter calibration)")
    ap.add_argument("--summarize-pmc", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "OUT_JSON"),
                    help="no run: write the traffic summary from two rocprofv3 --pmc output folders")
    ap.add_argument("--pmc-command", default="", help="command recorded in the traffic summary")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc, command=args.pmc_command)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (slices are "
              "independent; sharding along z is described in the design notes). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1506_02079_amd as gdf

    dev = torch.device("cuda:0")
    log("generating %dx%dx%d stack" % (S, H, W))
    stack = synth.make_stack(S, H, W, seed=SEED, ramp=True)
    st = torch.from_numpy(stack).to(dev)
    kw = dict(tol=TOL, precision="fp32", launch_mode=args.launch, autotune=args.autotune)
    if not args.autotune:
        kw.update(nu=args.nu, fine_sweeps=args.fine_sweeps, coarse_sweeps=args.coarse_sweeps,
                  tile_rows=args.tile_rows, sor=bool(args.sor))

    log("warmup" + (" (autotuning on the first call)" if args.autotune else ""))
    t0 = time.perf_counter()
    for _ in range(args.warmup):
        f, rep = gdf.fuse_stack(st, ALPHA, **kw)
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    tuned = gdf.autotune_last() if args.autotune else None

    if args.calib_copy:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters scale
        # the counters of the solver kernels to bytes
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # timed region: HIP events only around the dominant kernel (the fused
    # finest pass), on the library's stream
    gdf.profile_reset()
    gdf.profile_enable(True, fine_only=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        f, rep = gdf.fuse_stack(st, ALPHA, **kw)
        log("step %d done" % i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gdf.profile_enable(False)
    ms = (t1 - t0) * 1e3 / args.steps
    vox = S * H * W
    worst = max(r["rel_residual"] for r in rep)
    cycles = sorted(set(r["vcycles"] for r in rep))
    f_check = {z: f[z].cpu().numpy() for z in CHECK_SLICES}

    n_fine, ms_fine, bytes_fine = gdf.profile_read("vcycle_fine")
    per_launch_bytes = bytes_fine / max(1, n_fine)
    avg_ms = ms_fine / max(1, n_fine)
    achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9 if n_fine else None

    # per-class breakdown: a separate run with events around every kernel class
    # (the extra events slow the host's enqueueing, so it is not timed above)
    nb = max(2, args.steps // 2)
    gdf.profile_reset()
    gdf.profile_enable(True)
    for i in range(nb):
        gdf.fuse_stack(st, ALPHA, **kw)
    torch.cuda.synchronize()
    gdf.profile_enable(False)
    breakdown = {}
    for cls in ("smooth", "restrict_first", "vcycle_fine_first", "vcycle_fine", "coarse", "finalize"):
        n, m, b = gdf.profile_read(cls)
        breakdown[cls] = {"launches_per_step": n / nb, "ms_per_step": m / nb,
                          "algo_GBps": (b / (m * 1e-3) / 1e9) if m > 0 else None}

    out = {
        "metric": "Mvoxels/s to 1e-6 rel. residual",
        "value": vox / (ms * 1e-3) / 1e6,
        "unit": "Mvoxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "fuse_stack: 64 x 2048 x 2048 uint8 EM-like stack with per-slice gain, "
                               "offset and illumination ramp; sigma_xy=1, sigma_z=3; alpha=0.01; "
                               "Neumann; FP32 V-cycles to FP64 rel. residual 1e-6 per slice",
                   "slices": S, "height": H, "width": W, "alpha": ALPHA, "tol": TOL},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                     "traffic": traffic_from_profile(),
                     "kernel": "vcycle_fine (fused finest-level pass)",
                     "algo_bytes_per_launch": per_launch_bytes, "avg_launch_ms": avg_ms},
        "worst_rel_residual": worst,
        "vcycles": cycles,
        "settings": ({"autotuned": tuned} if args.autotune else
                     {"nu": args.nu, "fine_sweeps": args.fine_sweeps, "coarse_sweeps": args.coarse_sweeps,
                      "sor": bool(args.sor),
                      "tile_rows": args.tile_rows,
                      "launch_mode": args.launch}),
        "warmup_s": t_warm,
        "breakdown": breakdown,
    }
    del f, st
    checks = {}
    streamed_held = None
    if not args.no_forms:
        plain = out["value"]
        forms = {}
        for name, fn in (("batched", lambda: bench_batched(gdf, torch, dev, 3)),
                         ("mixed", lambda: bench_mixed(gdf, torch, dev, 2, 0.001)),
                         ("mixed_alpha_0.01", lambda: bench_mixed(gdf, torch, dev, 2, 0.01)),
                         ("adjoint", lambda: bench_adjoint(gdf, torch, dev, 5)),
                         ("plain_fp64_small", lambda: bench_plain_fp64_small(gdf, torch, dev, 10)),
                         ("robust", lambda: bench_robust(gdf, torch, dev, stack, kw, 3)),
                         ("stack_gradient", lambda: bench_stack_gradient(gdf, torch, dev, stack.shape, 5)),
                         ("color", lambda: bench_color(gdf, torch, dev, 3))):
            if args.forms and name not in args.forms.split(","):
                continue
            forms[name], checks[name] = fn()
            torch.cuda.empty_cache()
        if not args.forms or "host_streamed" in args.forms.split(","):
            forms["host_streamed"], streamed_held = bench_host_streamed(gdf, torch, stack, 3)
        for v in forms.values():
            v["vs_plain"] = v["value"] / plain
        out["forms"] = forms
    if not args.no_cpu:
        # the oracle leg: CPU baseline, then every result against the oracle
        log("oracle leg: cpu baseline")
        base, errs, refs = cpu_baseline(stack, f_check)
        out["cpu_baseline"] = base
        out["max_abs_err_vs_oracle"] = max(errs.values())
        out["err_measured_on"] = "whole slices %s (oracle smoothing of every voxel + CG to 1e-10)" % (
            ", ".join(str(z) for z in CHECK_SLICES))
        if streamed_held is not None:
            out["forms"]["host_streamed"]["max_abs_err_vs_oracle"] = max(
                _maxerr(streamed_held[z], refs[z]) for z in (31, 32))
            out["forms"]["host_streamed"]["err_measured_on"] = "slices 31 and 32 (either side of the chunk edge)"
        for name, chk in checks.items():
            if chk is not None:
                log("oracle leg: %s" % name)
                t0 = time.perf_counter()
                out["forms"][name].update(chk())
                out["forms"][name]["oracle_check_s"] = time.perf_counter() - t0
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
