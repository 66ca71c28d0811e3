"""Benchmark: gradient-domain fusion of a synthetic EM stack on one MI355X.

Workload (the headline): 64 slices of 2048 x 2048 uint8 (EM-like texture,
per-slice gain/offset and a linear illumination ramp), anisotropic smoothing
(sigma_xy = 1, sigma_z = 3) then the screened-Poisson blend of Eq. (1) with
alpha = 0.01, Neumann boundaries, FP32 V-cycles, every slice to an FP64
relative residual of 1e-6.  One step = one fuse_stack call on the stack
already resident in HBM (smoothing, all V-cycles, output formation).

Prints one JSON line: throughput in Mvoxels/s, the roofline of the dominant
kernel (the fused finest-level V-cycle pass) from HIP events around its
launches, and the CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import re
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
FINE_BYTES_PER_PX = 14.0   # FP32 fused finest pass: u 4 + b 4 + coarse 1 in, u 4 + coarse rhs 1 out


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


def cpu_baseline(stack, z):
    """The oracle as it stands on one slice of the workload: smoothing of every
    voxel of slice z (tap-by-tap sums over the full stack) plus its CG solve to
    the same 1e-6 relative residual."""
    import oracle
    oracle.build(force=False)
    yy, xx = np.mgrid[0:H, 0:W]
    pts = np.stack([np.full(H * W, z), yy.ravel(), xx.ravel()], axis=1).astype(np.int32)
    t0 = time.perf_counter()
    gs = oracle.smooth_points(stack, pts).reshape(H, W)
    t1 = time.perf_counter()
    oracle.solve(gs, stack[z].astype(np.float64), ALPHA, tol=TOL)
    t2 = time.perf_counter()
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": H * W / (t2 - t0) / 1e6, "unit": "Mvoxels/s", "cores": cores, "kind": "oracle",
            "sample": "slice %d of the 64x2048x2048 stack: FP64 tap-by-tap smoothing (%.1f s) + "
                      "unpreconditioned CG to rel. residual 1e-6 (%.1f s)" % (z, t1 - t0, t2 - t1)}


# the fused finest pass (FP32 level 0, bfloat16 coarse level): prolongation, no zero
# start, residual norm + restriction, unit stencil; one launch per pass
FINE_KERNEL_RE = r"strip_kernel<float, float, unsigned short, true, false, \d+, 3, false>"
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
    rec = {"kernel": "vcycle_fine (strip_kernel SK_FINE, FP32 with bfloat16 coarse level; one launch per pass)",
           "workload": "fuse_stack 64 x 2048 x 2048, alpha 0.01, tol 1e-6",
           "mg_kernels_sha256": hashlib.sha256(open(MG_SRC, "rb").read()).hexdigest(),
           "hbm_read_bytes_per_launch": rd, "hbm_write_bytes_per_launch": wr,
           "hbm_bytes_per_launch": (rd + wr) if rd and wr else None,
           "counters": res, "command": command}
    with open(out_json, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))


def _timed(torch, fn, steps, warmup):
    for _ in range(warmup):
        out = fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps, out


def bench_batched(gdf, torch, dev, steps):
    """512 uneven slices (sides 512..4096 step 256, alpha ~ U(0.001, 0.1)) in one
    graph-captured solve_slices call, settings autotuned on the first call."""
    desc = synth.uneven_batch(512, seed=synth.CONFIG_SEED[2])
    log("batched: generating %d slices" % len(desc))
    go, gs, al = [], [], []
    for H, W, a, sd in desc:
        o, s = synth.batch_slice_t(H, W, sd, dev)
        go.append(o)
        gs.append(s)
        al.append(a)
    px = float(sum(H * W for H, W, _, _ in desc))
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
    return {"value": px / (ms * 1e-3) / 1e6, "unit": "Mvoxels/s", "ms_per_step": ms, "steps": steps,
            "workload": "solve_slices: 512 uneven slices (H, W uniform on 512..4096 step 256, %.3f Gpx), "
                        "alpha per slice U(0.001, 0.1), FP32, tol 1e-6, one captured graph per call" % (px / 1e9),
            "autotuned": tuned, "autotune_s": t_tune,
            "worst_rel_residual": max(r["rel_residual"] for r in rep), "vcycles_min_max": [min(vc), max(vc)]}


def bench_mixed(gdf, torch, dev, steps, alpha):
    """4 slices of 21504 x 26624: FP32 V-cycles inside FP64 refinement to 1e-8."""
    S3, H3, W3 = 4, 21504, 26624
    log("mixed: generating %dx%dx%d" % (S3, H3, W3))
    st = synth.make_stack_t(S3, H3, W3, synth.CONFIG_SEED[3], dev)
    run = lambda: gdf.fuse_stack(st, alpha, tol=1e-8, precision="mixed")
    log("mixed alpha=%g: timing" % alpha)
    ms, (f, rep) = _timed(torch, run, steps, 1)
    del f
    vc = [r["vcycles"] for r in rep]
    return {"value": S3 * H3 * W3 / (ms * 1e-3) / 1e6, "unit": "Mvoxels/s", "ms_per_step": ms, "steps": steps,
            "workload": "fuse_stack mixed: 4 x 21504 x 26624 uint8, sigma_xy=1, sigma_z=3, alpha=%g, FP32 "
                        "V-cycles (3 per refinement step) + FP64 residual/update to FP64 rel. residual 1e-8"
                        % alpha,
            "worst_rel_residual": max(r["rel_residual"] for r in rep), "inner_vcycles_min_max": [min(vc), max(vc)]}


def bench_robust(gdf, torch, dev, stack, kw, steps):
    """The headline stack with robust cross-slice averaging ("Extensions and Applications")."""
    st = torch.from_numpy(stack).to(dev)
    run = lambda: gdf.fuse_stack(st, ALPHA, robust=True, **kw)
    log("robust: timing")
    ms, (f, rep) = _timed(torch, run, steps, 1)
    del f
    gdf.profile_reset()
    gdf.profile_enable(True)
    gdf.fuse_stack(st, ALPHA, robust=True, **kw)
    torch.cuda.synchronize()
    gdf.profile_enable(False)
    n, sm, _ = gdf.profile_read("smooth")
    S_, H_, W_ = stack.shape
    vc = [r["vcycles"] for r in rep]
    return {"value": S_ * H_ * W_ / (ms * 1e-3) / 1e6, "unit": "Mvoxels/s", "ms_per_step": ms, "steps": steps,
            "workload": "fuse_stack on the headline stack with robust cross-slice averaging (values beyond two "
                        "weighted standard deviations of the window mean left out), FP32, tol 1e-6",
            "smooth_ms": sm / max(1, n), "worst_rel_residual": max(r["rel_residual"] for r in rep),
            "vcycles_min_max": [min(vc), max(vc)]}


def bench_stack_gradient(gdf, torch, dev, shape, steps):
    """The transpose of the smoothing (the gradient through it) on an FP32
    gradient of the headline stack's shape: a fused in-plane pass and a
    cross-slice pass, each reading and writing 4 bytes per voxel."""
    g = torch.randn(shape, device=dev, dtype=torch.float32)
    log("stack gradient: timing")
    ms, out = _timed(torch, lambda: gdf.smooth_transpose(g, 1.0, 3.0), steps, 1)
    n = g.numel()
    del out, g
    return {"value": n / (ms * 1e-3) / 1e6, "unit": "Mvoxels/s", "ms_per_step": ms, "steps": steps,
            "workload": "smooth_transpose (dLoss/dstack through the smoothing) on a %d x %d x %d FP32 gradient, "
                        "sigma_xy=1, sigma_z=3" % tuple(shape),
            "algo_GBps": 2 * 2 * 4 * n / (ms * 1e-3) / 1e9}


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
    dev_out = torch.empty_like(out, device="cuda")
    d2h_ms, _ = _timed(torch, lambda: out.copy_(dev_out, non_blocking=True), 3, 1)
    del dev_out
    S_, H_, W_ = stack.shape
    vc = [r["vcycles"] for r in rep]
    return {"value": S_ * H_ * W_ / (ms * 1e-3) / 1e6, "unit": "Mvoxels/s", "ms_per_step": ms, "steps": steps,
            "result_download_ms": d2h_ms, "d2h_GBps": out.numel() * 4 / (d2h_ms * 1e-3) / 1e9,
            "workload": "fuse_stack_streamed: the headline stack in pinned host memory, chunks of %d slices " % CHUNK +
                        "(+9 halo slices each side), FP32 result back to pinned host memory, tol 1e-6",
            "worst_rel_residual": max(r["rel_residual"] for r in rep), "vcycles_min_max": [min(vc), max(vc)]}


def bench_color(gdf, torch, dev, steps):
    """Colour fusion: 3 channels of 4096 x 4096 (low-frequency colour) with one
    grey image's gradients, FP32 to 1e-6, one batch."""
    C, H, W = 3, 4096, 4096
    grey, _ = synth.batch_slice_t(H, W, 7, dev)
    grey = grey.to(torch.float32)
    color = torch.stack([grey * 0.6 + 40.0, grey * 0.9, 200.0 - 0.5 * grey])
    color = torch.nn.functional.avg_pool2d(color[None], 9, stride=1, padding=4, count_include_pad=False)[0]
    log("color: timing")
    ms, (f, rep) = _timed(torch, lambda: gdf.fuse_color(color.contiguous(), grey, 0.01, tol=1e-6), steps, 1)
    del f
    vc = [r["vcycles"] for r in rep]
    return {"value": C * H * W / (ms * 1e-3) / 1e6, "unit": "Mpixels/s (all channels)", "ms_per_step": ms,
            "steps": steps, "workload": "fuse_color: 3 x 4096 x 4096 FP32 colour target with the gradients of "
                                        "one grey image, alpha 0.01, tol 1e-6",
            "worst_rel_residual": max(r["rel_residual"] for r in rep), "vcycles_min_max": [min(vc), max(vc)]}


def bench_adjoint(gdf, torch, dev, steps):
    """16 x 1024 x 1024 FP32: loss = sum (f - t)^2 through the autograd function."""
    S4, H4, W4 = 16, 1024, 1024
    stack = synth.make_stack_t(S4, H4, W4, synth.CONFIG_SEED[4], dev)
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
    return {"value": vox / (ms_fb * 1e-3) / 1e6, "unit": "Mvoxels/s (forward + backward)",
            "ms_per_step": ms_fb, "steps": steps, "forward_ms": ms_f, "backward_ms": ms_fb - ms_f,
            "backward_Mvoxels_s": vox / ((ms_fb - ms_f) * 1e-3) / 1e6,
            "workload": "ScreenedPoissonSolve on 16 x 1024 x 1024 FP32 (g_s = the method's smoothing), "
                        "alpha=0.01, loss sum (f - t)^2; backward = adjoint solve (FP32 V-cycles in FP64 "
                        "refinement) to 1e-6 + gradient assembly"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    # defaults: the settings the autotuner picks for this workload on MI355X
    # (--autotune runs the tuner instead, inside the untimed warm-up)
    ap.add_argument("--nu", type=int, default=2)
    ap.add_argument("--fine-sweeps", type=int, default=5)
    ap.add_argument("--coarse-sweeps", type=int, default=3)
    ap.add_argument("--tile-rows", type=int, default=128)
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the batched, mixed-precision and adjoint measurements")
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
                  tile_rows=args.tile_rows)

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
                      "tile_rows": args.tile_rows,
                      "launch_mode": args.launch}),
        "warmup_s": t_warm,
        "breakdown": breakdown,
    }
    del f, st
    if not args.no_forms:
        plain = out["value"]
        forms = {}
        forms["batched"] = bench_batched(gdf, torch, dev, 3)
        torch.cuda.empty_cache()
        forms["mixed"] = bench_mixed(gdf, torch, dev, 2, 0.001)
        forms["mixed_alpha_0.01"] = bench_mixed(gdf, torch, dev, 2, 0.01)
        torch.cuda.empty_cache()
        forms["adjoint"] = bench_adjoint(gdf, torch, dev, 5)
        forms["robust"] = bench_robust(gdf, torch, dev, stack, kw, 3)
        forms["stack_gradient"] = bench_stack_gradient(gdf, torch, dev, stack.shape, 5)
        forms["color"] = bench_color(gdf, torch, dev, 3)
        forms["host_streamed"] = bench_host_streamed(gdf, torch, stack, 3)
        for v in forms.values():
            v["vs_plain"] = v["value"] / plain
        out["forms"] = forms
    if not args.no_cpu:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(stack, S // 2)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
