/*
 * gdf.h — C ABI of the gradient-domain fusion library for MI355X (gfx950).
 *
 * The method (Kazhdan et al., "Gradient-Domain Fusion for Color Correction in
 * Large EM Image Stacks", arXiv 1506.02079) corrects an EM image stack I0 in
 * two steps:
 *   1. anisotropic Gaussian smoothing across slices, I1 = I0 * G(sigma_xy,
 *      sigma_z), with the kernel truncated at three standard deviations
 *      (Section III-A; Implementation subsection);
 *   2. per slice j, the screened-Poisson blend of Eq. (1):
 *          (alpha - Laplacian) I2_j = alpha I1_j - Laplacian I0_j,
 *      the minimiser of the energy of Section III-B.
 *
 * Discretisation used by every entry point: unit pixel spacing; the Laplacian
 * is the 5-point graph Laplacian of the 4-connected pixel grid, so for
 * Neumann boundaries (the energy's natural boundary condition) a pixel only
 * couples to neighbours inside the slice.  The system solved per slice is
 *          (alpha I + L) f = alpha g_s + L g_o,
 * with g_s the smoothed slice (I1_j), g_o the original slice (I0_j), f = I2_j.
 * The relative residual is ||b - A f||_2 / ||b||_2 with b = alpha g_s + L g_o
 * (the definition the paper gives for its solver statistics), evaluated in
 * FP64, per slice.
 *
 * Conventions shared by all entry points
 *  - Pointers named *_dev are device (HBM) pointers owned by the caller; the
 *    library never frees or retains them past the call.  Host pointers are
 *    named *_host.
 *  - Images are row-major, x (width) fastest.  Element strides are given in
 *    elements of the buffer's own type.
 *  - `stream` is a hipStream_t passed as void*; NULL means the default
 *    stream.  All device work is enqueued on it.  Every entry point returns
 *    after the solve has finished on the device (convergence is decided on
 *    the host between V-cycles, or at the end of a captured graph), so
 *    outputs are ready when it returns.
 *  - `workspace_dev` is caller-allocated device memory of at least the size
 *    returned by the matching *_workspace_size call for the same arguments,
 *    aligned to 256 bytes.  The library allocates no device memory of its own
 *    apart from a small per-device cache of captured graphs (gdf_release) and
 *    the static scratch of solve_slices_noalloc.
 *  - Argument checks run on the host before any device work and return
 *    GDF_EINVAL (with gdf_last_error() describing the argument).  No C++
 *    exception crosses this interface.
 *  - GDF_ENOCONV / GDF_ENONFINITE: outputs are still written; per-slice
 *    status is in the report.
 */
#ifndef GDF_H
#define GDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GDF_OK = 0,
    GDF_EINVAL = 1,        /* invalid argument (message in gdf_last_error) */
    GDF_EUNSUPPORTED = 2,  /* valid but unsupported combination (e.g. Dirichlet) */
    GDF_ENOMEM = 3,        /* workspace smaller than required */
    GDF_EDEVICE = 4,       /* HIP runtime error (message in gdf_last_error) */
    GDF_ENOCONV = 5,       /* some slice did not reach tol within max_vcycles */
    GDF_ENONFINITE = 6     /* some slice produced a NaN/Inf residual */
} gdf_status;

typedef enum {
    GDF_BC_NEUMANN = 0,    /* reflecting edges: the energy's natural boundary condition */
    GDF_BC_PERIODIC = 1,   /* wrap-around (the paper's Fourier basis, Section III-B): the first
                              and last row and column of a slice are neighbours; a side of two
                              pixels couples them across both faces, a side of one has no
                              coupling.  Solved by a multigrid of its own (plain per-level
                              kernels); workspace sizes are the same for either boundary. */
    GDF_BC_DIRICHLET = 2   /* boundary values are not specified by the method: GDF_EUNSUPPORTED */
} gdf_bc;

typedef enum { GDF_U8 = 0, GDF_F32 = 1, GDF_F64 = 2 } gdf_dtype;

typedef enum {
    GDF_PREC_FP32 = 0,     /* FP32 V-cycles on u = f - g_o; FP64 residual norms */
    GDF_PREC_FP64 = 1,     /* FP64 throughout */
    GDF_PREC_MIXED = 2     /* FP32 V-cycles inside FP64 iterative refinement */
} gdf_precision;

/* Solver options.  Zero-initialise and set what you need; 0 selects the
 * default noted for each field. */
typedef struct {
    int precision;     /* gdf_precision (default GDF_PREC_FP32) */
    int max_vcycles;   /* cap on V-cycles per slice (default 40; for MIXED: total inner cycles) */
    int nu;            /* red-black Gauss-Seidel sweeps before and after each coarse
                          correction on the finest level: 1 or 2 (default 2) */
    int out_dtype;     /* GDF_F32 or GDF_F64 for f; 0 = F32 for FP32, F64 otherwise */
    int use_graph;     /* 1: record the whole V-cycle schedule once as a hipGraph and
                          replay it, with per-slice convergence flags on the device */
    int tile_rows;     /* rows per level-0 strip work item (even, >= 16); 0 = 80, halved
                          (down to 16) for batches too small to fill the GPU twice over */
    int inner_cycles;  /* MIXED: FP32 V-cycles per refinement step (default 3) */
    int launch_mode;   /* gdf_launch_mode for the multigrid passes (default GDF_LAUNCH_GRID) */
    int autotune;      /* 1: pick nu, fine_sweeps, coarse_sweeps, tile_rows and launch_mode by timing
                          candidate solves of this very call (see "Autotuning" below) */
    int fine_sweeps;   /* red-black sweeps in each fused finest-level pass (the post-sweeps
                          of one cycle plus the pre-sweeps of the next): 2 nu .. 2 nu + 2;
                          0 = 2 nu.  Extra sweeps lower the residual at each check and can
                          save a whole V-cycle. */
    int coarse_sweeps; /* red-black sweeps before and after each coarse correction on the
                          coarse levels: 1 .. 3, the same on every level; 0 = nu + 1, except
                          nu on levels where every slice's screening coefficient
                          (alpha 4^l on level l) is at least 0.05, where the extra sweep
                          buys no cycles (nu everywhere for GDF_PREC_MIXED, whose inner
                          solves run a fixed number of cycles).  The coarse levels are
                          small and latency-bound, so a third sweep there costs little and
                          lowers the residual of every cycle. */
    int robust;        /* fuse_stack: 1 = robust cross-slice averaging ("Extensions and
                          Applications"): at each voxel, of the in-plane smoothed values
                          of the slices in the cross-slice window, those more than two
                          weighted standard deviations from the window's weighted mean
                          are left out of the average (one pass).  FP32 and MIXED only
                          (GDF_EUNSUPPORTED with GDF_PREC_FP64); 0 = plain averaging. */
    int z_begin, z_end; /* fuse_stack: solve only the slices [z_begin, z_end) of the stack
                          (0, 0 = all).  The other slices only enter the cross-slice window
                          of these (Section III-A), so a chunk of a larger stack, given with
                          floor(3 sigma_z) slices on either side, gives the whole-stack
                          result for its own slices ("Distributed Processing").  f_dev,
                          g_smooth_dev and report_host then hold z_end - z_begin slices. */
    int sor;           /* 1: over-relaxed red-black sweeps in the fused finest passes: every
                          half-sweep after the first of a pass moves its pixels by 1.2 times
                          the Gauss-Seidel step (a solver choice, not the paper's).  FP32 and
                          MIXED hierarchies with fine_sweeps 4 or 5, Neumann boundary
                          (GDF_EUNSUPPORTED otherwise); 0 = Gauss-Seidel.  The autotuner
                          tries it when left at 0. */
    int reserved[1];
} gdf_solve_opts;

typedef enum {
    GDF_LAUNCH_DEFAULT = 0,     /* library default (GDF_LAUNCH_GRID) */
    GDF_LAUNCH_GRID = 1,        /* one wavefront per work item: the grid covers the work list */
    GDF_LAUNCH_PERSISTENT = 2   /* grid capped at the workgroups resident on the GPU at once;
                                   each wavefront loops over the work list */
} gdf_launch_mode;

/* Per-slice outcome (host memory, filled when a report pointer is given). */
typedef struct {
    int vcycles;                /* coarse-grid corrections applied */
    int status;                 /* gdf_status of this slice */
    double rel_residual;        /* FP64 ||b - A f|| / ||b|| of the returned f (before
                                   rounding to out_dtype) */
    double rel_residual_init;   /* the same for f = g_o (the zero correction) */
} gdf_slice_report;

/* One slice of a batch (host memory).  Offsets and row pitches are in
 * elements of the buffer they index. */
typedef struct {
    int H, W;                   /* slice height and width, >= 1; W <= 4194304 */
    double alpha;               /* screening weight of Eq. (1), > 0 */
    long long off_gs, pitch_gs; /* g_s (smoothed slice) */
    long long off_go, pitch_go; /* g_o (original slice) */
    long long off_f, pitch_f;   /* f (output); also grad_f / grad_gs / grad_go in the backward */
} gdf_slice_desc;

/* Message describing the last error on the calling thread ("" if none). */
const char *gdf_last_error(void);

/* Library version string. */
const char *gdf_version(void);

/* Releases the library's caches: captured graphs (per device), autotuning
 * choices and recent host-side plans (work lists and workspace layouts).
 * Safe to call at any time when no other call is running. */
void gdf_release(void);

/* ------------------------------------------------------------------------ */
/* fuse_stack: the whole method on a uint8 stack (Section III-A then Eq. (1)).
 *
 * stack_dev      uint8 [S][H][W] at element strides (pitch_slice, pitch_row);
 *                W <= 4194304.
 * alpha          screening weight, > 0 and finite.
 * bc             gdf_bc: GDF_BC_NEUMANN or GDF_BC_PERIODIC (the blend only: the
 *                smoothing renormalises at the stack's edges for either).
 * tol            target relative residual per slice, in (0, 1).
 * sigma_xy/z     Gaussian widths in pixels/slices, >= 0; 0 disables that axis.
 *                The kernel is truncated at floor(3 sigma) taps per axis and
 *                renormalised over the taps inside the stack.
 * f_dev          output [S][H][W] contiguous, dtype opts.out_dtype.
 * g_smooth_dev   optional output [S][H][W] contiguous (NULL to skip): I1 in
 *                FP32 (FP64 when precision is GDF_PREC_FP64).
 * report_host    optional [S] per-slice report.
 * With opts.use_graph the smoothing and the whole solve are captured as one
 * graph per (sizes, pointers, stream, options) and replayed, convergence
 * decided on the device: the call then waits for the device only to read the
 * report (cap opts.max_vcycles: the graph holds that many cycles, which
 * converged slices skip).  With use_graph and report_host NULL the call is
 * asynchronous: it returns GDF_OK once the work is enqueued on the stream,
 * without waiting; slices are not checked against tol on the host and
 * slices left at the FP32 floor are not re-solved (reading the report is
 * what decides both).  The workspace and buffers must stay valid until the
 * stream has run the work.
 * Returns GDF_OK when every slice reached tol.                              */
size_t gdf_fuse_workspace_size(int S, int H, int W, const gdf_solve_opts *opts);

gdf_status fuse_stack(const uint8_t *stack_dev, int S, int H, int W, long long pitch_row,
                      long long pitch_slice, double alpha, int bc, double tol, double sigma_xy,
                      double sigma_z, void *f_dev, void *g_smooth_dev, const gdf_solve_opts *opts,
                      void *workspace_dev, size_t workspace_bytes, gdf_slice_report *report_host,
                      void *stream);

/* ------------------------------------------------------------------------ */
/* solve_slices: Eq. (1) for a batch of slices of possibly different sizes and
 * screening weights, from caller-supplied g_s and g_o.
 *
 * desc_host      [n] slice descriptors (sizes, alpha, offsets, pitches).
 * gs_dtype/gs    g_s buffer: GDF_F32 or GDF_F64.
 * go_dtype/go    g_o buffer: GDF_U8, GDF_F32 or GDF_F64.
 * f_dev          output buffer, dtype opts.out_dtype.
 * Uneven batches run as one work list per multigrid level; with
 * opts.use_graph the schedule is captured once and replayed, and with
 * use_graph and report_host NULL the call is asynchronous (as fuse_stack).  */
size_t gdf_solve_workspace_size(int n, const gdf_slice_desc *desc_host, const gdf_solve_opts *opts);

gdf_status solve_slices(int n, const gdf_slice_desc *desc_host, int gs_dtype, const void *gs_dev,
                        int go_dtype, const void *go_dev, int bc, double tol, void *f_dev,
                        const gdf_solve_opts *opts, void *workspace_dev, size_t workspace_bytes,
                        gdf_slice_report *report_host, void *stream);

/* ------------------------------------------------------------------------ */
/* solve_slices_backward: gradients of a scalar loss through Eq. (1).
 *
 * Given grad_f = dLoss/df, solves the adjoint system A lambda = grad_f (A is
 * symmetric, so the same multigrid solver is reused) and forms
 *     dLoss/dg_s = alpha lambda,  dLoss/dg_o = L lambda,
 *     dLoss/dalpha_j = lambda_j . (g_s,j - f_j)   (FP64 sum per slice).
 * dtype (GDF_F32 or GDF_F64) applies to grad_f, f, g_s and the gradient
 * outputs; it must match opts.precision (F64 <-> GDF_PREC_FP64).  With F32
 * data the adjoint system is solved by FP32 V-cycles inside FP64 iterative
 * refinement: grad_f is usually rough (e.g. a data-misfit gradient) and lambda
 * then has large smooth components that an FP32 iterate cannot resolve to tol.  grad_f, f, grad_gs and grad_go use (off_f, pitch_f) of each
 * descriptor; g_s uses (off_gs, pitch_gs).  grad_gs_dev, grad_go_dev and
 * grad_alpha_host may each be NULL.
 * grad_alpha_sum_dev (device, one double, nullable): the sum over the slices
 * of dLoss/dalpha_j, formed on the device in slice order -- the gradient of a
 * scalar alpha shared by every slice.                                        */
size_t gdf_backward_workspace_size(int n, const gdf_slice_desc *desc_host,
                                   const gdf_solve_opts *opts);

gdf_status solve_slices_backward(int n, const gdf_slice_desc *desc_host, int dtype,
                                 const void *grad_f_dev, const void *f_dev, const void *gs_dev,
                                 int bc, double tol, void *grad_gs_dev, void *grad_go_dev,
                                 double *grad_alpha_host, double *grad_alpha_sum_dev, const gdf_solve_opts *opts,
                                 void *workspace_dev, size_t workspace_bytes,
                                 gdf_slice_report *report_host, void *stream);

/* ------------------------------------------------------------------------ */
/* Autotuning.  With opts.autotune = 1, any of the three solve entry points
 * first times complete solves of its own arguments under candidate settings
 * and then runs once more with the fastest, whose outputs and report it
 * returns.  Tuned, in this order, each among the values left at 0 by the
 * caller: nu (2, 1: sweeps per smoothing step), fine_sweeps (2 nu, 2 nu + 1,
 * 2 nu + 2: how many red-black sweeps the fused finest pass applies per pass
 * over HBM), coarse_sweeps (nu + 1, nu), tile_rows (heuristic, 32, 64, 128,
 * 256 rows per work item) and launch_mode (grid, persistent).  The choice is cached per
 * batch signature (entry point, sizes, alphas, tol, precision, dtypes, fixed
 * options) until gdf_release.  The workspace size functions return the
 * largest size over the candidates when opts.autotune = 1.  Candidate runs
 * write the outputs several times; a candidate that does not finish with
 * GDF_OK is discarded.
 *
 * gdf_autotune_last copies the settings used by the last autotuned call on
 * the calling thread into *opts_host and returns 1 (0 if there was none).   */
int gdf_autotune_last(gdf_solve_opts *opts_host);

/* ------------------------------------------------------------------------ */
/* Gradient through the smoothing (derived from Section III-A; the paper does
 * not differentiate).  The smoothing maps a stack I0 to I1(p) = sum_q K(q - p)
 * I0(q) / D(p), K the truncated anisotropic Gaussian (radius floor(3 sigma)
 * per axis) and D(p) the sum of its in-stack weights.  smooth_transpose
 * applies the transpose: out(q) = sum_p K(q - p) grad(p) / D(p), the gradient
 * of a loss with respect to the stack given grad = dLoss/dI1.  Together with
 * solve_slices_backward (dLoss/dg_s, dLoss/dg_o) it differentiates
 * fuse_stack: dLoss/dstack = smooth_transpose(dLoss/dg_s) + dLoss/dg_o (add_dev
 * = dLoss/dg_o, or out_dev holding it with add_dev = out_dev).
 *
 * grad_dev, out_dev  [S][H][W] FP32 device buffers, contiguous; out_dev must
 *                    not alias grad_dev.
 * add_dev            NULL, or [S][H][W] FP32 added to the result:
 *                    out = K (grad / D) + add.  It may be out_dev itself
 *                    (accumulate in place), not grad_dev.  With W a multiple of 4 and 16-byte
 *                    aligned buffers and workspace the passes move four
 *                    voxels per thread; any other shape or alignment is
 *                    accepted and takes one-voxel passes (equal up to FP32
 *                    rounding order).
 * sigma_xy, sigma_z  as for fuse_stack (in-plane radius <= 7, cross-slice
 *                    radius <= 12).
 * workspace          gdf_smooth_transpose_workspace_size(S, H, W) bytes of
 *                    device memory owned by the caller.
 * Returns GDF_EINVAL / GDF_EUNSUPPORTED on bad arguments and GDF_ENOMEM for a
 * workspace smaller than the query (nothing launched), GDF_EDEVICE on a HIP
 * error.  Asynchronous on `stream`: the per-axis weight-sum tables are
 * computed on the device, in the workspace.                                  */
size_t gdf_smooth_transpose_workspace_size(int S, int H, int W);
gdf_status smooth_transpose(const float *grad_dev, int S, int H, int W, double sigma_xy, double sigma_z,
                            float *out_dev, const float *add_dev, void *workspace, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* solve_slices_noalloc: solve_slices for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments and results as solve_slices, without the
 * workspace: the library's static device scratch of GDF_NOALLOC_SCRATCH_BYTES
 * per GPU (256 MiB, placed when the library is loaded on that GPU and held
 * until the process ends) serves instead.  The call allocates no device
 * memory and no page-locked host memory.
 *  - GDF_ENOMEM (nothing launched) when gdf_solve_workspace_size for the same
 *    batch and options exceeds GDF_NOALLOC_SCRATCH_BYTES (a single FP32 slice
 *    of up to about 2900 x 2900 pixels fits).
 *  - GDF_EUNSUPPORTED for opts.use_graph (instantiating a graph allocates).
 *  - The device is the stream's (the current device for a NULL stream).
 *  - Every call on one GPU uses that GPU's one scratch array, which keeps the
 *    last call's contents (each call initialises what it reads).  Calls from
 *    threads of one process are serialised per device, and each call returns
 *    after its work on the stream has finished, so they do not overlap; calls
 *    from two processes on one GPU use separate arrays.                       */
#define GDF_NOALLOC_SCRATCH_BYTES (256u << 20)
gdf_status solve_slices_noalloc(int n, const gdf_slice_desc *desc_host, int gs_dtype, const void *gs_dev,
                                int go_dtype, const void *go_dev, int bc, double tol, void *f_dev,
                                const gdf_solve_opts *opts, gdf_slice_report *report_host, void *stream);

/* ------------------------------------------------------------------------ */
/* Kernel timing for measurement.  When enabled, the library brackets every
 * launch of the named kernel class with HIP events on the launch stream and
 * accumulates their durations.  gdf_profile_enable(1) times every class,
 * gdf_profile_enable(2) only "vcycle_fine" (fewer events in flight),
 * gdf_profile_enable(0) stops.  Classes: "smooth", "vcycle_fine" (the fused
 * finest-level post-/pre-smoothing pass), "vcycle_fine_first" (the same pass
 * in the first cycle of a solve from zero, which reads no iterate),
 * "restrict_first" (the restriction of the right-hand side before the first
 * cycle; in an FP32 fuse_stack the smoothing pass does it and this class
 * records nothing), "coarse", "finalize", "prep", "refine", "adjoint".
 * Returns the number of launches
 * recorded and writes the summed milliseconds and the summed algorithmic
 * HBM bytes.                                                                 */
void gdf_profile_enable(int on);
int gdf_profile_read(const char *kernel_class, double *total_ms_host, double *algo_bytes_host);
void gdf_profile_reset(void);

#ifdef __cplusplus
}
#endif

#endif /* GDF_H */
