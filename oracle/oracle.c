/*
 * FP64 CPU oracle for gradient-domain fusion of EM stacks
 * (Kazhdan et al., "Gradient-Domain Fusion for Color Correction in Large EM
 * Image Stacks", arXiv 1506.02079).
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously correct C: every function
 * is the definition it cites, written out in double precision, with no
 * blocking, fusion or reordering.  It shares no code, header, table or helper
 * with the GPU library; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may call it.
 *
 * Readings of the paper taken here (each also listed in the design notes):
 *  - Smoothing (Section III-A; Implementation subsection): the kernel is the
 *    axis-aligned anisotropic Gaussian, truncated per axis at three standard
 *    deviations (taps with |d| <= 3 sigma are kept, so the radius is
 *    floor(3 sigma)), and the result is a weighted average: the sum is
 *    divided by the sum of the weights of the taps that fall inside the stack.
 *    The continuous normalising constant cancels in that division.  sigma = 0
 *    leaves that axis untouched.
 *  - Screened-Poisson blend (Section III-B, the energy and Eq. (1)): on the
 *    pixel grid with unit spacing, the per-slice system is
 *        (alpha I + L) f = alpha g_s + L g_o,
 *    where L is the graph Laplacian of the 4-connected pixel grid,
 *    (L v)_p = sum over neighbours q of p inside the slice of (v_p - v_q).
 *    This is the normal equation of the discrete energy
 *        alpha sum_p (f_p - g_s,p)^2 + sum_edges ((f_p - f_q) - (g_o,p - g_o,q))^2,
 *    i.e. -Laplacian with reflecting (Neumann) boundaries, the natural
 *    boundary condition of the paper's energy.  Periodic boundaries (the
 *    paper's Fourier basis) wrap the neighbours instead.
 *  - Relative residual (definition accompanying the solver-statistics table
 *    in the paper's unrendered results block): ||b - A f||_2 / ||b||_2 with
 *    b = alpha g_s + L g_o, per slice.
 *  - Adjoint (derived from Eq. (1); the paper does not differentiate): for a
 *    loss with gradient gbar = dLoss/df, lambda = A^{-1} gbar,
 *    dLoss/dg_s = alpha lambda, dLoss/dg_o = L lambda,
 *    dLoss/dalpha = lambda . (g_s - f).
 *  - Gradient through the smoothing (derived): the transpose of the linear
 *    map stack -> smoothed stack, see oracle_smooth_transpose.
 *  - Robust averaging ("Extensions and Applications"): see
 *    oracle_smooth_robust_voxel for the reading taken.
 */
#include <math.h>
#include <omp.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Threads the OpenMP loops below run on (reported beside oracle timings). */
int oracle_threads(void) { return omp_get_max_threads(); }

#define ORACLE_BC_NEUMANN 0
#define ORACLE_BC_PERIODIC 1

/* ---------------------------------------------------------------- smoothing */

/* Truncation radius: taps up to three standard deviations are kept. */
static int tap_radius(double sigma) { return sigma > 0.0 ? (int)floor(3.0 * sigma) : 0; }

/* One-axis factor of the anisotropic Gaussian exp(-d^2 / 2 sigma^2). */
static double gauss_factor(int d, double sigma)
{
    if (sigma <= 0.0) return d == 0 ? 1.0 : 0.0;
    return exp(-(double)d * (double)d / (2.0 * sigma * sigma));
}

/* I1(z,y,x): weighted average of the stack over the truncated anisotropic
 * Gaussian centred at (z,y,x), renormalised over the taps inside the stack.
 * Section III-A and the Implementation subsection (3-sigma support). */
double oracle_smooth_voxel(const uint8_t *stack, int S, int H, int W,
                           double sigma_xy, double sigma_z, int z, int y, int x)
{
    const int rxy = tap_radius(sigma_xy), rz = tap_radius(sigma_z);
    double num = 0.0, den = 0.0;
    for (int dz = -rz; dz <= rz; ++dz) {
        const int zz = z + dz;
        if (zz < 0 || zz >= S) continue;
        for (int dy = -rxy; dy <= rxy; ++dy) {
            const int yy = y + dy;
            if (yy < 0 || yy >= H) continue;
            for (int dx = -rxy; dx <= rxy; ++dx) {
                const int xx = x + dx;
                if (xx < 0 || xx >= W) continue;
                const double w = gauss_factor(dx, sigma_xy) * gauss_factor(dy, sigma_xy) *
                                 gauss_factor(dz, sigma_z);
                num += w * (double)stack[((size_t)zz * H + yy) * W + xx];
                den += w;
            }
        }
    }
    return num / den;
}

/* The whole smoothed stack, one voxel at a time (OpenMP over rows). */
void oracle_smooth(const uint8_t *stack, int S, int H, int W, double sigma_xy,
                   double sigma_z, double *out)
{
    const long long rows = (long long)S * H;
#pragma omp parallel for schedule(dynamic, 4)
    for (long long zy = 0; zy < rows; ++zy) {
        const int z = (int)(zy / H), y = (int)(zy % H);
        for (int x = 0; x < W; ++x)
            out[(size_t)zy * W + x] = oracle_smooth_voxel(stack, S, H, W, sigma_xy, sigma_z, z, y, x);
    }
}

/* Values at a list of voxels (z, y, x triples). */
void oracle_smooth_points(const uint8_t *stack, int S, int H, int W, double sigma_xy,
                          double sigma_z, const int *zyx, long long n, double *out)
{
#pragma omp parallel for schedule(static)
    for (long long i = 0; i < n; ++i)
        out[i] = oracle_smooth_voxel(stack, S, H, W, sigma_xy, sigma_z, zyx[3 * i], zyx[3 * i + 1],
                                     zyx[3 * i + 2]);
}

/* Robust cross-slice averaging ("Extensions and Applications": only colour
 * values within two standard deviations are averaged).  Reading taken here:
 * the robust step acts on the average across slices.  At (z,y,x) the window's
 * values are p_d, the in-plane smoothed value of slice z+d at (y,x) (the
 * renormalised in-plane Gaussian average), with weights w_d of the cross-slice
 * Gaussian for the slices inside the stack.  Their weighted mean mu and
 * weighted variance var = sum w (p - mu)^2 / sum w are taken once; the result
 * is the weighted average of the p_d with (p_d - mu)^2 <= 4 var.  With nothing
 * left out this is oracle_smooth_voxel (the 3D weights factor).  One pass,
 * weighted statistics. */
static double inplane_voxel(const uint8_t *stack, int H, int W, double sigma_xy, int z, int y, int x)
{
    const int rxy = tap_radius(sigma_xy);
    double num = 0.0, den = 0.0;
    for (int dy = -rxy; dy <= rxy; ++dy) {
        const int yy = y + dy;
        if (yy < 0 || yy >= H) continue;
        for (int dx = -rxy; dx <= rxy; ++dx) {
            const int xx = x + dx;
            if (xx < 0 || xx >= W) continue;
            const double w = gauss_factor(dx, sigma_xy) * gauss_factor(dy, sigma_xy);
            num += w * (double)stack[((size_t)z * H + yy) * W + xx];
            den += w;
        }
    }
    return num / den;
}

double oracle_smooth_robust_voxel(const uint8_t *stack, int S, int H, int W, double sigma_xy,
                                  double sigma_z, int z, int y, int x)
{
    const int rz = tap_radius(sigma_z);
    /* the window's arrays hold 64 taps: a wider window is refused (NaN), never cut short */
    if (2 * rz + 1 > 64) return NAN;
    double p[64], w[64];
    int n = 0;
    for (int dz = -rz; dz <= rz; ++dz) {
        const int zz = z + dz;
        if (zz < 0 || zz >= S) continue;
        p[n] = inplane_voxel(stack, H, W, sigma_xy, zz, y, x);
        w[n] = gauss_factor(dz, sigma_z);
        ++n;
    }
    double sw = 0.0, swp = 0.0;
    for (int i = 0; i < n; ++i) {
        sw += w[i];
        swp += w[i] * p[i];
    }
    const double mu = swp / sw;
    double sv = 0.0;
    for (int i = 0; i < n; ++i) sv += w[i] * (p[i] - mu) * (p[i] - mu);
    const double var = sv / sw;
    double num = 0.0, den = 0.0;
    for (int i = 0; i < n; ++i)
        if ((p[i] - mu) * (p[i] - mu) <= 4.0 * var) {
            num += w[i] * p[i];
            den += w[i];
        }
    return num / den;
}

/* Robust values at a list of voxels (z, y, x triples). */
void oracle_smooth_robust_points(const uint8_t *stack, int S, int H, int W, double sigma_xy, double sigma_z,
                                 const int *zyx, long long n, double *out)
{
#pragma omp parallel for schedule(static)
    for (long long i = 0; i < n; ++i)
        out[i] = oracle_smooth_robust_voxel(stack, S, H, W, sigma_xy, sigma_z, zyx[3 * i], zyx[3 * i + 1],
                                            zyx[3 * i + 2]);
}

void oracle_smooth_robust(const uint8_t *stack, int S, int H, int W, double sigma_xy, double sigma_z,
                          double *out)
{
    const long long rows = (long long)S * H;
#pragma omp parallel for schedule(dynamic, 4)
    for (long long zy = 0; zy < rows; ++zy) {
        const int z = (int)(zy / H), y = (int)(zy % H);
        for (int x = 0; x < W; ++x)
            out[(size_t)zy * W + x] = oracle_smooth_robust_voxel(stack, S, H, W, sigma_xy, sigma_z, z, y, x);
    }
}

/* Transpose of the smoothing operator, for the gradient through it (derived:
 * the paper does not differentiate).  Smoothing is I1(p) = sum_q K(q - p) I0(q)
 * / D(p) over the in-stack window of p, with D(p) the sum of its in-stack
 * weights; so for a gradient G on I1, dLoss/dI0(q) = sum_p K(q - p) G(p) / D(p)
 * over the voxels p whose window holds q (K is symmetric). */
void oracle_smooth_transpose(const double *g, int S, int H, int W, double sigma_xy, double sigma_z,
                             double *out)
{
    const int rxy = tap_radius(sigma_xy), rz = tap_radius(sigma_z);
    const long long n = (long long)S * H * W;
    double *gd = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int z = 0; z < S; ++z)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                double den = 0.0;
                for (int dz = -rz; dz <= rz; ++dz)
                    for (int dy = -rxy; dy <= rxy; ++dy)
                        for (int dx = -rxy; dx <= rxy; ++dx) {
                            const int zz = z + dz, yy = y + dy, xx = x + dx;
                            if (zz < 0 || zz >= S || yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
                            den += gauss_factor(dx, sigma_xy) * gauss_factor(dy, sigma_xy) * gauss_factor(dz, sigma_z);
                        }
                const size_t i = ((size_t)z * H + y) * W + x;
                gd[i] = g[i] / den;
            }
    for (int z = 0; z < S; ++z)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                double acc = 0.0;
                for (int dz = -rz; dz <= rz; ++dz)
                    for (int dy = -rxy; dy <= rxy; ++dy)
                        for (int dx = -rxy; dx <= rxy; ++dx) {
                            const int zz = z + dz, yy = y + dy, xx = x + dx;
                            if (zz < 0 || zz >= S || yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
                            acc += gauss_factor(dx, sigma_xy) * gauss_factor(dy, sigma_xy) * gauss_factor(dz, sigma_z) *
                                   gd[((size_t)zz * H + yy) * W + xx];
                        }
                out[((size_t)z * H + y) * W + x] = acc;
            }
    free(gd);
}

/* ---------------------------------------------------------- grid operators */

/* Neighbour index of (y,x) displaced by (dy,dx), or -1 if it leaves the slice
 * (Neumann: no edge) ; periodic boundaries wrap. */
static long long nbr(int y, int x, int dy, int dx, int H, int W, int bc)
{
    int yy = y + dy, xx = x + dx;
    if (bc == ORACLE_BC_PERIODIC) {
        yy = (yy % H + H) % H;
        xx = (xx % W + W) % W;
    } else if (yy < 0 || yy >= H || xx < 0 || xx >= W) {
        return -1;
    }
    return (long long)yy * W + xx;
}

/* (L v)_p = sum over grid neighbours q of (v_p - v_q). */
void oracle_laplacian(const double *v, int H, int W, int bc, double *out)
{
    static const int D[4][2] = {{-1, 0}, {1, 0}, {0, -1}, {0, 1}};
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const long long p = (long long)y * W + x;
            double s = 0.0;
            for (int k = 0; k < 4; ++k) {
                const long long q = nbr(y, x, D[k][0], D[k][1], H, W, bc);
                if (q >= 0) s += v[p] - v[q];
            }
            out[p] = s;
        }
}

/* (A v) = alpha v + L v : the left-hand side of Eq. (1). */
void oracle_apply_A(const double *v, int H, int W, double alpha, int bc, double *out)
{
    const long long n = (long long)H * W;
    oracle_laplacian(v, H, W, bc, out);
#pragma omp parallel for schedule(static)
    for (long long p = 0; p < n; ++p) out[p] += alpha * v[p];
}

/* b = alpha g_s + L g_o : the right-hand side of Eq. (1). */
void oracle_rhs(const double *gs, const double *go, int H, int W, double alpha, int bc, double *b)
{
    const long long n = (long long)H * W;
    oracle_laplacian(go, H, W, bc, b);
#pragma omp parallel for schedule(static)
    for (long long p = 0; p < n; ++p) b[p] += alpha * gs[p];
}

static double dot(const double *a, const double *b, long long n)
{
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (long long i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Unpreconditioned conjugate gradients on (alpha I + L) x = b from x = 0,
 * run until the true residual satisfies ||b - A x|| <= tol ||b||.  CG's
 * recursive residual is re-anchored to the true one when it reports
 * convergence.  Returns the iteration count, or -1 if maxit was reached. */
int oracle_cg(const double *b, int H, int W, double alpha, int bc, double tol, int maxit, double *x,
              double *relres_out)
{
    const long long n = (long long)H * W;
    double *r = malloc(n * sizeof(double)), *p = malloc(n * sizeof(double)),
           *Ap = malloc(n * sizeof(double));
    memset(x, 0, n * sizeof(double));
    memcpy(r, b, n * sizeof(double));
    const double bnorm = sqrt(dot(b, b, n));
    int it = 0, ok = 0;
    double rel = 0.0;
    if (bnorm == 0.0) {
        ok = 1;
        goto done;
    }
    for (int restart = 0; restart < 8 && !ok && it < maxit; ++restart) {
        /* r = b - A x (true residual) */
        oracle_apply_A(x, H, W, alpha, bc, Ap);
        for (long long i = 0; i < n; ++i) r[i] = b[i] - Ap[i];
        double rr = dot(r, r, n);
        if (sqrt(rr) <= tol * bnorm) {
            ok = 1;
            break;
        }
        memcpy(p, r, n * sizeof(double));
        while (it < maxit) {
            oracle_apply_A(p, H, W, alpha, bc, Ap);
            const double a = rr / dot(p, Ap, n);
#pragma omp parallel for schedule(static)
            for (long long i = 0; i < n; ++i) {
                x[i] += a * p[i];
                r[i] -= a * Ap[i];
            }
            const double rr_new = dot(r, r, n);
            ++it;
            if (sqrt(rr_new) <= 0.5 * tol * bnorm) break;
            const double beta = rr_new / rr;
            rr = rr_new;
#pragma omp parallel for schedule(static)
            for (long long i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        }
    }
done:
    oracle_apply_A(x, H, W, alpha, bc, Ap);
    {
        double s = 0.0;
        for (long long i = 0; i < n; ++i) s += (b[i] - Ap[i]) * (b[i] - Ap[i]);
        rel = bnorm > 0.0 ? sqrt(s) / bnorm : sqrt(s);
        ok = rel <= tol;
    }
    if (relres_out) *relres_out = rel;
    free(r);
    free(p);
    free(Ap);
    return ok ? it : -1;
}

/* Solve Eq. (1) for one slice: f = (alpha I + L)^{-1} (alpha g_s + L g_o). */
int oracle_solve(const double *gs, const double *go, int H, int W, double alpha, int bc, double tol,
                 int maxit, double *f, double *relres_out)
{
    double *b = malloc((size_t)H * W * sizeof(double));
    oracle_rhs(gs, go, H, W, alpha, bc, b);
    const int it = oracle_cg(b, H, W, alpha, bc, tol, maxit, f, relres_out);
    free(b);
    return it;
}

/* ||b - A f|| / ||b|| with b = alpha g_s + L g_o (plain norm of A f if b = 0). */
double oracle_relres(const double *f, const double *gs, const double *go, int H, int W, double alpha,
                     int bc)
{
    const long long n = (long long)H * W;
    double *b = malloc(n * sizeof(double)), *Af = malloc(n * sizeof(double));
    oracle_rhs(gs, go, H, W, alpha, bc, b);
    oracle_apply_A(f, H, W, alpha, bc, Af);
    double rr = 0.0, bb = 0.0;
    for (long long i = 0; i < n; ++i) {
        rr += (b[i] - Af[i]) * (b[i] - Af[i]);
        bb += b[i] * b[i];
    }
    free(b);
    free(Af);
    return bb > 0.0 ? sqrt(rr / bb) : sqrt(rr);
}

/* Gradients of a loss through the solve of Eq. (1), given gbar = dLoss/df. */
int oracle_adjoint(const double *gbar, const double *gs, const double *f, int H, int W, double alpha,
                   int bc, double tol, int maxit, double *d_gs, double *d_go, double *d_alpha)
{
    const long long n = (long long)H * W;
    double *lam = malloc(n * sizeof(double));
    const int it = oracle_cg(gbar, H, W, alpha, bc, tol, maxit, lam, NULL);
    if (d_gs)
        for (long long i = 0; i < n; ++i) d_gs[i] = alpha * lam[i];
    if (d_go) oracle_laplacian(lam, H, W, bc, d_go);
    if (d_alpha) {
        double s = 0.0;
        for (long long i = 0; i < n; ++i) s += lam[i] * (gs[i] - f[i]);
        *d_alpha = s;
    }
    free(lam);
    return it;
}
