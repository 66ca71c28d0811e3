// Per-pixel kernels around the multigrid solve of Eq. (1): right-hand side
// formation, output formation with the FP64 residual of the returned f, the
// adjoint assembly, the FP64 refinement step of the mixed-precision solve,
// and the fixed-order per-slice reductions.
//
// All of them walk 64 x 16 pixel tiles (256 threads; thread (tx, ty) handles
// rows ty, ty + 4, ty + 8, ty + 12 of column tx), so rows are read coalesced;
// stencil neighbours come from the same or adjacent rows and hit L2.  Partial
// sums are reduced per tile in FP64 and written to a per-tile slot; a second
// kernel sums each slice's slots in a fixed order.
#include "internal.h"

namespace gdf {

constexpr int kTileW = 64, kTileH = 16;

__device__ __forceinline__ int find_slice(const SliceIO *io, int n, long long tile)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (io[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <typename TV> __device__ __forceinline__ double ldv(const TV *p, long long i) { return (double)p[i]; }

__device__ double block_sum(double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

struct TileCtx {
    int si, x, ty0;
    SliceIO P;
};

__device__ __forceinline__ bool tile_ctx(const SliceIO *io, int n, long long n_tiles, TileCtx &c)
{
    const long long tile = blockIdx.x;
    if (tile >= n_tiles) return false;
    c.si = find_slice(io, n, tile);
    c.P = io[c.si];
    const long long lt = tile - c.P.tile_begin;
    c.x = (int)(lt % c.P.tiles_x) * kTileW + (threadIdx.x & 63);
    c.ty0 = (int)(lt / c.P.tiles_x) * kTileH;
    return true;
}

// ------------------------------------------------------------- finish ---

// One block per slice; fixed-order strided sum then a fixed tree, so the
// result does not depend on scheduling.
__global__ __launch_bounds__(256) void finish_kernel(int n_slices, const int *range,
                                                     const float2 *pf, const double *pd, int mode,
                                                     double tol, int max_cycles, int count_cycle,
                                                     double stall_ratio, SliceState *st, int *active)
{
    __shared__ double red[256];
    const int sidx = blockIdx.x;
    if (sidx >= n_slices) return;
    const int b0 = range[2 * sidx], b1 = range[2 * sidx + 1];
    double v = 0.0, w = 0.0;
    for (int i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
        if (pf) {
            v += (double)pf[i].x;
            w += (double)pf[i].y;
        } else {
            v += pd[i];
        }
    }
    const double sum = block_sum(v, red);
    const double rsum = pf ? block_sum(w, red) : 0.0;
    if (threadIdx.x != 0) return;
    SliceState &S = st[sidx];
    switch (mode) {
    case FIN_BB: S.bb = sum; break;
    case FIN_INIT: S.rel_init = S.bb > 0.0 ? sqrt(sum / S.bb) : sqrt(sum); break;
    case FIN_SUM: S.aux = sum; break;
    case FIN_MEAN:
        S.bmean = sum / S.npx;
        S.uoff = S.bmean / S.alpha;
        break;
    case FIN_FINAL:
        S.rr = sum;
        S.rel = S.bb > 0.0 ? sqrt(sum / S.bb) : sqrt(sum);
        if (!isfinite(sum)) S.status = 6;  // GDF_ENONFINITE
        break;
    case FIN_CHECK:
    default:
        if (!active[sidx]) return;   // frozen slice keeps its last state
        const double prev = S.rel;   // the previous check's (0 before the first)
        S.rr = sum;
        S.rel = S.bb > 0.0 ? sqrt(sum / S.bb) : sqrt(sum);
        if (count_cycle) S.cycles += 1;
        if (stall_ratio > 0.0 && count_cycle && S.cycles >= 2 && prev > 0.0 && S.rel > tol &&
            S.rel > stall_ratio * prev) {
            S.stalled = 1;
            active[sidx] = 0;
        }
        // Neumann: 1^T A = alpha 1^T, so the constant-mode error of the iterate is
        // exactly -mean(r) / alpha; adding it back removes mean(r) from the residual
        S.shift = pf ? rsum / (S.npx * S.alpha) : 0.0;
        if (!isfinite(sum)) S.status = 6;
        if (!isfinite(sum) || S.rel <= tol || S.cycles >= max_cycles) active[sidx] = 0;
        break;
    }
}

hipError_t launch_finish(int n_slices, const int *range, const float2 *partials_f,
                         const double *partials_d, int mode, double tol, int max_cycles,
                         int count_cycle, double stall_ratio, SliceState *state, int *active,
                         hipStream_t s)
{
    if (n_slices <= 0) return hipSuccess;
    hipLaunchKernelGGL(finish_kernel, dim3(n_slices), dim3(256), 0, s, n_slices, range, partials_f,
                       partials_d, mode, tol, max_cycles, count_cycle, stall_ratio, state, active);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void resume_flags_kernel(int n_slices, const SliceState *st, double tol,
                                                          int max_cycles, int *active, int *only)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_slices) return;
    const SliceState &S = st[i];
    const int again = S.status == 0 && !S.stalled && isfinite(S.rel) && S.rel > tol && S.cycles < max_cycles;
    active[i] = again;
    only[i] = again;
}

hipError_t launch_resume_flags(int n_slices, const SliceState *state, double tol, int max_cycles,
                               int *active, int *only, hipStream_t s)
{
    if (n_slices <= 0) return hipSuccess;
    hipLaunchKernelGGL(resume_flags_kernel, dim3((n_slices + 255) / 256), dim3(256), 0, s, n_slices, state,
                       tol, max_cycles, active, only);
    return hipGetLastError();
}

// --------------------------------------------------------------- prep ---

// b_u = alpha (g_s - g_o) and partial sums of ||alpha g_s + L g_o||^2 and ||b_u||^2.
template <typename T, typename TS, typename TO>
__global__ __launch_bounds__(256) void prep_kernel(const TS *gs, const TO *go, const SliceIO *io,
                                                   int n_slices, long long n_tiles,
                                                   const LevelDesc *levs, double *part_bb,
                                                   double *part_b0, double *part_bs)
{
    __shared__ double red[256];
    TileCtx c;
    if (!tile_ctx(io, n_slices, n_tiles, c)) return;
    const SliceIO &P = c.P;
    const LevelDesc &L = levs[P.lev0];
    const int x = c.x;
    const double al = P.alpha;
    double sbb = 0.0, sb0 = 0.0, sbs = 0.0;
    T *bdst = static_cast<T *>(L.b);
#pragma unroll
    for (int r0 = 0; r0 < kTileH; r0 += 4) {
        const int y = c.ty0 + r0 + (threadIdx.x >> 6);
        if (y >= P.H || x >= P.W) continue;
        const long long go_row = P.off_go + (long long)y * P.pitch_go;
        const double o = ldv(go, go_row + x);
        const double sv = ldv(gs, P.off_gs + (long long)y * P.pitch_gs + x);
        double lap = 0.0;   // (L g_o)_p over in-slice neighbours
        if (x > 0) lap += o - ldv(go, go_row + x - 1);
        if (x < P.W - 1) lap += o - ldv(go, go_row + x + 1);
        if (y > 0) lap += o - ldv(go, go_row - P.pitch_go + x);
        if (y < P.H - 1) lap += o - ldv(go, go_row + P.pitch_go + x);
        const double bf = al * sv + lap;
        const T bu = (T)(al * (sv - o));
        bdst[(size_t)y * L.pitch + x] = bu;
        sbb += bf * bf;
        sb0 += (double)bu * (double)bu;
        sbs += (double)bu;
    }
    const double tbb = block_sum(sbb, red);
    const double tb0 = block_sum(sb0, red);
    const double tbs = block_sum(sbs, red);
    if (threadIdx.x == 0) {
        part_bb[blockIdx.x] = tbb;
        part_b0[blockIdx.x] = tb0;
        part_bs[blockIdx.x] = tbs;
    }
}

template <typename T, typename TS>
static hipError_t prep_go(int go_dtype, const void *gs, const void *go, const SliceIO *io, int n,
                          long long nt, const LevelDesc *levs, double *pbb, double *pb0,
                          double *pbs, hipStream_t s)
{
    const dim3 g((unsigned)nt), blk(256);
    if (go_dtype == 0)
        hipLaunchKernelGGL((prep_kernel<T, TS, uint8_t>), g, blk, 0, s, (const TS *)gs, (const uint8_t *)go, io, n, nt, levs, pbb, pb0, pbs);
    else if (go_dtype == 1)
        hipLaunchKernelGGL((prep_kernel<T, TS, float>), g, blk, 0, s, (const TS *)gs, (const float *)go, io, n, nt, levs, pbb, pb0, pbs);
    else
        hipLaunchKernelGGL((prep_kernel<T, TS, double>), g, blk, 0, s, (const TS *)gs, (const double *)go, io, n, nt, levs, pbb, pb0, pbs);
    return hipGetLastError();
}

hipError_t launch_prep(bool fp64, int gs_dtype, const void *gs, int go_dtype, const void *go,
                       const SliceIO *io_dev, int n_slices, long long n_tiles,
                       const LevelDesc *levs, double *part_bb, double *part_b0, double *part_bs,
                       hipStream_t s)
{
    if (n_tiles <= 0) return hipSuccess;
    if (fp64)
        return gs_dtype == 2 ? prep_go<double, double>(go_dtype, gs, go, io_dev, n_slices, n_tiles, levs, part_bb, part_b0, part_bs, s)
                             : prep_go<double, float>(go_dtype, gs, go, io_dev, n_slices, n_tiles, levs, part_bb, part_b0, part_bs, s);
    return gs_dtype == 2 ? prep_go<float, double>(go_dtype, gs, go, io_dev, n_slices, n_tiles, levs, part_bb, part_b0, part_bs, s)
                         : prep_go<float, float>(go_dtype, gs, go, io_dev, n_slices, n_tiles, levs, part_bb, part_b0, part_bs, s);
}

// ----------------------------------------------------------- finalize ---

// f = g_o + u, and partial sums of the FP64 residual ||b_u - A u||^2 of the
// unrounded g_o + u (A(g_o + u) - (alpha g_s + L g_o) = A u - b_u).
template <typename T, typename TO, typename TF>
__global__ __launch_bounds__(256) void finalize_kernel(const TO *go, TF *f, const SliceIO *io,
                                                       int n_slices, long long n_tiles,
                                                       const LevelDesc *levs,
                                                       const SliceState *st, const int *only,
                                                       double *part_rr)
{
    __shared__ double red[256];
    TileCtx c;
    if (!tile_ctx(io, n_slices, n_tiles, c)) return;
    if (only && !only[c.si]) return;   // uniform per block: keeps this slice's partial sum
    const SliceIO &P = c.P;
    const LevelDesc &L = levs[P.lev0];
    const int x = c.x;
    const double sg = P.alpha;
    const T *u = static_cast<const T *>(L.u[st[c.si].cycles & 1]);
    const T *bu = static_cast<const T *>(L.b);
    // full correction = uoff (mean removed on load) + u + shift (constant-mode
    // correction); constants cancel in L, and b is used as stored
    const double shift = st[c.si].shift + st[c.si].uoff;
    const int pu = L.pitch;
    double srr = 0.0;
#pragma unroll
    for (int r0 = 0; r0 < kTileH; r0 += 4) {
        const int y = c.ty0 + r0 + (threadIdx.x >> 6);
        if (y >= P.H || x >= P.W) continue;
        const size_t p = (size_t)y * pu + x;
        const double uc = (double)u[p] + shift;
        double acc = 0.0;
        if (x > 0) acc += uc - ((double)u[p - 1] + shift);
        if (x < P.W - 1) acc += uc - ((double)u[p + 1] + shift);
        if (y > 0) acc += uc - ((double)u[p - pu] + shift);
        if (y < P.H - 1) acc += uc - ((double)u[p + pu] + shift);
        const double res = (double)bu[p] - sg * uc - acc;
        srr += res * res;
        const double o = ldv(go, P.off_go + (long long)y * P.pitch_go + x);
        f[P.off_f + (long long)y * P.pitch_f + x] = (TF)(o + uc);
    }
    const double t = block_sum(srr, red);
    if (threadIdx.x == 0) part_rr[blockIdx.x] = t;
}

template <typename T, typename TO>
static hipError_t fin_go(int out_dtype, const void *go, void *f, const SliceIO *io, int n,
                         long long nt, const LevelDesc *levs, const SliceState *st, const int *only,
                         double *prr, hipStream_t s)
{
    const dim3 g((unsigned)nt), blk(256);
    if (out_dtype == 2)
        hipLaunchKernelGGL((finalize_kernel<T, TO, double>), g, blk, 0, s, (const TO *)go, (double *)f, io, n, nt, levs, st, only, prr);
    else
        hipLaunchKernelGGL((finalize_kernel<T, TO, float>), g, blk, 0, s, (const TO *)go, (float *)f, io, n, nt, levs, st, only, prr);
    return hipGetLastError();
}

hipError_t launch_finalize(bool fp64, int go_dtype, const void *go, int out_dtype, void *f,
                           const SliceIO *io_dev, int n, long long n_tiles,
                           const LevelDesc *levs, const SliceState *st, const int *only,
                           double *part_rr, hipStream_t s)
{
    if (n_tiles <= 0) return hipSuccess;
    if (fp64) {
        if (go_dtype == 0) return fin_go<double, uint8_t>(out_dtype, go, f, io_dev, n, n_tiles, levs, st, only, part_rr, s);
        if (go_dtype == 1) return fin_go<double, float>(out_dtype, go, f, io_dev, n, n_tiles, levs, st, only, part_rr, s);
        return fin_go<double, double>(out_dtype, go, f, io_dev, n, n_tiles, levs, st, only, part_rr, s);
    }
    if (go_dtype == 0) return fin_go<float, uint8_t>(out_dtype, go, f, io_dev, n, n_tiles, levs, st, only, part_rr, s);
    if (go_dtype == 1) return fin_go<float, float>(out_dtype, go, f, io_dev, n, n_tiles, levs, st, only, part_rr, s);
    return fin_go<float, double>(out_dtype, go, f, io_dev, n, n_tiles, levs, st, only, part_rr, s);
}

// ------------------------------------------------------------ adjoint ---

template <typename T>
__global__ __launch_bounds__(256) void prep_adjoint_kernel(const T *gf, const SliceIO *io, int n,
                                                           long long n_tiles, const LevelDesc *levs,
                                                           double *part_bb, double *part_bs)
{
    __shared__ double red[256];
    TileCtx c;
    if (!tile_ctx(io, n, n_tiles, c)) return;
    const SliceIO &P = c.P;
    const LevelDesc &L = levs[P.lev0];
    T *bdst = static_cast<T *>(L.b);
    double sbb = 0.0, sbs = 0.0;
    for (int r = threadIdx.x >> 6; r < kTileH; r += 4) {
        const int y = c.ty0 + r;
        if (y >= P.H || c.x >= P.W) continue;
        const T v = gf[P.off_f + (long long)y * P.pitch_f + c.x];
        bdst[(size_t)y * L.pitch + c.x] = v;
        sbb += (double)v * (double)v;
        sbs += (double)v;
    }
    const double t = block_sum(sbb, red);
    const double t2 = block_sum(sbs, red);
    if (threadIdx.x == 0) {
        part_bb[blockIdx.x] = t;
        part_bs[blockIdx.x] = t2;
    }
}

hipError_t launch_prep_adjoint(bool fp64, const void *grad_f, const SliceIO *io_dev, int n,
                               long long n_tiles, const LevelDesc *levs, double *part_bb,
                               double *part_bs, hipStream_t s)
{
    if (n_tiles <= 0) return hipSuccess;
    if (fp64)
        hipLaunchKernelGGL(prep_adjoint_kernel<double>, dim3((unsigned)n_tiles), dim3(256), 0, s, (const double *)grad_f, io_dev, n, n_tiles, levs, part_bb, part_bs);
    else
        hipLaunchKernelGGL(prep_adjoint_kernel<float>, dim3((unsigned)n_tiles), dim3(256), 0, s, (const float *)grad_f, io_dev, n, n_tiles, levs, part_bb, part_bs);
    return hipGetLastError();
}

// lambda = A^{-1} grad_f (level-0 iterate): grad_gs = alpha lambda,
// grad_go = L lambda, partials of lambda . (g_s - f).
template <typename T, typename TL>
__device__ __forceinline__ void adjoint_tile(const TL *lam, double shift, const T *gs, const T *f,
                                             T *ggs, T *ggo, const TileCtx &c, int pl, double &sda)
{
    const SliceIO &P = c.P;
    const int x = c.x;
    for (int r = threadIdx.x >> 6; r < kTileH; r += 4) {
        const int y = c.ty0 + r;
        if (y >= P.H || x >= P.W) continue;
        const size_t p = (size_t)y * pl + x;
        const double lraw = (double)lam[p];
        const double l = lraw + shift;
        double lap = 0.0;   // L is blind to the constant shift
        if (x > 0) lap += lraw - (double)lam[p - 1];
        if (x < P.W - 1) lap += lraw - (double)lam[p + 1];
        if (y > 0) lap += lraw - (double)lam[p - pl];
        if (y < P.H - 1) lap += lraw - (double)lam[p + pl];
        const long long fo = P.off_f + (long long)y * P.pitch_f + x;
        if (ggs) ggs[fo] = (T)(P.alpha * l);
        if (ggo) ggo[fo] = (T)lap;
        sda += l * ((double)gs[P.off_gs + (long long)y * P.pitch_gs + x] - (double)f[fo]);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void adjoint_kernel(const T *gs, const T *f, T *ggs, T *ggo,
                                                      const SliceIO *io, int n, long long n_tiles,
                                                      const LevelDesc *levs, const SliceState *st,
                                                      double *const *u64, double *part_da)
{
    __shared__ double red[256];
    TileCtx c;
    if (!tile_ctx(io, n, n_tiles, c)) return;
    const SliceIO &P = c.P;
    const LevelDesc &L = levs[P.lev0];
    const int par = st[c.si].cycles & 1;
    double sda = 0.0;
    if (u64) {
        adjoint_tile<T, double>(u64[par * n + c.si], 0.0, gs, f, ggs, ggo, c, L.pitch, sda);
    } else {
        const T *lam = static_cast<const T *>(L.u[par]);
        const double shift = st[c.si].shift + st[c.si].uoff;   // constant parts of lambda
        adjoint_tile<T, T>(lam, shift, gs, f, ggs, ggo, c, L.pitch, sda);
    }
    const double t = block_sum(sda, red);
    if (threadIdx.x == 0) part_da[blockIdx.x] = t;
}

hipError_t launch_adjoint_assemble(bool fp64, const void *gs, const void *f, void *ggs, void *ggo,
                                   const SliceIO *io_dev, int n, long long n_tiles,
                                   const LevelDesc *levs, const SliceState *st, double *const *u64,
                                   double *part_da, hipStream_t s)
{
    if (n_tiles <= 0) return hipSuccess;
    if (fp64)
        hipLaunchKernelGGL(adjoint_kernel<double>, dim3((unsigned)n_tiles), dim3(256), 0, s, (const double *)gs, (const double *)f, (double *)ggs, (double *)ggo, io_dev, n, n_tiles, levs, st, u64, part_da);
    else
        hipLaunchKernelGGL(adjoint_kernel<float>, dim3((unsigned)n_tiles), dim3(256), 0, s, (const float *)gs, (const float *)f, (float *)ggs, (float *)ggo, io_dev, n, n_tiles, levs, st, u64, part_da);
    return hipGetLastError();
}

// ---------------------------------------------------- mixed refinement ---

template <typename TS, typename TO>
__global__ __launch_bounds__(256) void refine_kernel(RefineArgs a)
{
    __shared__ double red[256];
    TileCtx c;
    if (!tile_ctx(a.io, a.n_slices, a.n_tiles, c)) return;
    const SliceIO &P = c.P;
    double srr = 0.0;
    if (a.active[c.si]) {
        const LevelDesc &L = a.levs[P.lev0];
        const int pl = L.pitch, x = c.x, H = P.H, W = P.W;
        const double *uin = a.u64[a.in_sel * a.n_slices + c.si];
        double *uout = a.u64[(a.in_sel ^ 1) * a.n_slices + c.si];
        const float *e = static_cast<const float *>(L.u[a.e_sel]);
        float *rdst = static_cast<float *>(L.b);
        const TS *gs = static_cast<const TS *>(a.gs);
        const TO *go = static_cast<const TO *>(a.go);
        const bool first = a.first;
        auto val = [&](size_t p) -> double { return first ? 0.0 : uin[p] + (double)e[p]; };
        for (int r = threadIdx.x >> 6; r < kTileH; r += 4) {
            const int y = c.ty0 + r;
            if (y >= H || x >= W) continue;
            const size_t p = (size_t)y * pl + x;
            const double uc = val(p);
            double acc = 0.0;
            if (x > 0) acc += uc - val(p - 1);
            if (x < W - 1) acc += uc - val(p + 1);
            if (y > 0) acc += uc - val(p - pl);
            if (y < H - 1) acc += uc - val(p + pl);
            double bval;
            if (a.rhs) {
                bval = (double)static_cast<const TS *>(a.rhs)[P.off_f + (long long)y * P.pitch_f + x];
            } else {
                const double sv = (double)gs[P.off_gs + (long long)y * P.pitch_gs + x];
                const double o = (double)go[P.off_go + (long long)y * P.pitch_go + x];
                bval = P.alpha * (sv - o);
            }
            const double res = bval - P.alpha * uc - acc;
            uout[p] = uc;
            rdst[p] = (float)res;
            srr += res * res;
        }
    }
    const double t = block_sum(srr, red);
    if (threadIdx.x == 0) a.part_rr[blockIdx.x] = t;
}

hipError_t launch_refine(const RefineArgs &a, hipStream_t s)
{
    if (a.n_tiles <= 0) return hipSuccess;
    const dim3 g((unsigned)a.n_tiles), b(256);
    const bool s64 = a.gs_dtype == 2;
    switch (a.go_dtype) {
    case 0:
        if (s64) hipLaunchKernelGGL((refine_kernel<double, uint8_t>), g, b, 0, s, a);
        else hipLaunchKernelGGL((refine_kernel<float, uint8_t>), g, b, 0, s, a);
        break;
    case 1:
        if (s64) hipLaunchKernelGGL((refine_kernel<double, float>), g, b, 0, s, a);
        else hipLaunchKernelGGL((refine_kernel<float, float>), g, b, 0, s, a);
        break;
    default:
        if (s64) hipLaunchKernelGGL((refine_kernel<double, double>), g, b, 0, s, a);
        else hipLaunchKernelGGL((refine_kernel<float, double>), g, b, 0, s, a);
        break;
    }
    return hipGetLastError();
}

template <typename TO, typename TF>
__global__ __launch_bounds__(256) void finalize64_kernel(const TO *go, TF *f, const SliceIO *io,
                                                         int n, long long n_tiles,
                                                         double *const *u64, const SliceState *st,
                                                         const LevelDesc *levs)
{
    TileCtx c;
    if (!tile_ctx(io, n, n_tiles, c)) return;
    const SliceIO &P = c.P;
    const double *u = u64[(st[c.si].cycles & 1) * n + c.si];   // latest FP64 iterate
    const int pl = levs[P.lev0].pitch;
    for (int r = threadIdx.x >> 6; r < kTileH; r += 4) {
        const int y = c.ty0 + r;
        if (y >= P.H || c.x >= P.W) continue;
        const double o = (double)go[P.off_go + (long long)y * P.pitch_go + c.x];
        f[P.off_f + (long long)y * P.pitch_f + c.x] = (TF)(o + u[(size_t)y * pl + c.x]);
    }
}

hipError_t launch_finalize64(int go_dtype, const void *go, int out_dtype, void *f,
                             const SliceIO *io, int n, long long nt, double *const *u64,
                             const SliceState *st, const LevelDesc *levs, hipStream_t s)
{
    if (nt <= 0) return hipSuccess;
    const dim3 g((unsigned)nt), b(256);
#define GDF_F64(TO, TF) hipLaunchKernelGGL((finalize64_kernel<TO, TF>), g, b, 0, s, (const TO *)go, (TF *)f, io, n, nt, u64, st, levs)
    if (out_dtype == 2) {
        if (go_dtype == 0) GDF_F64(uint8_t, double); else if (go_dtype == 1) GDF_F64(float, double); else GDF_F64(double, double);
    } else {
        if (go_dtype == 0) GDF_F64(uint8_t, float); else if (go_dtype == 1) GDF_F64(float, float); else GDF_F64(double, float);
    }
#undef GDF_F64
    return hipGetLastError();
}

}  // namespace gdf
