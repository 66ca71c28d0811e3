// Per-pixel kernels around the multigrid solve of Eq. (1): right-hand side
// formation, output formation with the FP64 residual of the returned f, the
// adjoint assembly, the FP64 refinement step of the mixed-precision solve,
// and the fixed-order per-slice reductions.
//
// All of them walk 64 x 16 pixel tiles with 256 threads; each thread handles
// four consecutive pixels of one tile row (vector loads and stores), so rows
// are read coalesced; horizontal stencil neighbours come from the adjacent
// threads by DPP row shifts, vertical ones from the adjacent rows (L2 hits).
// Partial sums are reduced per tile in FP64 and written to a per-tile slot; a
// second kernel sums each slice's slots in a fixed order.
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

// Sum over a 256-thread block in a fixed order (butterfly within each wave,
// then the four wave sums in order), so results do not depend on scheduling.
__device__ double block_sum(double v, double *red)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return r;
}

// ---- quad mapping: thread t of a tile handles the four pixels x .. x + 3 of
// one row, x = tile_x0 + 4 (t & 15), y = ty0 + (t >> 4).  The 16 threads of a
// tile row form one DPP row, so horizontal neighbours across threads come from
// row shifts; the tile's two outer neighbours are loaded.

template <typename T> struct Vec4 { typedef T type __attribute__((ext_vector_type(4))); };

// p[i .. i + 3] as doubles; elements at or past nvalid read as 0
template <typename TV>
__device__ __forceinline__ void load4(const TV *p, long long i, int nvalid, double v[4])
{
    using V = typename Vec4<TV>::type;
    if (nvalid >= 4 && (reinterpret_cast<uintptr_t>(p + i) & (sizeof(V) - 1)) == 0) {
        const V q = *reinterpret_cast<const V *>(p + i);
        v[0] = (double)q.x;
        v[1] = (double)q.y;
        v[2] = (double)q.z;
        v[3] = (double)q.w;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = k < nvalid ? (double)p[i + k] : 0.0;
    }
}

template <typename T> struct Vec2 { typedef T type __attribute__((ext_vector_type(2))); };

// Level-0 iterates store each row by colour (see LevelDesc): pixel (x, y) at
// element x / 2 of the half (x + y) & 1 of row y, the halves pitch / 2 long.
template <typename S> struct RBView {
    const S *u;
    long long pitch, half;
    __device__ RBView(const S *u_, long long pitch_) : u(u_), pitch(pitch_), half(pitch_ >> 1) {}
    __device__ double at(int x, int y) const
    {
        return (double)u[(long long)y * pitch + ((x + y) & 1) * half + (x >> 1)];
    }
    // pixels x .. x + 3 of row y (x a multiple of 4); past nvalid: 0
    __device__ void quad(int x, int y, int nvalid, double v[4]) const
    {
        using V2 = typename Vec2<S>::type;
        if (nvalid <= 0) {
            v[0] = v[1] = v[2] = v[3] = 0.0;
            return;
        }
        const S *r0 = u + (long long)y * pitch + (x >> 1), *r1 = r0 + half;
        const S *re = (y & 1) ? r1 : r0, *ro = (y & 1) ? r0 : r1;   // colours of pixels x and x + 1
        if (nvalid >= 4) {
            const V2 a = *reinterpret_cast<const V2 *>(re), b = *reinterpret_cast<const V2 *>(ro);
            v[0] = (double)a.x;
            v[1] = (double)b.x;
            v[2] = (double)a.y;
            v[3] = (double)b.y;
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = k < nvalid ? (double)((k & 1) ? ro : re)[k >> 1] : 0.0;
        }
    }
};
// A row-major array (the FP64 iterates of the mixed scheme), same interface.
template <typename S> struct RowView {
    const S *u;
    long long pitch;
    __device__ RowView(const S *u_, long long pitch_) : u(u_), pitch(pitch_) {}
    __device__ double at(int x, int y) const { return (double)u[(long long)y * pitch + x]; }
    __device__ void quad(int x, int y, int nvalid, double v[4]) const { load4(u, (long long)y * pitch + x, nvalid, v); }
};

template <typename TV>
__device__ __forceinline__ void store4(TV *p, long long i, int nvalid, const double v[4])
{
    using V = typename Vec4<TV>::type;
    if (nvalid >= 4 && (reinterpret_cast<uintptr_t>(p + i) & (sizeof(V) - 1)) == 0) {
        V q;
        q.x = (TV)v[0];
        q.y = (TV)v[1];
        q.z = (TV)v[2];
        q.w = (TV)v[3];
        *reinterpret_cast<V *>(p + i) = q;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < nvalid) p[i + k] = (TV)v[k];
    }
}

// value of the previous / next thread in the 16-lane DPP row (0 at the row ends)
__device__ __forceinline__ double row_prev(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x111, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x111, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double row_next(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x101, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x101, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

struct QuadCtx {
    long long tile;         // logical tile index (also the slot of its partial sums)
    int si, x, y, nvalid;   // nvalid: pixels of the quad inside the row (<= 0: none)
    bool row_in;
    SliceIO P;
};

__device__ __forceinline__ bool quad_ctx(const SliceIO *io, int n, long long n_tiles, QuadCtx &c)
{
    const long long tile = xcd_tile(blockIdx.x, gridDim.x);
    c.tile = tile;
    if (tile >= n_tiles) return false;
    c.si = find_slice(io, n, tile);
    c.P = io[c.si];
    const long long lt = tile - c.P.tile_begin;
    c.x = (int)(lt % c.P.tiles_x) * 64 + 4 * (threadIdx.x & 15);
    c.y = (int)(lt / c.P.tiles_x) * 16 + (threadIdx.x >> 4);
    c.nvalid = min(4, c.P.W - c.x);
    c.row_in = c.y < c.P.H && c.nvalid > 0;
    return true;
}

// ------------------------------------------------------------- finish ---

// One block per slice; fixed-order strided sum then a fixed tree, so the
// result does not depend on scheduling.
__global__ __launch_bounds__(256) void finish_kernel(int n_slices, const int *range,
                                                     const float2 *pf, const double *pd, const double *pd2,
                                                     int mode, double tol, int max_cycles, int count_cycle,
                                                     double stall_ratio, SliceState *st, int *active)
{
    __shared__ double red[4];
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
            if (pd2) w += pd2[i];
        }
    }
    const bool has_r = pf || pd2;   // (uniform)
    const double sum = block_sum(v, red);
    const double rsum = has_r ? block_sum(w, red) : 0.0;
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
        S.shift = has_r ? rsum / (S.npx * S.alpha) : 0.0;
        if (!isfinite(sum)) S.status = 6;
        if (!isfinite(sum) || S.rel <= tol || S.cycles >= max_cycles) active[sidx] = 0;
        break;
    }
}

// The three sums after right-hand-side formation in one launch: ||b||^2,
// rel_init = sqrt(||b_u||^2 / ||b||^2), and the mean of b_u (bmean, uoff).
__global__ __launch_bounds__(256) void finish_rhs_kernel(int n_slices, const int *range, const double *pbb,
                                                         const double *pb0, const double *pbs, SliceState *st)
{
    __shared__ double red[4];
    const int sidx = blockIdx.x;
    if (sidx >= n_slices) return;
    const int b0 = range[2 * sidx], b1 = range[2 * sidx + 1];
    double v = 0.0, w = 0.0, x = 0.0;
    for (int i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
        v += pbb[i];
        w += pb0[i];
        x += pbs[i];
    }
    const double sbb = block_sum(v, red), sb0 = block_sum(w, red), sbs = block_sum(x, red);
    if (threadIdx.x != 0) return;
    SliceState &S = st[sidx];
    S.bb = sbb;
    S.rel_init = sbb > 0.0 ? sqrt(sb0 / sbb) : sqrt(sb0);
    S.bmean = sbs / S.npx;
    S.uoff = S.bmean / S.alpha;
}

hipError_t launch_finish_rhs(int n_slices, const int *range, const double *pbb, const double *pb0,
                             const double *pbs, SliceState *state, hipStream_t s)
{
    if (n_slices <= 0) return hipSuccess;
    hipLaunchKernelGGL(finish_rhs_kernel, dim3(n_slices), dim3(256), 0, s, n_slices, range, pbb, pb0, pbs, state);
    return hipGetLastError();
}

hipError_t launch_finish(int n_slices, const int *range, const float2 *partials_f,
                         const double *partials_d, const double *partials_d2, int mode, double tol,
                         int max_cycles, int count_cycle, double stall_ratio, SliceState *state, int *active,
                         hipStream_t s)
{
    if (n_slices <= 0) return hipSuccess;
    hipLaunchKernelGGL(finish_kernel, dim3(n_slices), dim3(256), 0, s, n_slices, range, partials_f,
                       partials_d, partials_d2, mode, tol, max_cycles, count_cycle, stall_ratio, state, active);
    return hipGetLastError();
}

__global__ __launch_bounds__(64) void sum_aux_kernel(int n_slices, const SliceState *st, double *dst)
{
    if (threadIdx.x != 0) return;
    double v = 0.0;
    for (int i = 0; i < n_slices; ++i) v += st[i].aux;   // fixed order
    *dst = v;
}

hipError_t launch_sum_aux(int n_slices, const SliceState *state, double *dst, hipStream_t s)
{
    hipLaunchKernelGGL(sum_aux_kernel, dim3(1), dim3(64), 0, s, n_slices, state, dst);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void done_kernel(int n_slices, const int *active, int *done)
{
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    int a = 0;
    for (int i = threadIdx.x; i < n_slices; i += blockDim.x) a |= active[i];
    if (a) any = 1;   // benign race: every writer stores 1
    __syncthreads();
    if (threadIdx.x == 0) *done = any ? 0 : 1;
}

hipError_t launch_done(int n_slices, const int *active, int *done, hipStream_t s)
{
    hipLaunchKernelGGL(done_kernel, dim3(1), dim3(256), 0, s, n_slices, active, done);
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

// b_u = alpha (g_s - g_o) and partial sums of ||alpha g_s + L g_o||^2, ||b_u||^2
// and sum(b_u).  Quad mapping.
template <typename T, typename TS, typename TO>
__global__ __launch_bounds__(256) void prep_kernel(const TS *gs, const TO *go, const SliceIO *io,
                                                   int n_slices, long long n_tiles,
                                                   const LevelDesc *levs, double *part_bb,
                                                   double *part_b0, double *part_bs)
{
    __shared__ double red[4];
    QuadCtx c;
    if (!quad_ctx(io, n_slices, n_tiles, c)) return;
    const SliceIO &P = c.P;
    const LevelDesc &L = levs[P.lev0];
    const int x = c.x, y = c.y, nv = c.row_in ? c.nvalid : 0;
    const double al = P.alpha;
    const long long go_row = P.off_go + (long long)min(y, P.H - 1) * P.pitch_go;
    double o[4], on[4], os[4], sv[4];
    load4(go, go_row + x, nv, o);
    load4(go, go_row - P.pitch_go + x, (y > 0) ? nv : 0, on);
    load4(go, go_row + P.pitch_go + x, (y < P.H - 1) ? nv : 0, os);
    load4(gs, P.off_gs + (long long)min(y, P.H - 1) * P.pitch_gs + x, nv, sv);
    double ol = row_prev(o[3]), orr = row_next(o[0]);
    const int g = threadIdx.x & 15;
    if (nv > 0 && g == 0 && x > 0) ol = (double)go[go_row + x - 1];
    if (nv > 0 && g == 15 && x + nv < P.W) orr = (double)go[go_row + x + nv];
    double sbb = 0.0, sb0 = 0.0, sbs = 0.0, bq[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double l = k == 0 ? ol : o[k - 1], r = k == 3 ? orr : o[k + 1];
        double lap = 0.0;   // (L g_o)_p over in-slice neighbours
        if (x + k > 0) lap += o[k] - l;
        if (x + k < P.W - 1) lap += o[k] - r;
        if (y > 0) lap += o[k] - on[k];
        if (y < P.H - 1) lap += o[k] - os[k];
        const double bf = al * sv[k] + lap;
        const T bu = (T)(al * (sv[k] - o[k]));
        bq[k] = (double)bu;
        if (k < nv) {
            sbb += bf * bf;
            sb0 += (double)bu * (double)bu;
            sbs += (double)bu;
        }
    }
    store4(static_cast<T *>(L.b), (long long)min(y, P.H - 1) * L.pitch + x, nv, bq);
    const double tbb = block_sum(sbb, red);
    const double tb0 = block_sum(sb0, red);
    const double tbs = block_sum(sbs, red);
    if (threadIdx.x == 0) {
        part_bb[c.tile] = tbb;
        part_b0[c.tile] = tb0;
        part_bs[c.tile] = tbs;
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
// unrounded g_o + u (A(g_o + u) - (alpha g_s + L g_o) = A u - b_u).  Quad
// mapping: one tile row of four-pixel vectors per thread.
template <typename T, typename TO, typename TF>
__global__ __launch_bounds__(256) void finalize_quad_kernel(const TO *go, TF *f, const SliceIO *io,
                                                       int n_slices, long long n_tiles,
                                                       const LevelDesc *levs,
                                                       const SliceState *st, const int *only,
                                                       double *part_rr)
{
    __shared__ double red[4];
    QuadCtx c;
    if (!quad_ctx(io, n_slices, n_tiles, c)) return;
    if (only && !only[c.si]) return;   // uniform per block: keeps this slice's partial sum
    const SliceIO &P = c.P;
    const LevelDesc &L = levs[P.lev0];
    const int x = c.x, y = c.y, nv = c.row_in ? c.nvalid : 0;
    const double sg = P.alpha;
    const RBView<T> u(static_cast<const T *>(L.u[st[c.si].cycles & 1]), L.pitch);
    const T *bu = static_cast<const T *>(L.b);
    // full correction = uoff (mean removed on load) + u + shift (constant-mode
    // correction); constants cancel in L, and b is used as stored
    const double shift = st[c.si].shift + st[c.si].uoff;
    const long long pu = L.pitch;
    const int yc = min(y, P.H - 1);   // clamped row: loads stay in the slice
    const long long p = (long long)yc * pu + x;
    double uc[4], un[4], us[4], bb[4];
    u.quad(x, yc, nv, uc);
    load4(bu, p, nv, bb);
    u.quad(x, yc - 1, (y > 0) ? nv : 0, un);
    u.quad(x, yc + 1, (y < P.H - 1) ? nv : 0, us);
    // horizontal neighbours of the quad's first and last pixel
    double ul = row_prev(uc[3]), ur = row_next(uc[0]);
    const int g = threadIdx.x & 15;
    if (nv > 0 && g == 0 && x > 0) ul = u.at(x - 1, yc);
    if (nv > 0 && (g == 15 || nv < 4) && x + nv < P.W) ur = u.at(x + nv, yc);
    double srr = 0.0, o[4], fo[4];
    load4(go, P.off_go + (long long)y * P.pitch_go + x, nv, o);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double l = k == 0 ? ul : uc[k - 1], r = k == 3 ? ur : uc[k + 1];
        double acc = 0.0;
        if (x + k > 0) acc += uc[k] - l;
        if (x + k < P.W - 1) acc += uc[k] - r;
        if (y > 0) acc += uc[k] - un[k];
        if (y < P.H - 1) acc += uc[k] - us[k];
        const double res = bb[k] - sg * (uc[k] + shift) - acc;
        if (k < nv) srr += res * res;
        fo[k] = o[k] + (uc[k] + shift);
    }
    store4(f, P.off_f + (long long)y * P.pitch_f + x, nv, fo);
    const double t = block_sum(srr, red);
    if (threadIdx.x == 0) part_rr[c.tile] = t;
}

// Row-marching output pass (the common case: widths are multiples of four
// and the g_o and f rows start on four-element boundaries).  One wave owns a block of kFinCols columns (four
// per lane) by kFinRows rows and walks down it holding the iterate's rows
// y - 1, y, y + 1, so every row is read once; the loads of the next rows are
// in flight kFinQ - 1 rows ahead.  The wave's two outer horizontal neighbours
// come from one extra element per row; the others cross lanes by DPP.
constexpr int kFinQ = 4;   // rows of loads in flight

__device__ __forceinline__ int find_fslice(const SliceIO *io, int n, long long t)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (io[mid].ftile_begin <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// lane i receives lane i - 1's / i + 1's value (0 at the wave's ends)
__device__ __forceinline__ double wave_prev(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x138, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double wave_next(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x130, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename V> __device__ __forceinline__ void v4_to_d(const V &q, double v[4])
{
    v[0] = (double)q.x;
    v[1] = (double)q.y;
    v[2] = (double)q.z;
    v[3] = (double)q.w;
}

#define GDF_GLOBAL __attribute__((address_space(1)))

template <typename T, typename TO, typename TF>
__global__ __launch_bounds__(64) void finalize_kernel(const TO *go_, TF *f_, const SliceIO *io, int n_slices,
                                                      long long n_ft, const LevelDesc *levs,
                                                      const SliceState *st, const int *only, double *part_rr)
{
    using VT = typename Vec4<T>::type;
    using VO = typename Vec4<TO>::type;
    using VF = typename Vec4<TF>::type;
    constexpr int Q = kFinQ;
    const long long ft = xcd_tile(blockIdx.x, gridDim.x);
    if (ft >= n_ft) return;
    const int si = find_fslice(io, n_slices, ft);
    if (only && !only[si]) return;   // uniform per wave: keeps this slice's partial sum
    // the slice's fields as wave-uniform scalars (stores to f cannot alias them)
    const int H = __builtin_amdgcn_readfirstlane(io[si].H), W = __builtin_amdgcn_readfirstlane(io[si].W);
    const int ftx = __builtin_amdgcn_readfirstlane(io[si].ftiles_x);
    const long long lt = ft - io[si].ftile_begin;
    const long long off_go = io[si].off_go, pitch_go = io[si].pitch_go;
    const long long off_f = io[si].off_f, pitch_f = io[si].pitch_f;
    const double sg = io[si].alpha;
    const LevelDesc &L = levs[io[si].lev0];
    const long long pu = L.pitch;
    const GDF_GLOBAL T *u = (const GDF_GLOBAL T *)L.u[st[si].cycles & 1];
    const GDF_GLOBAL T *bu = (const GDF_GLOBAL T *)L.b;
    const GDF_GLOBAL TO *go = (const GDF_GLOBAL TO *)go_;
    GDF_GLOBAL TF *f = (GDF_GLOBAL TF *)f_;
    // full correction = uoff (mean removed on load) + u + shift (constant-mode
    // correction); constants cancel in L, and b is used as stored
    const double shift = st[si].shift + st[si].uoff;

    const int lane = threadIdx.x;
    const int X0 = (int)(lt % ftx) * kFinCols, Y0 = (int)(lt / ftx) * kFinRows;
    const int Y1 = min(Y0 + kFinRows, H);
    const int x = X0 + 4 * lane;
    const bool in = x < W;          // the lane's quad lies in the slice (W is a multiple of 4)
    const int xl = min(x, W - 4);   // a valid quad for every lane
    // the wave's outer neighbour columns (lane 0: left, lane 63: right), clamped
    const int xe = min(max(lane == 0 ? X0 - 1 : X0 + kFinCols, 0), W - 1);
    // horizontal neighbour masks of the quad's first and last pixel
    const double ml = x > 0 ? 1.0 : 0.0, mr = x + 3 < W - 1 ? 1.0 : 0.0;
    // The iterate stores each row by colour (LevelDesc): pixel (x, y) at
    // element x / 2 of the half (x + y) & 1 of row y (halves pu / 2 long).  A
    // lane's quad (xl a multiple of 4) is two pairs: pixels xl, xl + 2 of one
    // colour and xl + 1, xl + 3 of the other.  Rows are clamped into the slice;
    // arena rows are multiples of 64 elements, so a pair never leaves its half.
    using VT2 = typename Vec2<T>::type;
    const long long pu2 = pu >> 1;
    auto uat = [&](int x, int y) -> T {
        const int yc = min(max(y, 0), H - 1);
        return u[(long long)yc * pu + ((x + yc) & 1) * pu2 + (x >> 1)];
    };
    auto uquad = [&](int y, VT2 &ev, VT2 &od) {   // the colours of pixels xl (ev) and xl + 1 (od)
        const int yc = min(max(y, 0), H - 1);
        const GDF_GLOBAL T *r0 = u + (long long)yc * pu + (xl >> 1);
        ev = *reinterpret_cast<const GDF_GLOBAL VT2 *>((yc & 1) ? r0 + pu2 : r0);
        od = *reinterpret_cast<const GDF_GLOBAL VT2 *>((yc & 1) ? r0 : r0 + pu2);
    };
    auto quad_d = [](const VT2 &ev, const VT2 &od, double v[4]) {
        v[0] = (double)ev.x;
        v[1] = (double)od.x;
        v[2] = (double)ev.y;
        v[3] = (double)od.y;
    };

    double un[4], uc[4], us[4];
    {
        VT2 ev, od;
        uquad(Y0 - 1, ev, od);   // (row -1: masked below)
        quad_d(ev, od, un);
        uquad(Y0, ev, od);
        quad_d(ev, od, uc);
    }
    double ue = (double)uat(xe, Y0);

    // queue: u of row y + 1 (and its outer element), b and g_o of row y; past
    // the block's last row the queue re-reads that row (cache hits, unused)
    VT2 qev[Q], qod[Q];
    VT qb[Q];
    VO qo[Q];
    T qe[Q];
    auto issue = [&](int t, int slot) {
        const int y = min(Y0 + t, Y1 - 1);
        uquad(y + 1, qev[slot], qod[slot]);
        qe[slot] = uat(xe, y + 1);
        qb[slot] = *reinterpret_cast<const GDF_GLOBAL VT *>(bu + (long long)y * pu + xl);
        qo[slot] = *reinterpret_cast<const GDF_GLOBAL VO *>(go + off_go + (long long)y * pitch_go + xl);
    };
#pragma unroll
    for (int q = 0; q < Q - 1; ++q) issue(q, q);
    // one full wait here, so the wait at the head of the row loop (which merges
    // the entry with the back edge) stays partial
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)

    double srr = 0.0;
    const int n_rows = Y1 - Y0;
    for (int tb = 0; tb < n_rows; tb += Q) {
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const int t = tb + k;
            issue(t + Q - 1, (k + Q - 1) % Q);
            const int y = Y0 + t;
            const double mu = y > 0 ? 1.0 : 0.0, md = y < H - 1 ? 1.0 : 0.0;   // uniform
            const double wrow = (t < n_rows && in) ? 1.0 : 0.0;
            double bb[4], o[4];
            quad_d(qev[k], qod[k], us);
            v4_to_d(qb[k], bb);
            v4_to_d(qo[k], o);
            const double ue_next = (double)qe[k];
            double ul = wave_prev(uc[3]), ur = wave_next(uc[0]);
            ul = lane == 0 ? ue : ul;
            ur = lane == 63 ? ue : ur;
            VF fv;
            double rr = 0.0;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const double l = m == 0 ? ul : uc[m - 1], r = m == 3 ? ur : uc[m + 1];
                const double kl = m == 0 ? ml : 1.0, kr = m == 3 ? mr : 1.0;
                double acc = kl * (uc[m] - l);
                acc = fma(kr, uc[m] - r, acc);
                acc = fma(mu, uc[m] - un[m], acc);
                acc = fma(md, uc[m] - us[m], acc);
                const double res = bb[m] - sg * (uc[m] + shift) - acc;
                rr = fma(res, res, rr);
                fv[m] = (TF)(o[m] + (uc[m] + shift));
            }
            srr = fma(wrow, rr, srr);
            if (t < n_rows && in)
                *reinterpret_cast<GDF_GLOBAL VF *>(f + off_f + (long long)y * pitch_f + x) = fv;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                un[m] = uc[m];
                uc[m] = us[m];
            }
            ue = ue_next;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) srr += __shfl_xor(srr, off);
    if (lane == 0) part_rr[ft] = srr;
}

template <typename T, typename TO>
static hipError_t fin_go(bool rows, int out_dtype, const void *go, void *f, const SliceIO *io, int n,
                         long long nt, const LevelDesc *levs, const SliceState *st, const int *only,
                         double *prr, hipStream_t s)
{
    if (rows) {
        const dim3 g((unsigned)nt), blk(64);
        if (out_dtype == 2)
            hipLaunchKernelGGL((finalize_kernel<T, TO, double>), g, blk, 0, s, (const TO *)go, (double *)f, io, n, nt, levs, st, only, prr);
        else
            hipLaunchKernelGGL((finalize_kernel<T, TO, float>), g, blk, 0, s, (const TO *)go, (float *)f, io, n, nt, levs, st, only, prr);
    } else {
        const dim3 g((unsigned)nt), blk(256);
        if (out_dtype == 2)
            hipLaunchKernelGGL((finalize_quad_kernel<T, TO, double>), g, blk, 0, s, (const TO *)go, (double *)f, io, n, nt, levs, st, only, prr);
        else
            hipLaunchKernelGGL((finalize_quad_kernel<T, TO, float>), g, blk, 0, s, (const TO *)go, (float *)f, io, n, nt, levs, st, only, prr);
    }
    return hipGetLastError();
}

hipError_t launch_finalize(bool fp64, bool rows, int go_dtype, const void *go, int out_dtype, void *f,
                           const SliceIO *io_dev, int n, long long n_tiles,
                           const LevelDesc *levs, const SliceState *st, const int *only,
                           double *part_rr, hipStream_t s)
{
    if (n_tiles <= 0) return hipSuccess;
    if (fp64) {
        if (go_dtype == 0) return fin_go<double, uint8_t>(rows, out_dtype, go, f, io_dev, n, n_tiles, levs, st, only, part_rr, s);
        if (go_dtype == 1) return fin_go<double, float>(rows, out_dtype, go, f, io_dev, n, n_tiles, levs, st, only, part_rr, s);
        return fin_go<double, double>(rows, out_dtype, go, f, io_dev, n, n_tiles, levs, st, only, part_rr, s);
    }
    if (go_dtype == 0) return fin_go<float, uint8_t>(rows, out_dtype, go, f, io_dev, n, n_tiles, levs, st, only, part_rr, s);
    if (go_dtype == 1) return fin_go<float, float>(rows, out_dtype, go, f, io_dev, n, n_tiles, levs, st, only, part_rr, s);
    return fin_go<float, double>(rows, out_dtype, go, f, io_dev, n, n_tiles, levs, st, only, part_rr, s);
}

// ------------------------------------------------------------ adjoint ---
//
// These kernels use the quad mapping (four pixels of one tile row per thread).

template <typename T>
__global__ __launch_bounds__(256) void prep_adjoint_kernel(const T *gf, const SliceIO *io, int n,
                                                           long long n_tiles, const LevelDesc *levs,
                                                           double *part_bb, double *part_bs)
{
    __shared__ double red[4];
    QuadCtx c;
    if (!quad_ctx(io, n, n_tiles, c)) return;
    const SliceIO &P = c.P;
    const LevelDesc &L = levs[P.lev0];
    const int y = min(c.y, P.H - 1), nv = c.row_in ? c.nvalid : 0;
    double v[4];
    load4(gf, P.off_f + (long long)y * P.pitch_f + c.x, nv, v);
    store4(static_cast<T *>(L.b), (long long)y * L.pitch + c.x, nv, v);
    double sbb = 0.0, sbs = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {   // elements past nv are 0
        sbb += v[k] * v[k];
        sbs += v[k];
    }
    const double t = block_sum(sbb, red);
    const double t2 = block_sum(sbs, red);
    if (threadIdx.x == 0) {
        part_bb[c.tile] = t;
        part_bs[c.tile] = t2;
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

// The quad of level-0 values at row y and its four-neighbour sums: c (the
// quad), and sum over in-slice neighbours q of (c_k - v_q).
template <typename View>
__device__ __forceinline__ void quad_lap(const View &v, const QuadCtx &q, int nv, double c[4], double lap[4])
{
    const int x = q.x, y = min(q.y, q.P.H - 1), H = q.P.H, W = q.P.W;
    double n[4], s[4];
    v.quad(x, y, nv, c);
    v.quad(x, y - 1, y > 0 ? nv : 0, n);
    v.quad(x, y + 1, y < H - 1 ? nv : 0, s);
    double l = row_prev(c[3]), r = row_next(c[0]);
    const int g = threadIdx.x & 15;
    if (nv > 0 && g == 0 && x > 0) l = v.at(x - 1, y);
    if (nv > 0 && g == 15 && x + nv < W) r = v.at(x + nv, y);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double vl = k == 0 ? l : c[k - 1], vr = k == 3 ? r : c[k + 1];
        double acc = 0.0;
        if (x + k > 0) acc += c[k] - vl;
        if (x + k < W - 1) acc += c[k] - vr;
        if (y > 0) acc += c[k] - n[k];
        if (y < H - 1) acc += c[k] - s[k];
        lap[k] = acc;
    }
}

// lambda = A^{-1} grad_f (level-0 iterate): grad_gs = alpha lambda,
// grad_go = L lambda, partials of lambda . (g_s - f).
template <typename T, typename View>
__device__ __forceinline__ void adjoint_quad(const View &lam, double shift, const T *gs, const T *f, T *ggs,
                                             T *ggo, const QuadCtx &q, double &sda)
{
    const SliceIO &P = q.P;
    const int nv = q.row_in ? q.nvalid : 0;
    const int y = min(q.y, P.H - 1);
    double lc[4], lap[4], g[4], fv[4], og[4], oo[4];
    quad_lap(lam, q, nv, lc, lap);   // L is blind to the constant shift
    const long long fo = P.off_f + (long long)y * P.pitch_f + q.x;
    load4(gs, P.off_gs + (long long)y * P.pitch_gs + q.x, nv, g);
    load4(f, fo, nv, fv);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double l = lc[k] + shift;
        og[k] = P.alpha * l;
        oo[k] = lap[k];
        if (k < nv) sda += l * (g[k] - fv[k]);
    }
    if (ggs) store4(ggs, fo, nv, og);
    if (ggo) store4(ggo, fo, nv, oo);
}

template <typename T>
__global__ __launch_bounds__(256) void adjoint_kernel(const T *gs, const T *f, T *ggs, T *ggo,
                                                      const SliceIO *io, int n, long long n_tiles,
                                                      const LevelDesc *levs, const SliceState *st,
                                                      double *const *u64, double *part_da)
{
    __shared__ double red[4];
    QuadCtx c;
    if (!quad_ctx(io, n, n_tiles, c)) return;
    const SliceIO &P = c.P;
    const LevelDesc &L = levs[P.lev0];
    const int par = st[c.si].cycles & 1;
    double sda = 0.0;
    if (u64) {
        adjoint_quad<T>(RowView<double>(u64[par * n + c.si], L.pitch), 0.0, gs, f, ggs, ggo, c, sda);
    } else {
        const RBView<T> lam(static_cast<const T *>(L.u[par]), L.pitch);
        const double shift = st[c.si].shift + st[c.si].uoff;   // constant parts of lambda
        adjoint_quad<T>(lam, shift, gs, f, ggs, ggo, c, sda);
    }
    const double t = block_sum(sda, red);
    if (threadIdx.x == 0) part_da[c.tile] = t;
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

// u64_out = u64_in + e (e: the FP32 correction of the last inner solve; the
// first step starts from zero), then the FP64 residual of u64_out stored as
// the FP32 right-hand side of the next inner solve, and its squared norm.
template <typename TS, typename TO>
__global__ __launch_bounds__(256) void refine_kernel(RefineArgs a)
{
    __shared__ double red[4];
    QuadCtx c;
    if (!quad_ctx(a.io, a.n_slices, a.n_tiles, c)) return;
    const SliceIO &P = c.P;
    double srr = 0.0;
    if (a.active[c.si]) {   // uniform per block
        const LevelDesc &L = a.levs[P.lev0];
        const long long pl = L.pitch;
        const int x = c.x, y = min(c.y, P.H - 1), H = P.H, W = P.W;
        const int nv = c.row_in ? c.nvalid : 0;
        const double *uin = a.u64[a.in_sel * a.n_slices + c.si];
        double *uout = a.u64[(a.in_sel ^ 1) * a.n_slices + c.si];
        const RBView<float> e(static_cast<const float *>(L.u[a.e_sel]), pl);
        const long long p = (long long)y * pl + x;
        // new iterate on the quad and its four neighbour rows / columns
        double uc[4], un[4], us[4], t0[4], t1[4];
        double ul = 0.0, ur = 0.0;
        if (a.first) {
#pragma unroll
            for (int k = 0; k < 4; ++k) uc[k] = un[k] = us[k] = 0.0;
        } else {
            load4(uin, p, nv, uc);
            e.quad(x, y, nv, t0);
            load4(uin, p - pl, y > 0 ? nv : 0, un);
            e.quad(x, y - 1, y > 0 ? nv : 0, t1);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                uc[k] += t0[k];
                un[k] += t1[k];
            }
            load4(uin, p + pl, y < H - 1 ? nv : 0, us);
            e.quad(x, y + 1, y < H - 1 ? nv : 0, t1);
#pragma unroll
            for (int k = 0; k < 4; ++k) us[k] += t1[k];
        }
        ul = row_prev(uc[3]);
        ur = row_next(uc[0]);
        const int g = threadIdx.x & 15;
        if (!a.first && nv > 0 && g == 0 && x > 0) ul = uin[p - 1] + e.at(x - 1, y);
        if (!a.first && nv > 0 && g == 15 && x + nv < W) ur = uin[p + nv] + e.at(x + nv, y);
        double bv[4];
        if (a.rhs) {
            load4(static_cast<const TS *>(a.rhs), P.off_f + (long long)y * P.pitch_f + x, nv, bv);
        } else {
            double sv[4], o[4];
            load4(static_cast<const TS *>(a.gs), P.off_gs + (long long)y * P.pitch_gs + x, nv, sv);
            load4(static_cast<const TO *>(a.go), P.off_go + (long long)y * P.pitch_go + x, nv, o);
#pragma unroll
            for (int k = 0; k < 4; ++k) bv[k] = P.alpha * (sv[k] - o[k]);
        }
        double res[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double vl = k == 0 ? ul : uc[k - 1], vr = k == 3 ? ur : uc[k + 1];
            double acc = 0.0;
            if (x + k > 0) acc += uc[k] - vl;
            if (x + k < W - 1) acc += uc[k] - vr;
            if (y > 0) acc += uc[k] - un[k];
            if (y < H - 1) acc += uc[k] - us[k];
            res[k] = bv[k] - P.alpha * uc[k] - acc;
            if (k < nv) srr += res[k] * res[k];
        }
        store4(uout, p, nv, uc);
        store4(static_cast<float *>(L.b), p, nv, res);
    }
    const double t = block_sum(srr, red);
    if (threadIdx.x == 0) a.part_rr[c.tile] = t;
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
    QuadCtx c;
    if (!quad_ctx(io, n, n_tiles, c)) return;
    const SliceIO &P = c.P;
    const double *u = u64[(st[c.si].cycles & 1) * n + c.si];   // latest FP64 iterate
    const long long pl = levs[P.lev0].pitch;
    const int y = min(c.y, P.H - 1), nv = c.row_in ? c.nvalid : 0;
    double o[4], uv[4];
    load4(go, P.off_go + (long long)y * P.pitch_go + c.x, nv, o);
    load4(u, (long long)y * pl + c.x, nv, uv);
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] += uv[k];
    store4(f, P.off_f + (long long)y * P.pitch_f + c.x, nv, o);
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
