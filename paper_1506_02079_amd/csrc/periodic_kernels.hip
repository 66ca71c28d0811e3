// Kernels of the per-slice screened-Poisson solve of Eq. (1) with periodic
// (wrap-around) boundaries: the paper's own Fourier basis (Section III-B,
// frequency-space interpretation), where the grid Laplacian couples the
// first and last row and column of a slice.
//
// The levels are those of the Neumann hierarchy (ceil-halving, sigma_l =
// alpha 4^l, finite volumes with a narrower last column and row when a side
// is odd).  On the torus a cell's neighbours are taken modulo the side, and
// the coupling across a face is 2 / (width left + width right), so the faces
// on either side of the narrower last cell carry 2 / (1 + wL).  A side of one
// cell has no couplings (its neighbour is itself); a side of two cells couples
// the two cells across both faces, as the pixel graph of a two-pixel ring
// does.  Red-black Gauss-Seidel runs one launch per half-sweep, reading one
// buffer and writing the other; where an odd side brings two cells of one
// colour together across the wrap, each reads the other's previous value.
// The restriction sums a coarse cell's children's residuals; the
// prolongation is cell-centred bilinear with the neighbour taken across the
// wrap.  Every kernel walks kPTileW x kPTileH tiles (items) with 256 threads,
// one column each, four rows per thread; per-item partial sums are FP64.
#include "internal.h"

namespace gdf {

namespace {

// a level's arrays: T on level 0, Coarse on the others (bfloat16 for FP32
// hierarchies, as in the Neumann hierarchy)
template <typename T> struct PStor { typedef T Coarse; };
template <> struct PStor<float> { typedef unsigned short Coarse; };

template <typename S> __device__ __forceinline__ float pget(const S *p, size_t i);
template <> __device__ __forceinline__ float pget<float>(const float *p, size_t i) { return p[i]; }
template <> __device__ __forceinline__ float pget<unsigned short>(const unsigned short *p, size_t i)
{
    return __uint_as_float((unsigned)p[i] << 16);
}
__device__ __forceinline__ double pget(const double *p, size_t i) { return p[i]; }

__device__ __forceinline__ void pput(float *p, size_t i, float v) { p[i] = v; }
__device__ __forceinline__ void pput(double *p, size_t i, double v) { p[i] = v; }
__device__ __forceinline__ void pput(unsigned short *p, size_t i, float v)
{
    p[i] = __builtin_bit_cast(unsigned short, (__bf16)v);   // round to nearest even
}

// coupling across the face between cell i and cell (i + 1) mod n of a side of
// n >= 2 cells whose last cell has relative width wl
template <typename T> __device__ __forceinline__ T pface(int i, int n, T wl)
{
    return i >= n - 2 ? T(2) / (T(1) + wl) : T(1);
}

// The periodic finite-volume stencil of cell (y, x) of a level:
// (A v)_p = m v_p + wy (kl (v_p - v_l) + kr (v_p - v_r)) + wx (ku (v_p - v_u) + kd (v_p - v_d))
template <typename T> struct PSt {
    int xl, xr, yu, yd;
    T wx, wy, kl, kr, ku, kd, m, diag;
};
template <typename T> __device__ __forceinline__ PSt<T> pstencil(const LevelDesc &L, int y, int x)
{
    const int w = L.W, h = L.H;
    const T wxl = (T)L.wxL, wyl = (T)L.wyL;
    PSt<T> c;
    c.xl = x == 0 ? w - 1 : x - 1;
    c.xr = x == w - 1 ? 0 : x + 1;
    c.yu = y == 0 ? h - 1 : y - 1;
    c.yd = y == h - 1 ? 0 : y + 1;
    c.wx = x == w - 1 ? wxl : T(1);
    c.wy = y == h - 1 ? wyl : T(1);
    c.kl = w > 1 ? pface<T>(c.xl, w, wxl) : T(0);
    c.kr = w > 1 ? pface<T>(x, w, wxl) : T(0);
    c.ku = h > 1 ? pface<T>(c.yu, h, wyl) : T(0);
    c.kd = h > 1 ? pface<T>(y, h, wyl) : T(0);
    c.m = (T)L.sigma * c.wx * c.wy;
    c.diag = c.m + c.wy * (c.kl + c.kr) + c.wx * (c.ku + c.kd);
    return c;
}

// neighbour sum wy (kl v_l + kr v_r) + wx (ku v_u + kd v_d)
template <typename T, typename S>
__device__ __forceinline__ T pnbr(const PSt<T> &c, const S *v, int pitch, int y, int x)
{
    const T h = c.kl * (T)pget(v, (size_t)y * pitch + c.xl) + c.kr * (T)pget(v, (size_t)y * pitch + c.xr);
    const T u = c.ku * (T)pget(v, (size_t)c.yu * pitch + x) + c.kd * (T)pget(v, (size_t)c.yd * pitch + x);
    return c.wy * h + c.wx * u;
}

__device__ double pblock_sum(double v, double *red)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return r;
}

constexpr int kPRows = kPTileH / 4;   // rows per thread

template <typename T> __device__ __forceinline__ T level0_shift(const LevelDesc &L)
{
    return L.bshift ? (T)*L.bshift : T(0);
}

// ---------------------------------------------------------------- kernels

// One half-sweep: cells of colour a.colour take (b - shift + neighbour sum) /
// diag from buffer in_sel, the others are copied; written to buffer out_sel.
template <typename T, typename S>
__global__ __launch_bounds__(256) void psmooth_kernel(PLaunch a)
{
    if (blockIdx.x >= (unsigned)a.n_items) return;
    const PItem it = a.items[blockIdx.x];
    if (!a.active[it.slice]) return;
    const LevelDesc L = a.levs[it.lev];
    const int x = it.x0 + (threadIdx.x & 63);
    if (x >= L.W) return;   // (no barrier in this kernel)
    const S *uin = static_cast<const S *>(L.u[a.in_sel]);
    S *uout = static_cast<S *>(L.u[a.out_sel]);
    const S *b = static_cast<const S *>(L.b);
    const T bsh = level0_shift<T>(L);
#pragma unroll
    for (int i = 0; i < kPRows; ++i) {
        const int y = it.y0 + (threadIdx.x >> 6) + 4 * i;
        if (y >= L.H) break;
        const size_t p = (size_t)y * L.pitch + x;
        T v;
        if (((x + y) & 1) == a.colour) {
            const PSt<T> c = pstencil<T>(L, y, x);
            const T nb = a.zero_in ? T(0) : pnbr<T>(c, uin, L.pitch, y, x);
            v = ((T)pget(b, p) - bsh + nb) / c.diag;
        } else {
            v = a.zero_in ? T(0) : (T)pget(uin, p);
        }
        pput(uout, p, v);
    }
}

// Coarse right-hand side: each cell of the coarser level (items of that level)
// sums the residuals b - A u of its children on the finer level (buffer in_sel).
template <typename T, typename SF, typename SC>
__global__ __launch_bounds__(256) void prestrict_kernel(PLaunch a)
{
    if (blockIdx.x >= (unsigned)a.n_items) return;
    const PItem it = a.items[blockIdx.x];
    if (!a.active[it.slice]) return;
    const LevelDesc C = a.levs[it.lev];
    const LevelDesc F = a.levs[it.lev - 1];
    const int X = it.x0 + (threadIdx.x & 63);
    if (X >= C.W) return;
    const SF *u = static_cast<const SF *>(F.u[a.in_sel]);
    const SF *b = static_cast<const SF *>(F.b);
    SC *bc = static_cast<SC *>(C.b);
    const T bsh = level0_shift<T>(F);
#pragma unroll
    for (int i = 0; i < kPRows; ++i) {
        const int Y = it.y0 + (threadIdx.x >> 6) + 4 * i;
        if (Y >= C.H) break;
        T sum = T(0);
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const int y = 2 * Y + dy, x = 2 * X + dx;
                if (y >= F.H || x >= F.W) continue;
                const PSt<T> c = pstencil<T>(F, y, x);
                const T uc = (T)pget(u, (size_t)y * F.pitch + x);
                sum += (T)pget(b, (size_t)y * F.pitch + x) - bsh - (c.diag * uc - pnbr<T>(c, u, F.pitch, y, x));
            }
        pput(bc, (size_t)Y * C.pitch + X, sum);
    }
}

// Level-0 residual r = b - shift - A u (buffer in_sel) in the working
// precision: per-item sums of r^2 and r in FP64.
template <typename T>
__global__ __launch_bounds__(256) void pnorm_kernel(PLaunch a)
{
    __shared__ double red[4];
    if (blockIdx.x >= (unsigned)a.n_items) return;
    const PItem it = a.items[blockIdx.x];
    double s2 = 0.0, s1 = 0.0;
    const bool act = a.active[it.slice] != 0;   // (uniform per block)
    if (act) {
        const LevelDesc L = a.levs[it.lev];
        const int x = it.x0 + (threadIdx.x & 63);
        const T *u = static_cast<const T *>(L.u[a.in_sel]);
        const T *b = static_cast<const T *>(L.b);
        const T bsh = level0_shift<T>(L);
        if (x < L.W) {
#pragma unroll
            for (int i = 0; i < kPRows; ++i) {
                const int y = it.y0 + (threadIdx.x >> 6) + 4 * i;
                if (y >= L.H) break;
                const PSt<T> c = pstencil<T>(L, y, x);
                const T uc = u[(size_t)y * L.pitch + x];
                const T r = b[(size_t)y * L.pitch + x] - bsh - (c.diag * uc - pnbr<T>(c, u, L.pitch, y, x));
                s2 += (double)r * (double)r;
                s1 += (double)r;
            }
        }
    }
    const double t2 = pblock_sum(s2, red), t1 = pblock_sum(s1, red);
    if (threadIdx.x == 0) {
        a.part_rr[blockIdx.x] = act ? t2 : 0.0;
        a.part_r[blockIdx.x] = act ? t1 : 0.0;
    }
}

// u (buffer in_sel) += bilinear prolongation of the coarser level's iterate
// (buffer coarse_sel): weights 9/16 on the parent, 3/16 on the parent's
// neighbours towards the cell in x and in y, 1/16 on the diagonal one, the
// neighbours taken across the wrap.
template <typename T, typename SF, typename SC>
__global__ __launch_bounds__(256) void pprolong_kernel(PLaunch a)
{
    if (blockIdx.x >= (unsigned)a.n_items) return;
    const PItem it = a.items[blockIdx.x];
    if (!a.active[it.slice]) return;
    const LevelDesc F = a.levs[it.lev];
    const LevelDesc C = a.levs[it.lev + 1];
    const int x = it.x0 + (threadIdx.x & 63);
    if (x >= F.W) return;
    SF *u = static_cast<SF *>(F.u[a.in_sel]);
    const SC *e = static_cast<const SC *>(C.u[a.coarse_sel]);
    const int X = x >> 1;
    int Xn = (x & 1) ? X + 1 : X - 1;
    Xn = Xn < 0 ? C.W - 1 : (Xn >= C.W ? 0 : Xn);
#pragma unroll
    for (int i = 0; i < kPRows; ++i) {
        const int y = it.y0 + (threadIdx.x >> 6) + 4 * i;
        if (y >= F.H) break;
        const int Y = y >> 1;
        int Yn = (y & 1) ? Y + 1 : Y - 1;
        Yn = Yn < 0 ? C.H - 1 : (Yn >= C.H ? 0 : Yn);
        const T e00 = (T)pget(e, (size_t)Y * C.pitch + X), e01 = (T)pget(e, (size_t)Y * C.pitch + Xn);
        const T e10 = (T)pget(e, (size_t)Yn * C.pitch + X), e11 = (T)pget(e, (size_t)Yn * C.pitch + Xn);
        const T v = T(0.5625) * e00 + T(0.1875) * (e01 + e10) + T(0.0625) * e11;
        const size_t p = (size_t)y * F.pitch + x;
        pput(u, p, (T)pget(u, p) + v);
    }
}

template <typename V> __device__ __forceinline__ double ldd(const V *p, long long i) { return (double)p[i]; }

// (L v)_p with the periodic pixel graph (level 0: unit couplings; a side of
// one pixel has none, a side of two couples across both faces)
template <typename V>
__device__ __forceinline__ double plap(const V *v, long long off, long long pitch, int H, int W, int y, int x)
{
    const double c = ldd(v, off + (long long)y * pitch + x);
    double s = 0.0;
    if (W > 1) {
        const int xl = x == 0 ? W - 1 : x - 1, xr = x == W - 1 ? 0 : x + 1;
        s += (c - ldd(v, off + (long long)y * pitch + xl)) + (c - ldd(v, off + (long long)y * pitch + xr));
    }
    if (H > 1) {
        const int yu = y == 0 ? H - 1 : y - 1, yd = y == H - 1 ? 0 : y + 1;
        s += (c - ldd(v, off + (long long)yu * pitch + x)) + (c - ldd(v, off + (long long)yd * pitch + x));
    }
    return s;
}

// b_u = alpha (g_s - g_o) into level-0 b, partials of ||alpha g_s + L g_o||^2,
// ||b_u||^2 and sum(b_u).  With gs null, g_s is taken as b_u / alpha + g_o from
// the b_u already in level-0 b (written by the smoothing), which is then kept.
template <typename T, typename TS, typename TO>
__global__ __launch_bounds__(256) void pprep_kernel(const TS *gs, const TO *go, const SliceIO *io, PLaunch a,
                                                    double *pbb, double *pb0, double *pbs)
{
    __shared__ double red[4];
    if (blockIdx.x >= (unsigned)a.n_items) return;
    const PItem it = a.items[blockIdx.x];
    const SliceIO P = io[it.slice];
    const LevelDesc L = a.levs[it.lev];
    T *b = static_cast<T *>(L.b);
    const int x = it.x0 + (threadIdx.x & 63);
    double sbb = 0.0, sb0 = 0.0, sbs = 0.0;
    if (x < P.W) {
#pragma unroll
        for (int i = 0; i < kPRows; ++i) {
            const int y = it.y0 + (threadIdx.x >> 6) + 4 * i;
            if (y >= P.H) break;
            const double o = ldd(go, P.off_go + (long long)y * P.pitch_go + x);
            const size_t pb = (size_t)y * L.pitch + x;
            T bu;
            double bf;
            if (gs) {
                const double sv = ldd(gs, P.off_gs + (long long)y * P.pitch_gs + x);
                bu = (T)(P.alpha * (sv - o));
                bf = P.alpha * sv + plap(go, P.off_go, P.pitch_go, P.H, P.W, y, x);
                b[pb] = bu;
            } else {
                bu = b[pb];
                bf = (double)bu + P.alpha * o + plap(go, P.off_go, P.pitch_go, P.H, P.W, y, x);
            }
            sbb += bf * bf;
            sb0 += (double)bu * (double)bu;
            sbs += (double)bu;
        }
    }
    const double t1 = pblock_sum(sbb, red), t2 = pblock_sum(sb0, red), t3 = pblock_sum(sbs, red);
    if (threadIdx.x == 0) {
        pbb[blockIdx.x] = t1;
        pb0[blockIdx.x] = t2;
        pbs[blockIdx.x] = t3;
    }
}

// f = g_o + (u + uoff + shift) and the FP64 residual b_u - A (u + uoff + shift)
// of the returned correction (constants cancel in L).
template <typename T, typename TO, typename TF>
__global__ __launch_bounds__(256) void pfinalize_kernel(const TO *go, TF *f, const SliceIO *io, PLaunch a,
                                                        const SliceState *st, const int *only)
{
    __shared__ double red[4];
    if (blockIdx.x >= (unsigned)a.n_items) return;
    const PItem it = a.items[blockIdx.x];
    if (only && !only[it.slice]) return;   // uniform per block: keeps this slice's partial sum
    const SliceIO P = io[it.slice];
    const LevelDesc L = a.levs[it.lev];
    const T *u = static_cast<const T *>(L.u[a.in_sel]);
    const T *b = static_cast<const T *>(L.b);
    const double shift = st[it.slice].shift + st[it.slice].uoff;
    const int x = it.x0 + (threadIdx.x & 63);
    double srr = 0.0;
    if (x < P.W) {
#pragma unroll
        for (int i = 0; i < kPRows; ++i) {
            const int y = it.y0 + (threadIdx.x >> 6) + 4 * i;
            if (y >= P.H) break;
            const double uc = (double)u[(size_t)y * L.pitch + x];
            const double res = (double)b[(size_t)y * L.pitch + x] - P.alpha * (uc + shift) -
                               plap(u, 0, L.pitch, P.H, P.W, y, x);
            srr += res * res;
            f[P.off_f + (long long)y * P.pitch_f + x] =
                (TF)(ldd(go, P.off_go + (long long)y * P.pitch_go + x) + (uc + shift));
        }
    }
    const double t = pblock_sum(srr, red);
    if (threadIdx.x == 0) a.part_rr[blockIdx.x] = t;
}

// Mixed refinement: u64_out = u64_in + e (e = level-0 FP32 iterate, buffer
// r.e_sel; not on the first step), r = rhs - A u64_out in FP64 with
// rhs = alpha (g_s - g_o) or r.rhs, stored as FP32 into level-0 b; ||r||^2.
template <typename TS, typename TO>
__global__ __launch_bounds__(256) void prefine_kernel(RefineArgs r, PLaunch a)
{
    __shared__ double red[4];
    if (blockIdx.x >= (unsigned)a.n_items) return;
    const PItem it = a.items[blockIdx.x];
    double srr = 0.0;
    if (r.active[it.slice]) {   // uniform per block
        const SliceIO P = r.io[it.slice];
        const LevelDesc L = a.levs[it.lev];
        const long long pl = L.pitch;
        const double *uin = r.u64[r.in_sel * r.n_slices + it.slice];
        double *uout = r.u64[(r.in_sel ^ 1) * r.n_slices + it.slice];
        const float *e = static_cast<const float *>(L.u[r.e_sel]);
        float *b = static_cast<float *>(L.b);
        const int x = it.x0 + (threadIdx.x & 63);
        auto unew = [&](int y, int xx) -> double {
            const long long q = (long long)y * pl + xx;
            return r.first ? 0.0 : uin[q] + (double)e[q];
        };
        if (x < P.W) {
#pragma unroll
            for (int i = 0; i < kPRows; ++i) {
                const int y = it.y0 + (threadIdx.x >> 6) + 4 * i;
                if (y >= P.H) break;
                const double uc = unew(y, x);
                double lap = 0.0;
                if (P.W > 1) {
                    const int xl = x == 0 ? P.W - 1 : x - 1, xr = x == P.W - 1 ? 0 : x + 1;
                    lap += (uc - unew(y, xl)) + (uc - unew(y, xr));
                }
                if (P.H > 1) {
                    const int yu = y == 0 ? P.H - 1 : y - 1, yd = y == P.H - 1 ? 0 : y + 1;
                    lap += (uc - unew(yu, x)) + (uc - unew(yd, x));
                }
                double bv;
                if (r.rhs)
                    bv = ldd(static_cast<const TS *>(r.rhs), P.off_f + (long long)y * P.pitch_f + x);
                else
                    bv = P.alpha * (ldd(static_cast<const TS *>(r.gs), P.off_gs + (long long)y * P.pitch_gs + x) -
                                    ldd(static_cast<const TO *>(r.go), P.off_go + (long long)y * P.pitch_go + x));
                const double res = bv - P.alpha * uc - lap;
                srr += res * res;
                uout[(long long)y * pl + x] = uc;
                b[(long long)y * pl + x] = (float)res;
            }
        }
    }
    const double t = pblock_sum(srr, red);
    if (threadIdx.x == 0) r.part_rr[blockIdx.x] = t;
}

// lambda = A^-1 grad_f: grad_gs = alpha lambda, grad_go = L lambda, partials
// of lambda . (g_s - f).
template <typename T, typename TL>
__global__ __launch_bounds__(256) void padjoint_kernel(const T *gs, const T *f, T *ggs, T *ggo, const SliceIO *io,
                                                       int n, PLaunch a, const SliceState *st,
                                                       double *const *u64, double *part_da)
{
    __shared__ double red[4];
    if (blockIdx.x >= (unsigned)a.n_items) return;
    const PItem it = a.items[blockIdx.x];
    const SliceIO P = io[it.slice];
    const LevelDesc L = a.levs[it.lev];
    const TL *lam = u64 ? reinterpret_cast<const TL *>(u64[(st[it.slice].cycles & 1) * n + it.slice])
                        : static_cast<const TL *>(L.u[a.in_sel]);
    const double shift = u64 ? 0.0 : st[it.slice].shift + st[it.slice].uoff;   // constant parts of lambda
    const int x = it.x0 + (threadIdx.x & 63);
    double sda = 0.0;
    if (x < P.W) {
#pragma unroll
        for (int i = 0; i < kPRows; ++i) {
            const int y = it.y0 + (threadIdx.x >> 6) + 4 * i;
            if (y >= P.H) break;
            const double l = ldd(lam, (long long)y * L.pitch + x) + shift;
            const long long fo = P.off_f + (long long)y * P.pitch_f + x;
            if (ggs) ggs[fo] = (T)(P.alpha * l);
            if (ggo) ggo[fo] = (T)plap(lam, 0, L.pitch, P.H, P.W, y, x);   // L is blind to the shift
            sda += l * (ldd(gs, P.off_gs + (long long)y * P.pitch_gs + x) - ldd(f, fo));
        }
    }
    const double t = pblock_sum(sda, red);
    if (threadIdx.x == 0) part_da[blockIdx.x] = t;
}

template <class K> hipError_t plaunch(K kernel, int n_items, hipStream_t s, const PLaunch &a)
{
    if (n_items <= 0) return hipSuccess;
    hipLaunchKernelGGL(kernel, dim3((unsigned)n_items), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace

// ------------------------------------------------------------------- launch

// level 0 of a list (items of level 0) has the arithmetic type; coarse levels
// the coarse storage; a.levs[it.lev] tells which level an item is on, so each
// list is launched with the storage of its level (fine: level 0)
hipError_t launch_psmooth_level(bool fp64, bool level0, const PLaunch &a, hipStream_t s)
{
    if (fp64) return plaunch(psmooth_kernel<double, double>, a.n_items, s, a);
    return level0 ? plaunch(psmooth_kernel<float, float>, a.n_items, s, a)
                  : plaunch(psmooth_kernel<float, unsigned short>, a.n_items, s, a);
}

hipError_t launch_prestrict_level(bool fp64, bool from_level0, const PLaunch &a, hipStream_t s)
{
    if (fp64) return plaunch(prestrict_kernel<double, double, double>, a.n_items, s, a);
    return from_level0 ? plaunch(prestrict_kernel<float, float, unsigned short>, a.n_items, s, a)
                       : plaunch(prestrict_kernel<float, unsigned short, unsigned short>, a.n_items, s, a);
}

hipError_t launch_pprolong_level(bool fp64, bool into_level0, const PLaunch &a, hipStream_t s)
{
    if (fp64) return plaunch(pprolong_kernel<double, double, double>, a.n_items, s, a);
    return into_level0 ? plaunch(pprolong_kernel<float, float, unsigned short>, a.n_items, s, a)
                       : plaunch(pprolong_kernel<float, unsigned short, unsigned short>, a.n_items, s, a);
}

hipError_t launch_pnorm(bool fp64, const PLaunch &a, hipStream_t s)
{
    return fp64 ? plaunch(pnorm_kernel<double>, a.n_items, s, a) : plaunch(pnorm_kernel<float>, a.n_items, s, a);
}

hipError_t launch_pprep(bool fp64, int gs_dtype, const void *gs, int go_dtype, const void *go, const SliceIO *io,
                        const PLaunch &a, double *pbb, double *pb0, double *pbs, hipStream_t s)
{
    if (a.n_items <= 0) return hipSuccess;
    const dim3 g((unsigned)a.n_items), blk(256);
#define GDF_PP(T, TS, TO)                                                                                       \
    hipLaunchKernelGGL((pprep_kernel<T, TS, TO>), g, blk, 0, s, (const TS *)gs, (const TO *)go, io, a, pbb, pb0, pbs)
#define GDF_PPO(T, TS)                                   \
    do {                                                 \
        if (go_dtype == GDF_DT_U8) GDF_PP(T, TS, uint8_t); \
        else if (go_dtype == GDF_DT_F32) GDF_PP(T, TS, float); \
        else GDF_PP(T, TS, double);                      \
    } while (0)
    if (fp64) {
        if (gs_dtype == GDF_DT_F64) GDF_PPO(double, double); else GDF_PPO(double, float);
    } else {
        if (gs_dtype == GDF_DT_F64) GDF_PPO(float, double); else GDF_PPO(float, float);
    }
#undef GDF_PPO
#undef GDF_PP
    return hipGetLastError();
}

hipError_t launch_pfinalize(bool fp64, int go_dtype, const void *go, int out_dtype, void *f, const SliceIO *io,
                            const PLaunch &a, const SliceState *st, const int *only, hipStream_t s)
{
    if (a.n_items <= 0) return hipSuccess;
    const dim3 g((unsigned)a.n_items), blk(256);
#define GDF_PF(T, TO, TF) hipLaunchKernelGGL((pfinalize_kernel<T, TO, TF>), g, blk, 0, s, (const TO *)go, (TF *)f, io, a, st, only)
#define GDF_PFO(T, TF)                                   \
    do {                                                 \
        if (go_dtype == GDF_DT_U8) GDF_PF(T, uint8_t, TF); \
        else if (go_dtype == GDF_DT_F32) GDF_PF(T, float, TF); \
        else GDF_PF(T, double, TF);                      \
    } while (0)
    if (fp64) {
        if (out_dtype == GDF_DT_F64) GDF_PFO(double, double); else GDF_PFO(double, float);
    } else {
        if (out_dtype == GDF_DT_F64) GDF_PFO(float, double); else GDF_PFO(float, float);
    }
#undef GDF_PFO
#undef GDF_PF
    return hipGetLastError();
}

hipError_t launch_prefine(const RefineArgs &r, const PLaunch &a, hipStream_t s)
{
    if (a.n_items <= 0) return hipSuccess;
    const dim3 g((unsigned)a.n_items), blk(256);
    const bool s64 = r.gs_dtype == GDF_DT_F64;
    switch (r.go_dtype) {
    case GDF_DT_U8:
        if (s64) hipLaunchKernelGGL((prefine_kernel<double, uint8_t>), g, blk, 0, s, r, a);
        else hipLaunchKernelGGL((prefine_kernel<float, uint8_t>), g, blk, 0, s, r, a);
        break;
    case GDF_DT_F32:
        if (s64) hipLaunchKernelGGL((prefine_kernel<double, float>), g, blk, 0, s, r, a);
        else hipLaunchKernelGGL((prefine_kernel<float, float>), g, blk, 0, s, r, a);
        break;
    default:
        if (s64) hipLaunchKernelGGL((prefine_kernel<double, double>), g, blk, 0, s, r, a);
        else hipLaunchKernelGGL((prefine_kernel<float, double>), g, blk, 0, s, r, a);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_padjoint(bool fp64, const void *gs, const void *f, void *ggs, void *ggo, const SliceIO *io, int n,
                           const PLaunch &a, const SliceState *st, double *const *u64, double *part_da,
                           hipStream_t s)
{
    if (a.n_items <= 0) return hipSuccess;
    const dim3 g((unsigned)a.n_items), blk(256);
    if (fp64)
        hipLaunchKernelGGL((padjoint_kernel<double, double>), g, blk, 0, s, (const double *)gs, (const double *)f,
                           (double *)ggs, (double *)ggo, io, n, a, st, u64, part_da);
    else if (u64)
        hipLaunchKernelGGL((padjoint_kernel<float, double>), g, blk, 0, s, (const float *)gs, (const float *)f,
                           (float *)ggs, (float *)ggo, io, n, a, st, u64, part_da);
    else
        hipLaunchKernelGGL((padjoint_kernel<float, float>), g, blk, 0, s, (const float *)gs, (const float *)f,
                           (float *)ggs, (float *)ggo, io, n, a, st, u64, part_da);
    return hipGetLastError();
}

}  // namespace gdf
