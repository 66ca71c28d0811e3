// Multigrid kernels for the per-slice screened-Poisson solve of Eq. (1),
//     (alpha I + L) f = alpha g_s + L g_o,
// solved in correction form u = f - g_o:  (alpha I + L) u = alpha (g_s - g_o).
//
// Level l of a slice is a finite-volume discretisation of the same operator on
// cells of side h = 2^l (cell-centred coarsening by ceil-halving), written per
// cell area h^2: a full cell reads sigma_l e + sum_q (e - e_q) = rhs with
// sigma_l = alpha h^2 and unit couplings.  When a side is odd the last coarse
// column/row is narrower; there the mass term scales with the cell's area and
// each coupling is face length / centre distance, so the coarse problem covers
// exactly the fine domain.  The right-hand side of a coarse cell is the plain
// sum of its children's residuals (area-integrated).  Prolongation is
// cell-centred bilinear interpolation (weights 9/16, 3/16, 3/16, 1/16) with
// mirrored coarse values at the slice edges.  The smoother is red-black
// Gauss-Seidel; cell (y, x) is red when x + y is even.  Level 0 (unit cells)
// runs a specialised update with unit coefficients.
//
// The strip kernel is the hot path.  One wavefront owns a strip of 128
// columns (two adjacent columns per lane) and marches down its rows, keeping a
// ring of rows in registers.  Successive half-sweeps are skewed by two rows
// (stage s processes the row loaded 2s steps earlier), which is exactly the
// schedule under which each red/black update sees its neighbours at the
// previous half-sweep, so several sweeps plus the residual happen in a single
// pass over HBM.  Horizontal neighbours across lanes come from DPP wave
// shifts; there is no LDS traffic and no barrier.  The strip reads a halo of
// G columns and G rows on each side and recomputes it redundantly.
#include "internal.h"

#include <atomic>
#include <type_traits>

namespace gdf {

// ------------------------------------------------------------------ DPP ---

// lane i receives lane i-1's value (lane 0 receives 0)
__device__ __forceinline__ float wave_shr1(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}
// lane i receives lane i+1's value (lane 63 receives 0)
__device__ __forceinline__ float wave_shl1(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ double wave_shr1(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x138, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double wave_shl1(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x130, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Values every lane of the wave holds alike, moved into scalar registers (the
// work item and level descriptor are read with vector loads, so the compiler
// cannot tell they are uniform; scalar copies keep the address arithmetic on
// the scalar unit and allow scalar-base loads).
template <typename P> __device__ __forceinline__ P *uniform_ptr(P *p)
{
    const unsigned long long v = reinterpret_cast<unsigned long long>(p);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return reinterpret_cast<P *>(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ double uniform_d(double d)
{
    const unsigned long long v = (unsigned long long)__double_as_longlong(d);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ Item uniform_item(const Item &i)
{
    return Item{uniform(i.lev), uniform(i.x0), uniform(i.y0), uniform(i.y1), uniform(i.pidx)};
}
__device__ __forceinline__ LevelDesc uniform_level(const LevelDesc &d)
{
    LevelDesc r;
    r.u[0] = uniform_ptr(d.u[0]);
    r.u[1] = uniform_ptr(d.u[1]);
    r.b = uniform_ptr(d.b);
    r.ec = uniform_ptr(d.ec);
    r.bc = uniform_ptr(d.bc);
    r.H = uniform(d.H);
    r.W = uniform(d.W);
    r.pitch = uniform(d.pitch);
    r.Hc = uniform(d.Hc);
    r.Wc = uniform(d.Wc);
    r.pitch_c = uniform(d.pitch_c);
    r.sigma = uniform_d(d.sigma);
    r.wxL = uniform_d(d.wxL);
    r.wyL = uniform_d(d.wyL);
    r.bshift = uniform_ptr(d.bshift);
    r.slice = uniform(d.slice);
    r.pad_ = 0;
    r.bshift_fine = uniform_ptr(d.bshift_fine);
    return r;
}

// Storage of a level's arrays: the arithmetic type itself, or bfloat16 (raw
// 16-bit patterns, `unsigned short`) on the coarse levels of an FP32
// hierarchy.  Coarse levels only carry corrections, whose relative accuracy
// (2^-8 here) stays far below the cycle's convergence factor, so the cycle
// converges as with FP32 coarse levels while moving half the bytes there.
// Pair: two adjacent elements as one memory access.
template <typename S> struct Stor;
template <> struct Stor<float> {
    typedef float Pair __attribute__((ext_vector_type(2)));
    __device__ static float lo(Pair p) { return p.x; }
    __device__ static float hi(Pair p) { return p.y; }
    __device__ static float get(float s) { return s; }
    __device__ static float put(float v) { return v; }
    __device__ static Pair pair(float a, float b) { Pair p; p.x = a; p.y = b; return p; }
};
template <> struct Stor<double> {
    typedef double Pair __attribute__((ext_vector_type(2)));
    __device__ static double lo(Pair p) { return p.x; }
    __device__ static double hi(Pair p) { return p.y; }
    __device__ static double get(double s) { return s; }
    __device__ static double put(double v) { return v; }
    __device__ static Pair pair(double a, double b) { Pair p; p.x = a; p.y = b; return p; }
};
template <> struct Stor<unsigned short> {   // bfloat16
    typedef unsigned int Pair;
    typedef __bf16 BF2 __attribute__((ext_vector_type(2)));
    typedef float F2 __attribute__((ext_vector_type(2)));
    __device__ static float lo(Pair p) { return __uint_as_float(p << 16); }
    __device__ static float hi(Pair p) { return __uint_as_float(p & 0xFFFF0000u); }
    __device__ static float get(unsigned short s) { return __uint_as_float((unsigned)s << 16); }
    // round to nearest even (the hardware conversion)
    __device__ static unsigned short put(float v) { return __builtin_bit_cast(unsigned short, (__bf16)v); }
    __device__ static Pair pair(float a, float b)
    {
        F2 f;
        f.x = a;
        f.y = b;
        return __builtin_bit_cast(Pair, __builtin_convertvector(f, BF2));
    }
};

template <> struct Buf<Stor<float>::Pair> : BufBits<Stor<float>::Pair, U2> {};
template <> struct Buf<Stor<double>::Pair> : BufBits<Stor<double>::Pair, U4> {};

// storage of a level-0 pass (own arrays, coarse arrays) and of a coarse pass
template <typename T> struct LevelStor { typedef T Fine; typedef T Coarse; };
template <> struct LevelStor<float> { typedef float Fine; typedef unsigned short Coarse; };

// Map hardware block ids to logical blocks so that consecutive logical blocks
// (neighbouring strips, which share halo rows/columns) run on the same XCD and
// hit the same L2.  Hardware dispatch places block b on XCD b % 8; the grid
// is padded to a multiple of 8 blocks.
__device__ __forceinline__ int xcd_logical_block()
{
    const int nb8 = gridDim.x >> 3;
    return (blockIdx.x & 7) * nb8 + (blockIdx.x >> 3);
}

// ------------------------------------------------------------ strip pass ---

// Over-relaxation factor of the SOR instances of the fused finest pass
// (red-black order, level 0 only)
constexpr double kOmega = 1.2;

// length of the load queue for a register ring of rs rows (a divisor of rs, so
// that queue slots are compile-time constants in the unrolled ring loop)
#ifndef GDF_QUEUE_MAX
#define GDF_QUEUE_MAX 4
#endif
#ifndef GDF_QUEUE_ZERO
#define GDF_QUEUE_ZERO 4
#endif
constexpr int queue_len(int rs, int qmax)
{
    for (int q = qmax; q >= 2; --q)
        if (rs % q == 0) return q;
    return 1;
}

// QM: the deepest load queue wanted (passes that start from zero load only b
// and afford a deeper one)
template <bool PROLONG, int NHS, int RMODE, int QM = GDF_QUEUE_MAX> struct StripShape {
    static constexpr int NS = NHS + (RMODE != RES_NONE ? 1 : 0);  // stages after the load
    static constexpr int G = (NS + (PROLONG ? 1 : 0) + 1) & ~1;   // halo, even
    static constexpr int VW = kStripCols - 2 * G;                  // owned columns
    // register ring rows: at least 2 NS + 2, rounded up so that a full-depth
    // load queue divides it
    static constexpr int RS = (2 * NS + 2 + QM - 1) / QM * QM;
    // loads run Q - 1 rows ahead of the row entering the ring, so each wave keeps
    // several rows of HBM reads in flight
    static constexpr int Q = queue_len(RS, QM);
};

// Variants.  VAR 1 (interior): the item's rows y0 - G .. y1 + G all lie in
// [1, H - 2] and its columns x0 - G .. x0 - G + 127 in [1, W - 2].  VAR 2
// (column edge): the rows do, but some columns touch or leave the slice.  VAR 0
// (guarded): anything else (the top and bottom bands of a slice).
// With interior rows every stage runs on every step with no row guards: a row
// outside a stage's cone of validity ([y0 - G + s, y1 + G - s) at stage s) gets
// a finite throwaway value, and no row inside the cone ever reads one (the
// cones are nested), so the owned rows come out exactly as in the guarded
// variant.  Inside the cones every row is an interior row (unit vertical
// couplings) on every level; the b ring holds b times the inverse diagonal, so
// an update is one fused multiply-add on the neighbour sum.  With interior
// columns as well (VAR 1) the stencil is the same for every lane (unit
// couplings, diagonal sigma + 4); at column edges it is per lane (masks and,
// on coarse levels, the narrower last column).
// SO: storage of this level's arrays; SC: storage of the next coarser level's
// (prolongation source, restriction target).  Arithmetic is in T.
template <typename T, typename SO, typename SC, bool PROLONG, bool ZERO, int NHS, int RMODE, bool GEN, int VAR,
          bool SOR = false>
__device__ __forceinline__ void strip_item(const StripLaunch &a, int item_id)
{
    constexpr bool RIN = VAR != 0;   // rows interior: no row guards
    constexpr bool CIN = VAR == 1;   // columns interior as well: one stencil for all lanes
    using Sh = StripShape<PROLONG, NHS, RMODE, ZERO ? GDF_QUEUE_ZERO : GDF_QUEUE_MAX>;
    constexpr int NS = Sh::NS, G = Sh::G, VW = Sh::VW, RS = Sh::RS, Q = Sh::Q;
    static_assert((RS & 1) == 0 && RS % Q == 0, "ring slots and queue slots must be static");
    using PO = typename Stor<SO>::Pair;
    using SOt = Stor<SO>;
    using SCt = Stor<SC>;
    constexpr unsigned ES = sizeof(SO), CS = sizeof(SC);

    const int lane = threadIdx.x & (kWave - 1);
    const Item it = uniform_item(a.items[item_id]);
    const LevelDesc L = uniform_level(a.levs[it.lev]);
    if (!uniform(a.active[L.slice])) {
        if ((RMODE & RES_NORM) && lane == 0) a.partials[it.pidx] = make_float2(0.f, 0.f);
        return;
    }
    // copy what is used into scalars (a by-reference lambda capture of the
    // descriptor would force it into scratch memory)
    const int H = L.H, W = L.W, pitch = L.pitch;
    const int Hc = L.Hc, Wc = L.Wc, pitch_c = L.pitch_c;
    const T sig = (T)L.sigma;
    const int y0 = it.y0, y1 = it.y1;
    const int ybase = y0 - G, yend = y1 + G;
    const int NL = yend - ybase;
    const int yo0 = max(y0, 0), yo1 = min(y1, H);   // owned rows inside the slice

    // ---- per-lane column geometry
    const int cx0 = it.x0 - G + 2 * lane;   // even; this lane holds columns cx0, cx0 + 1
    const bool in0 = cx0 >= 0 && cx0 < W;
    const bool in1 = cx0 + 1 >= 0 && cx0 + 1 < W;
    const int cxl = min(max(cx0, 0), (W - 1) & ~1);  // clamped, even: safe vector address
    const unsigned cxb = (unsigned)cxl * ES;          // byte offset of the lane's pair
    const bool own = in0 && cx0 >= it.x0 && cx0 < it.x0 + VW;
    const unsigned vo_own = own ? (unsigned)cx0 * ES : kNoLane;   // the lane's stores
    // neighbour-inside masks (zero for columns outside the slice)
    const T ml0 = (in0 && cx0 - 1 >= 0) ? T(1) : T(0);
    const T mr0 = (in0 && cx0 + 1 < W) ? T(1) : T(0);
    const T ml1 = (in1 && cx0 >= 0) ? T(1) : T(0);
    const T mr1 = (in1 && cx0 + 2 < W) ? T(1) : T(0);
    // inverse diagonal sigma + deg for 0, 1, 2 vertical neighbours (0 outside)
    T inv0[3], inv1[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        inv0[d] = in0 ? T(1) / (sig + ml0 + mr0 + T(d)) : T(0);
        inv1[d] = in1 ? T(1) / (sig + ml1 + mr1 + T(d)) : T(0);
    }
    // unit interior stencil (unguarded items): diagonal and its inverse
    const T dg = sig + T(4), ivs = T(1) / dg;
    // ---- finite-volume coefficients of a coarse level (GEN)
    // columns: relative width wx (only the last column may be narrower); the
    // coupling across a column face is 2 / (wx_left + wx_right) per unit row height
    const T wxL = (T)L.wxL, wyL = (T)L.wyL;
    const T kxe = T(2) / (T(1) + wxL);                 // face next to the last column
    const T wx0 = (cx0 == W - 1) ? wxL : T(1), wx1 = (cx0 + 1 == W - 1) ? wxL : T(1);
    const T kl0 = ml0 * ((cx0 == W - 1) ? kxe : T(1));
    const T kr0 = mr0 * ((cx0 + 1 == W - 1) ? kxe : T(1));
    const T kl1 = ml1 * ((cx0 + 1 == W - 1) ? kxe : T(1));
    const T kr1 = mr1 * ((cx0 + 2 == W - 1) ? kxe : T(1));
    // rows: class 0 interior, 1 first, 2 second-to-last, 3 last; (wy, k_up, k_down)
    const T kye = T(2) / (T(1) + wyL);
    // (scalars with explicit selects: a runtime-indexed array would live in scratch)
    const T ckd1 = (H == 2) ? kye : T(1), cku3 = (H == 1) ? T(0) : kye;
    auto ginv = [sig](T wx, T kl, T kr, bool in, T wy, T ku, T kd) -> T {
        return GEN && in ? T(1) / (sig * wx * wy + wy * (kl + kr) + wx * (ku + kd)) : T(0);
    };
    const T gi00 = ginv(wx0, kl0, kr0, in0, T(1), T(1), T(1)), gi10 = ginv(wx1, kl1, kr1, in1, T(1), T(1), T(1));
    const T gi01 = ginv(wx0, kl0, kr0, in0, T(1), T(0), ckd1), gi11 = ginv(wx1, kl1, kr1, in1, T(1), T(0), ckd1);
    const T gi02 = ginv(wx0, kl0, kr0, in0, T(1), T(1), kye), gi12 = ginv(wx1, kl1, kr1, in1, T(1), T(1), kye);
    const T gi03 = ginv(wx0, kl0, kr0, in0, wyL, cku3, T(0)), gi13 = ginv(wx1, kl1, kr1, in1, wyL, cku3, T(0));
    // row class: 0 interior, 1 first, 2 second-to-last, 3 last -> (wy, k_up, k_down, inverses)
    struct RowC { T wy, ku, kd, i0, i1; };
    auto row_coef = [=](int y) -> RowC {
        if (y == H - 1) return RowC{wyL, cku3, T(0), gi03, gi13};
        if (y == 0) return RowC{T(1), T(0), ckd1, gi01, gi11};
        if (y == H - 2) return RowC{T(1), T(1), kye, gi02, gi12};
        return RowC{T(1), T(1), T(1), gi00, gi10};
    };

    // interior rows, per column j of the lane: inverse diagonal g, its
    // diagonal d, and on coarse levels the couplings scaled by g (left, right,
    // vertical); unit and uniform with interior columns
    const T g0 = CIN ? ivs : (GEN ? gi00 : inv0[2]), g1 = CIN ? ivs : (GEN ? gi10 : inv1[2]);
    const T d0 = CIN ? dg : (GEN ? sig * wx0 + kl0 + kr0 + T(2) * wx0 : sig + ml0 + mr0 + T(2));
    const T d1 = CIN ? dg : (GEN ? sig * wx1 + kl1 + kr1 + T(2) * wx1 : sig + ml1 + mr1 + T(2));
    const T al0 = gi00 * kl0, ar0 = gi00 * kr0, av0 = gi00 * wx0;
    const T al1 = gi10 * kl1, ar1 = gi10 * kr1, av1 = gi10 * wx1;

    // level 0: the slice's mean right-hand side is removed on load, so the
    // iterate is the zero-mean part of the correction (smaller values, smaller
    // FP32 rounding); the mean is added back when f is formed
    const T bsh = L.bshift ? (T)uniform_d(*L.bshift) : T(0);
    // level 1 after a restriction of the unshifted level-0 right-hand side: a
    // cell's children (4 wx wy of them) each carry the level-0 mean
    const T bsc = (a.raw_rhs && L.bshift_fine) ? T(4) * (T)uniform_d(*L.bshift_fine) : T(0);
    const T bsx0 = bsh + bsc * wx0, bsx1 = bsh + bsc * wx1;   // (rows other than the last)
    const T bshg0 = bsx0 * g0, bshg1 = bsx1 * g1;
    // (selects, not a runtime index into the descriptor's array: that would spill it)
    int in_sel = a.in_sel, out_sel = a.out_sel;
    if (a.cycles) {   // per-slice parity: the latest iterate sits in buffer cycles & 1
        in_sel = uniform(a.cycles[(size_t)L.slice * a.cycles_stride]) & 1;
        out_sel = in_sel ^ 1;
    }

    // ---- the item's windows: rows [wlo, whi] of this level and [cwlo, cwhi] of
    // the coarser one hold every access (clamped rows included), so row offsets
    // within them are 32-bit scalars
    const int wlo = max(ybase, 0), whi = min(yend - 1, H - 1);
    const unsigned rowB = (unsigned)pitch * ES;
    const unsigned winB = (unsigned)(whi - wlo + 1) * rowB;
    const size_t wofs = (size_t)wlo * pitch;
    const Rsrc rb = make_rsrc((const SO *)L.b + wofs, winB);
    // The iterate: on level 0 each row stored by colour (see LevelDesc): pixel
    // (x, y) at element x / 2 of the half (x + y) & 1 of row y, the halves
    // pitch / 2 long.  A lane's two columns are element cx0 / 2 of both
    // halves, and the black pixel it loads is in half 1.  Coarse levels keep
    // rows of pixels.
    constexpr bool RB = !GEN;
    const SO *uin = (const SO *)(in_sel ? L.u[1] : L.u[0]);
    SO *uout = (SO *)(out_sel ? L.u[1] : L.u[0]);
    const Rsrc ru = make_rsrc(uin + wofs, winB), rw = make_rsrc(uout + wofs, winB);
    const unsigned hB = RB ? (unsigned)(pitch >> 1) * ES : 0u;                   // half 1 of a row
    const unsigned cxu = RB ? (unsigned)(cxl >> 1) * ES : cxb;                   // the lane's loads
    // Level-0 stores go in lane pairs (cx0 / 2 even: the first of a pair, whose
    // element is 8-byte aligned): the first stores its own and its right
    // neighbour's column-0 values (row parity p: both of half p), the second
    // its left neighbour's and its own column-1 values (both of half 1 - p), so
    // each lane issues one 2-element store.  Owned columns start and end at pair
    // boundaries (x0 and the owned width are multiples of 4); a pair is stored
    // when its first column is owned (its second may lie in the row padding).
    const bool pfirst = ((cx0 >> 1) & 1) == 0;
    const int cxp = pfirst ? cx0 : cx0 - 2;   // the pair's first column
    const bool own_pair = cxp >= 0 && cxp < W && cxp >= it.x0 && cxp < it.x0 + VW;
    const unsigned vo_p0 = own_pair ? (pfirst ? 0u : hB) + (unsigned)(cxp >> 1) * ES : kNoLane;   // p = 0
    const unsigned vo_p1 = own_pair ? (pfirst ? hB : 0u) + (unsigned)(cxp >> 1) * ES : kNoLane;   // p = 1
    const Rsrc rnone = make_rsrc(L.b, 0u);   // drops every store
    // (row offsets go through readfirstlane: a value the compiler happens to
    // compute in vector registers would otherwise get a per-lane loop around
    // each access that takes it)
    auto row_off = [=](int y) -> unsigned {   // y clamped into the slice
        return (unsigned)uniform((RIN ? y - wlo : min(max(y, 0), H - 1) - wlo) * (int)rowB);
    };
    auto win_off = [=](int y) -> unsigned {   // y clamped into the window
        return (unsigned)uniform((min(max(y, wlo), whi) - wlo) * (int)rowB);
    };
    // store one row of the iterate (row parity p = y & 1, static): the lane's
    // two columns, by colour and in lane pairs on level 0
    auto store_u = [&](T v0, T v1, int p, bool keep, int y) {
        if constexpr (RB) {
            const T n0 = wave_shl1(v0), n1 = wave_shr1(v1);
            Buf<PO>::st(pfirst ? SOt::pair(v0, n0) : SOt::pair(n1, v1), keep ? rw : rnone, p ? vo_p1 : vo_p0,
                        win_off(y));
        } else {
            Buf<PO>::st(SOt::pair(v0, v1), keep ? rw : rnone, vo_own, win_off(y));
        }
    };
    const int cwlo = max((wlo >> 1) - 1, 0), cwhi = min((whi >> 1) + 1, Hc - 1);
    const unsigned crowB = (unsigned)pitch_c * CS;
    const unsigned cwinB = (unsigned)max(cwhi - cwlo + 1, 0) * crowB;
    const size_t cofs = (size_t)max(cwlo, 0) * pitch_c;
    auto crow_off = [=](int m) -> unsigned {   // m clamped into the coarse slice
        return (unsigned)uniform((min(max(m, 0), Hc - 1) - cwlo) * (int)crowB);
    };

    // ---- prolongation state (coarse column lc = cx0 / 2)
    const int lc = cx0 >> 1;
    const bool cin = PROLONG && lc >= 0 && lc < Wc;
    const int lcl = PROLONG ? min(max(lc, 0), Wc - 1) : 0;
    const bool ledge = lc == 0, redge = PROLONG && lc == Wc - 1;
    const unsigned lclb = (CIN || cin) ? (unsigned)lcl * CS : kNoLane;   // outside: reads zero
    const Rsrc re = PROLONG ? make_rsrc((const SC *)L.ec + cofs, cwinB) : rnone;

    // ---- restriction state: a coarse cell's right-hand side is the sum of its
    // children's residuals (children outside the slice contribute zero)
    const Rsrc rc = (RMODE & RES_RESTRICT) ? make_rsrc((SC *)L.bc + cofs, cwinB) : rnone;
    const unsigned vo_rc = own ? (unsigned)lc * CS : kNoLane;
    T rpair = T(0);
    const float ownw = own ? 1.f : 0.f;

    T u[RS][2], b[RS][2];
#pragma unroll
    for (int k = 0; k < RS; ++k) u[k][0] = u[k][1] = b[k][0] = b[k][1] = T(0);

    float nacc = 0.f, sacc = 0.f;

    // ---- load queue: raw values of the rows ybase + t + 1 .. ybase + t + Q - 1,
    // issued with clamped (always valid) addresses and consumed Q - 1 steps
    // later, when the row enters the ring (masks and corrections applied there)
    // In the unguarded variant the first half-sweep (red) runs on every row
    // before anything reads the row's red pixel, and a Gauss-Seidel update
    // does not read the old value of the pixel it updates: the old red value
    // is dead.  Only the lane's black column (1 - row parity; ybase and cx0 are
    // even) is loaded, so no load result is dead on arrival (a dead half of a
    // vector load would make the compiler wait for the load to land before
    // reusing its register).
    PO qb[Q], qu[Q];    // raw storage values
    SO qus[Q];          // unguarded: the black column only
    SC qe0[Q], qe1[Q];  // coarse rows m and m -/+ 1 of the row (prolongation)
    auto issue_row = [&](int tq, int par, PO &vb, PO &vu, SO &vus, SC &ve0, SC &ve1) {
        // past the last loaded row the queue re-reads that row (cache hits);
        // outside the slice the row is clamped (the commit zeroes it)
        const int yq = ybase + min(tq, NL - 1);
        const unsigned so = row_off(yq);
        vb = Buf<PO>::ld(rb, cxb, so);
        if (!ZERO) {
            if constexpr (RB) {
                // the black pixel (half 1); the guarded variant both halves, in
                // colour order (the commit maps them to columns)
                if (RIN) vus = Buf<SO>::ld(ru, cxu + hB, so);
                else vu = SOt::pair((T)SOt::get(Buf<SO>::ld(ru, cxu, so)), (T)SOt::get(Buf<SO>::ld(ru, cxu + hB, so)));
            } else {
                if (RIN) vus = Buf<SO>::ld(ru, par ? cxb : cxb + ES, so);
                else vu = Buf<PO>::ld(ru, cxb, so);
            }
        }
        if (PROLONG) {
            const int m = yq >> 1;
            ve0 = Buf<SC>::ld(re, lclb, crow_off(m));
            ve1 = Buf<SC>::ld(re, lclb, crow_off((yq & 1) ? m + 1 : m - 1));
        }
    };
#pragma unroll
    for (int q = 0; q < Q - 1; ++q) issue_row(q, q & 1, qb[q], qu[q], qus[q], qe0[q], qe1[q]);
    // SOR: every half-sweep after the first moves its pixels by kOmega times
    // the Gauss-Seidel step (successive over-relaxation); the first keeps
    // omega = 1, so the red values it overwrites are still never read (and
    // never loaded)
    auto relax = [](T v_gs, T v_old, int s) -> T {
        if constexpr (SOR) return s > 1 ? fma(T(kOmega), v_gs - v_old, v_old) : v_gs;
        else return v_gs;
    };
    // Wait for the first rows here, once per item: with loads still in flight
    // on entry, the wait at the head of the ring loop (which merges the entry
    // with the loop's own back edge) would become a full drain on every trip.
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)

    const int T_end = NL + 2 * NS;
    for (int tb = 0; tb < T_end; tb += RS) {
#pragma unroll
        for (int k = 0; k < RS; ++k) {
            const int t = tb + k;
            // ------------------------------------------------ load (stage 0)
            // issue and commit are unconditional: a conditional consumer would let
            // the compiler sink each load down to it and wait right there
            issue_row(t + Q - 1, (k + Q - 1) & 1, qb[(k + Q - 1) % Q], qu[(k + Q - 1) % Q],
                      qus[(k + Q - 1) % Q], qe0[(k + Q - 1) % Q], qe1[(k + Q - 1) % Q]);
            {
                // rows past the loaded range enter the ring as throwaway copies: no
                // stage inside its cone of validity reads them
                const int y = ybase + t;
                const int qs = k % Q;
                T cor0 = T(0), cor1 = T(0);
                if (PROLONG) {
                    // cell-centred bilinear: 3/4 of the parent row plus 1/4 of the
                    // next coarse row towards this fine row, then the same in x
                    // (lanes whose coarse column lies outside read zero)
                    const T e0 = (T)SCt::get(qe0[qs]);
                    const T e1 = (T)SCt::get(qe1[qs]);
                    const T V = T(0.75) * e0 + T(0.25) * e1;
                    T VL = wave_shr1(V), VR = wave_shl1(V);
                    if (!CIN) {
                        VL = ledge ? V : VL;
                        VR = redge ? V : VR;
                    }
                    cor0 = T(0.75) * V + T(0.25) * VL;
                    cor1 = T(0.75) * V + T(0.25) * VR;
                }
                if (RIN) {
                    b[k][0] = fma((T)SOt::lo(qb[qs]), g0, -bshg0);
                    b[k][1] = fma((T)SOt::hi(qb[qs]), g1, -bshg1);
                    // a column outside the slice (its g is zero) may hold any bits
                    if (!CIN) {
                        b[k][0] = in0 ? b[k][0] : T(0);
                        b[k][1] = in1 ? b[k][1] : T(0);
                    }
                    if (!ZERO || PROLONG) {
                        // row parity = k parity (ybase and tb even): black column 1 - (k & 1);
                        // from a zero iterate (ZERO) the prolonged correction alone
                        if (k & 1) {
                            const T v = (ZERO ? T(0) : (T)SOt::get(qus[qs])) + cor0;
                            u[k][0] = (CIN || in0) ? v : T(0);
                            u[k][1] = T(0);   // red: rewritten by the first half-sweep unread
                        } else {
                            const T v = (ZERO ? T(0) : (T)SOt::get(qus[qs])) + cor1;
                            u[k][0] = T(0);
                            u[k][1] = (CIN || in1) ? v : T(0);
                        }
                    } else {
                        u[k][0] = u[k][1] = T(0);
                    }
                } else {
                    // zero outside the slice (selects, not a branch: a branch here
                    // splits the ring into per-path copies that wait for every load)
                    const bool rin = y >= 0 && y < H;   // uniform
                    const bool v0 = rin && in0, v1 = rin && in1;
                    const T wyr = y == H - 1 ? wyL : T(1);
                    b[k][0] = v0 ? (T)SOt::lo(qb[qs]) - fma(bsc * wx0, wyr, bsh) : T(0);
                    b[k][1] = v1 ? (T)SOt::hi(qb[qs]) - fma(bsc * wx1, wyr, bsh) : T(0);
                    // (level 0: qu holds colours 0 and 1; column cx0 has colour k & 1)
                    const T q0 = (T)(RB && (k & 1) ? SOt::hi(qu[qs]) : SOt::lo(qu[qs]));
                    const T q1 = (T)(RB && (k & 1) ? SOt::lo(qu[qs]) : SOt::hi(qu[qs]));
                    u[k][0] = v0 ? (ZERO ? T(0) : q0) + cor0 : T(0);
                    u[k][1] = v1 ? (ZERO ? T(0) : q1) + cor1 : T(0);
                }
            }
            // ------------------------------------------------ stages 1..NS
#pragma unroll
            for (int s = 1; s <= NS; ++s) {
                const int sl = ((k - 2 * s) % RS + RS) % RS;
                const int su = (sl + RS - 1) % RS;   // row y-1
                const int sd = (sl + 1) % RS;        // row y+1
                const int y = ybase + t - 2 * s;
                const bool owned_row = y >= yo0 && y < yo1;   // uniform
                if (s <= NHS) {
                    const int c = (s - 1) & 1;         // 0: red, 1: black
                    const int j = (k & 1) ^ c;         // column of that colour (y parity = k parity)
                    if (RIN) {
                        // b ring scaled by the inverse diagonal g; neighbours outside
                        // the slice hold zero
                        if (!GEN || CIN) {   // unit couplings
                            if (j == 0) {
                                const T nb = wave_shr1(u[sl][1]) + u[sl][1] + u[su][0] + u[sd][0];
                                u[sl][0] = relax(fma(nb, g0, b[sl][0]), u[sl][0], s);
                            } else {
                                const T nb = wave_shl1(u[sl][0]) + u[sl][0] + u[su][1] + u[sd][1];
                                u[sl][1] = relax(fma(nb, g1, b[sl][1]), u[sl][1], s);
                            }
                        } else {             // coarse level at a column edge: per-lane couplings
                            if (j == 0) {
                                const T v = fma(av0, u[su][0] + u[sd][0], b[sl][0]);
                                u[sl][0] = fma(al0, wave_shr1(u[sl][1]), fma(ar0, u[sl][1], v));
                            } else {
                                const T v = fma(av1, u[su][1] + u[sd][1], b[sl][1]);
                                u[sl][1] = fma(ar1, wave_shl1(u[sl][0]), fma(al1, u[sl][0], v));
                            }
                        }
                        if (s == NHS)
                            store_u(u[sl][0], u[sl][1], k & 1, owned_row, y);
                    } else {
                        const int lo = max(ybase + s, 0), hi = min(yend - s, H);
                        if (y >= lo && y < hi) {
                            if (!GEN) {
                                const int dy = (y > 0) + (y < H - 1);
                                if (j == 0) {
                                    const T iv = dy == 2 ? inv0[2] : (dy == 1 ? inv0[1] : inv0[0]);
                                    const T nb = wave_shr1(u[sl][1]) + u[sl][1] + u[su][0] + u[sd][0];
                                    u[sl][0] = relax((b[sl][0] + nb) * iv, u[sl][0], s);
                                } else {
                                    const T iv = dy == 2 ? inv1[2] : (dy == 1 ? inv1[1] : inv1[0]);
                                    const T nb = wave_shl1(u[sl][0]) + u[sl][0] + u[su][1] + u[sd][1];
                                    u[sl][1] = relax((b[sl][1] + nb) * iv, u[sl][1], s);
                                }
                            } else {
                                const RowC rc = row_coef(y);
                                if (j == 0) {
                                    const T h = fma(kl0, wave_shr1(u[sl][1]), kr0 * u[sl][1]);
                                    const T v = fma(rc.ku, u[su][0], rc.kd * u[sd][0]);
                                    u[sl][0] = (b[sl][0] + fma(rc.wy, h, wx0 * v)) * rc.i0;
                                } else {
                                    const T h = fma(kl1, u[sl][0], kr1 * wave_shl1(u[sl][0]));
                                    const T v = fma(rc.ku, u[su][1], rc.kd * u[sd][1]);
                                    u[sl][1] = (b[sl][1] + fma(rc.wy, h, wx1 * v)) * rc.i1;
                                }
                            }
                            if (s == NHS && owned_row) store_u(u[sl][0], u[sl][1], k & 1, true, y);
                        }
                    }
                } else if (RMODE != RES_NONE) {
                    // r = b - sigma u - sum_q k_q (u - u_q): neighbour differences are
                    // (nearly) exact, so the residual stays accurate in FP32
                    const T uc0 = u[sl][0], uc1 = u[sl][1];
                    T r0 = T(0), rr1 = T(0);
                    if (CIN) {
                        // every row, owned or not (masked below): no branch
                        const T dd = uc0 - uc1;
                        T acc0 = (uc0 - wave_shr1(uc1)) + dd;
                        T acc1 = (uc1 - wave_shl1(uc0)) - dd;
                        acc0 += uc0 - u[su][0];
                        acc1 += uc1 - u[su][1];
                        acc0 += uc0 - u[sd][0];
                        acc1 += uc1 - u[sd][1];
                        // b = (sigma + 4) x the ring's scaled value, exact inside the fma
                        r0 = fma(dg, b[sl][0], -fma(sig, uc0, acc0));
                        rr1 = fma(dg, b[sl][1], -fma(sig, uc1, acc1));
                    } else if (RIN) {
                        // column edge: masked couplings (kl, kr are zero across the
                        // slice edge; wx is 1 but for a narrower last coarse column)
                        const T dd = uc0 - uc1;
                        const T h0 = fma(kr0, dd, kl0 * (uc0 - wave_shr1(uc1)));
                        const T h1 = fma(kl1, -dd, kr1 * (uc1 - wave_shl1(uc0)));
                        const T v0 = (uc0 - u[su][0]) + (uc0 - u[sd][0]);
                        const T v1 = (uc1 - u[su][1]) + (uc1 - u[sd][1]);
                        const T sw0 = GEN ? sig * wx0 : sig, sw1 = GEN ? sig * wx1 : sig;
                        const T acc0 = GEN ? fma(wx0, v0, h0) : v0 + h0;
                        const T acc1 = GEN ? fma(wx1, v1, h1) : v1 + h1;
                        // b = d x the ring's scaled value, exact inside the fma
                        r0 = fma(d0, b[sl][0], -fma(sw0, uc0, acc0));
                        rr1 = fma(d1, b[sl][1], -fma(sw1, uc1, acc1));
                        r0 = in0 ? r0 : T(0);
                        rr1 = in1 ? rr1 : T(0);
                    } else if (owned_row) {
                        const T l0 = wave_shr1(uc1), r1 = wave_shl1(uc0);
                        if (!GEN) {
                            const T mu = y > 0 ? T(1) : T(0), md = y < H - 1 ? T(1) : T(0);
                            T acc0 = ml0 * (uc0 - l0);
                            acc0 = fma(mr0, uc0 - uc1, acc0);
                            acc0 = fma(mu, uc0 - u[su][0], acc0);
                            acc0 = fma(md, uc0 - u[sd][0], acc0);
                            T acc1 = ml1 * (uc1 - uc0);
                            acc1 = fma(mr1, uc1 - r1, acc1);
                            acc1 = fma(mu, uc1 - u[su][1], acc1);
                            acc1 = fma(md, uc1 - u[sd][1], acc1);
                            r0 = fma(-sig, uc0, b[sl][0]) - acc0;
                            rr1 = fma(-sig, uc1, b[sl][1]) - acc1;
                        } else {
                            const RowC rc = row_coef(y);
                            const T wy = rc.wy, ku = rc.ku, kd = rc.kd;
                            const T h0 = fma(kl0, uc0 - l0, kr0 * (uc0 - uc1));
                            const T v0 = fma(ku, uc0 - u[su][0], kd * (uc0 - u[sd][0]));
                            const T h1 = fma(kl1, uc1 - uc0, kr1 * (uc1 - r1));
                            const T v1 = fma(ku, uc1 - u[su][1], kd * (uc1 - u[sd][1]));
                            r0 = fma(-sig * wx0 * wy, uc0, b[sl][0]) - fma(wy, h0, wx0 * v0);
                            rr1 = fma(-sig * wx1 * wy, uc1, b[sl][1]) - fma(wy, h1, wx1 * v1);
                        }
                    }
                    if (RIN || owned_row) {
                        if (RMODE & RES_NORM) {
                            // owned lanes of owned rows (zero for columns outside the slice)
                            const float w = owned_row ? ownw : 0.f;
                            const float f0 = (float)r0, f1 = (float)rr1;
                            nacc = fmaf(w, fmaf(f0, f0, f1 * f1), nacc);
                            sacc = fmaf(w, f0 + f1, sacc);
                        }
                        if (RMODE & RES_RESTRICT) {
                            const T pr = r0 + rr1;      // zero for columns outside the slice
                            if ((k & 1) == 0) {         // y even: first row of a coarse cell
                                if (!RIN && y + 1 >= H)
                                    Buf<SC>::st(SCt::put(pr), rc, vo_rc, crow_off(y >> 1));
                                else
                                    rpair = pr;
                            } else {                    // owned rows come in pairs (y0, y1 even)
                                Buf<SC>::st(SCt::put(rpair + pr), owned_row ? rc : rnone, vo_rc,
                                            crow_off(min(max(y, wlo), whi) >> 1));
                            }
                        }
                    }
                }
            }
        }
    }

    if (RMODE & RES_NORM) {
        double v = (double)nacc, w = (double)sacc;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            v += __shfl_xor(v, off);
            w += __shfl_xor(w, off);
        }
        if (lane == 0) a.partials[it.pidx] = make_float2((float)v, (float)w);
    }
}

// Each wave takes work items w, w + P, w + 2P, ... (P = waves in the grid).
// With a grid covering the list every wave runs one item; a persistent grid
// (capped at the waves the chip holds at once) loops over the list.  Items
// [0, n_fast) run the interior variant, [n_fast, n_rows_in) the column-edge
// one and the rest the guarded one.
template <typename T, typename SO, typename SC, bool PROLONG, bool ZERO, int NHS, int RMODE, bool GEN, bool SOR = false>
__global__ __launch_bounds__(256) void strip_kernel(StripLaunch a)
{
    if (a.done && uniform(*a.done)) return;   // a captured pass after the last active slice
    const int stride = gridDim.x * kWavesPerBlock;
    for (int id = uniform(xcd_logical_block() * kWavesPerBlock + (threadIdx.x >> 6)); id < a.n_items;
         id += stride) {
        if (id < a.n_fast)
            strip_item<T, SO, SC, PROLONG, ZERO, NHS, RMODE, GEN, 1, SOR>(a, id);
        else if (id < a.n_rows_in)
            strip_item<T, SO, SC, PROLONG, ZERO, NHS, RMODE, GEN, 2, SOR>(a, id);
        else
            strip_item<T, SO, SC, PROLONG, ZERO, NHS, RMODE, GEN, 0, SOR>(a, id);
    }
}

// Half-sweeps of the fused finest pass for fsw red-black sweeps.
template <bool PROLONG, int RMODE> static int halo_by_sweeps(int sw)
{
    switch (sw) {
    case 1: return StripShape<PROLONG, 2, RMODE>::G;
    case 2: return StripShape<PROLONG, 4, RMODE>::G;
    case 3: return StripShape<PROLONG, 6, RMODE>::G;
    case 4: return StripShape<PROLONG, 8, RMODE>::G;
    case 5: return StripShape<PROLONG, 10, RMODE>::G;
    case 6: return StripShape<PROLONG, 12, RMODE>::G;
    default: return -1;
    }
}

int strip_halo(StripKind k, int csw, int fsw)
{
    switch (k) {
    case SK_FIRST_RESTRICT: return StripShape<false, 0, RES_RESTRICT>::G;
    case SK_FINE_ZERO:
    case SK_FINE: return halo_by_sweeps<true, RES_BOTH>(fsw);
    case SK_DOWN: return halo_by_sweeps<false, RES_RESTRICT>(csw);
    case SK_UP: return halo_by_sweeps<true, RES_NONE>(csw);
    case SK_COARSE_ZERO:
    case SK_COARSE: return StripShape<false, 4, RES_NONE>::G;
    case SK_SINGLE_ZERO:
    case SK_SINGLE: return StripShape<false, 4, RES_NORM>::G;
    default: return -1;
    }
}

// Workgroups of one kernel that fit on the device at once (occupancy x CUs),
// a multiple of 8; 0 if the runtime cannot tell.
static int resident_blocks(const void *kernel)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess) return 0;
    return (cus * per_cu) & ~7;
}

// Persistent grid size of one kernel instantiation, queried once (a query that
// fails is retried on the next call).  One device type per process.
template <typename T, typename SO, typename SC, bool PROLONG, bool ZERO, int NHS, int RMODE, bool GEN, bool SOR>
static int persistent_cap()
{
    static std::atomic<int> cap{0};
    int c = cap.load(std::memory_order_relaxed);
    if (c == 0) {
        c = resident_blocks(
            reinterpret_cast<const void *>(&strip_kernel<T, SO, SC, PROLONG, ZERO, NHS, RMODE, GEN, SOR>));
        if (c > 0) cap.store(c, std::memory_order_relaxed);
    }
    return c;
}

// Passes on level 0 (GEN false) keep their own arrays in T and the coarse ones
// in LevelStor<T>::Coarse; coarse-level passes (GEN true) keep everything in
// LevelStor<T>::Coarse.  waves non-null: only store the waves resident at once
// (0 if unknown); n_items < 0: only resolve the persistent grid size.
template <typename T, bool PROLONG, bool ZERO, int NHS, int RMODE, bool GEN = false, bool SOR = false>
static hipError_t go(const StripLaunch &a, bool persistent, hipStream_t s, int *waves)
{
    typedef typename LevelStor<T>::Coarse SC;
    typedef typename std::conditional<GEN, SC, T>::type SO;
    if (waves) {
        *waves = persistent_cap<T, SO, SC, PROLONG, ZERO, NHS, RMODE, GEN, SOR>() * kWavesPerBlock;
        return hipSuccess;
    }
    if (a.n_items < 0) {
        persistent_cap<T, SO, SC, PROLONG, ZERO, NHS, RMODE, GEN, SOR>();
        return hipSuccess;
    }
    if (a.n_items == 0) return hipSuccess;
    const int nblocks = (a.n_items + kWavesPerBlock - 1) / kWavesPerBlock;
    int grid = ((nblocks + 7) / 8) * 8;   // multiple of 8 for the XCD remap
    if (persistent) {
        const int cap = persistent_cap<T, SO, SC, PROLONG, ZERO, NHS, RMODE, GEN, SOR>();
        if (cap >= 8 && grid > cap) grid = cap;
    }
    hipLaunchKernelGGL((strip_kernel<T, SO, SC, PROLONG, ZERO, NHS, RMODE, GEN, SOR>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_strip_t(StripKind k, int csw, int fsw, bool p, const StripLaunch &a, hipStream_t s,
                                 int *w = nullptr, bool sor = false)
{
    if (sor) {
        // over-relaxed fused finest passes: FP32 hierarchies, 4 or 5 sweeps
        if (!std::is_same<T, float>::value) return hipErrorInvalidValue;
        const bool zero = k == SK_FINE_ZERO;
        if (k != SK_FINE && !zero) return hipErrorInvalidValue;
        switch (fsw) {
        case 4: return zero ? go<T, true, true, 8, RES_BOTH, false, true>(a, p, s, w)
                            : go<T, true, false, 8, RES_BOTH, false, true>(a, p, s, w);
        case 5: return zero ? go<T, true, true, 10, RES_BOTH, false, true>(a, p, s, w)
                            : go<T, true, false, 10, RES_BOTH, false, true>(a, p, s, w);
        default: return hipErrorInvalidValue;
        }
    }
    switch (k) {
    case SK_FINE:
        switch (fsw) {
        case 2: return go<T, true, false, 4, RES_BOTH>(a, p, s, w);
        case 3: return go<T, true, false, 6, RES_BOTH>(a, p, s, w);
        case 4: return go<T, true, false, 8, RES_BOTH>(a, p, s, w);
        case 5: return go<T, true, false, 10, RES_BOTH>(a, p, s, w);
        case 6: return go<T, true, false, 12, RES_BOTH>(a, p, s, w);
        default: return hipErrorInvalidValue;
        }
    case SK_DOWN:
        switch (csw) {
        case 1: return go<T, false, true, 2, RES_RESTRICT, true>(a, p, s, w);
        case 2: return go<T, false, true, 4, RES_RESTRICT, true>(a, p, s, w);
        case 3: return go<T, false, true, 6, RES_RESTRICT, true>(a, p, s, w);
        default: return hipErrorInvalidValue;
        }
    case SK_UP:
        switch (csw) {
        case 1: return go<T, true, false, 2, RES_NONE, true>(a, p, s, w);
        case 2: return go<T, true, false, 4, RES_NONE, true>(a, p, s, w);
        case 3: return go<T, true, false, 6, RES_NONE, true>(a, p, s, w);
        default: return hipErrorInvalidValue;
        }
    case SK_COARSE_ZERO: return go<T, false, true, 4, RES_NONE, true>(a, p, s, w);
    case SK_COARSE: return go<T, false, false, 4, RES_NONE, true>(a, p, s, w);
    case SK_SINGLE_ZERO: return go<T, false, true, 4, RES_NORM>(a, p, s, w);
    case SK_SINGLE: return go<T, false, false, 4, RES_NORM>(a, p, s, w);
    case SK_FIRST_RESTRICT: return go<T, false, true, 0, RES_RESTRICT>(a, p, s, w);
    case SK_FINE_ZERO:
        switch (fsw) {
        case 2: return go<T, true, true, 4, RES_BOTH>(a, p, s, w);
        case 3: return go<T, true, true, 6, RES_BOTH>(a, p, s, w);
        case 4: return go<T, true, true, 8, RES_BOTH>(a, p, s, w);
        case 5: return go<T, true, true, 10, RES_BOTH>(a, p, s, w);
        case 6: return go<T, true, true, 12, RES_BOTH>(a, p, s, w);
        default: return hipErrorInvalidValue;
        }
    default: return hipErrorInvalidValue;
    }
}

int strip_resident_waves(StripKind k, int csw, int fsw, bool fp64)
{
    StripLaunch a{};
    a.n_items = -1;
    int w = 0;
    const hipError_t e = fp64 ? launch_strip_t<double>(k, csw, fsw, true, a, nullptr, &w)
                              : launch_strip_t<float>(k, csw, fsw, true, a, nullptr, &w);
    return e == hipSuccess ? w : 0;
}

void strip_prepare(int csw, int fsw, bool fp64)
{
    StripLaunch a{};
    a.n_items = -1;
    for (int k = 0; k < SK_COUNT; ++k)
        (void)(fp64 ? launch_strip_t<double>((StripKind)k, csw, fsw, true, a, nullptr)
                    : launch_strip_t<float>((StripKind)k, csw, fsw, true, a, nullptr));
}

hipError_t launch_strip(StripKind k, int csw, int fsw, bool fp64, bool persistent, const StripLaunch &a,
                        hipStream_t s, bool sor)
{
    return fp64 ? launch_strip_t<double>(k, csw, fsw, persistent, a, s, nullptr, sor)
                : launch_strip_t<float>(k, csw, fsw, persistent, a, s, nullptr, sor);
}

}  // namespace gdf
