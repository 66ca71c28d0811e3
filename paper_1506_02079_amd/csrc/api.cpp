// Host side of the gradient-domain fusion library: argument validation, the
// per-slice multigrid hierarchy, the work lists, the V-cycle schedule and the
// C entry points declared in include/gdf.h.
//
// Method (arXiv 1506.02079): anisotropic smoothing across slices (Section
// III-A), then per slice the screened-Poisson blend of Eq. (1).  The solve is
// a multigrid V-cycle iteration on the correction u = f - g_o:
//   level 0 is the pixel grid; level l + 1 halves each side (ceil) and carries
//   sigma_{l+1} = 4 sigma_l; coarsening stops once sigma_l >= 2 (the screened
//   operator is then diagonally dominant enough for a few red-black sweeps to
//   solve it) or the grid is a single pixel.
//   Cycle k (k >= 1): restrict down through the coarse levels (2nu sweeps,
//   residual, restriction), 2 sweeps on the coarsest level, back up
//   (prolongation, 2nu sweeps), then one fused pass on level 0: prolongate,
//   nu post-sweeps of cycle k, nu pre-sweeps of cycle k + 1, residual (its
//   norm is the convergence test), restriction.
// The paper's own solver (the out-of-core streaming multigrid of Kazhdan et
// al. 2010, Implementation subsection) is prior art for a disk-bound CPU; this
// schedule keeps each slice resident in HBM and fuses sweeps instead.
#include "gdf.h"
#include "internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

using namespace gdf;

namespace {

thread_local std::string g_err;

gdf_status set_err(gdf_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return set_err(GDF_EDEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                           __LINE__);                                                          \
    } while (0)

constexpr double kSigmaStop = 2.0;
// Levels whose screening coefficient (alpha 4^l on level l) is at least this
// take nu sweeps per smoothing step instead of the default nu + 1: measured
// on 64 x 2048^2 stacks at alpha 0.001 to 0.1, 1-2% faster at every alpha
// (0.02 and 0.15 each lose at one of them).
constexpr double kSigmaLight = 0.05;
// An FP32 V-cycle that shrinks the residual by less than this factor (the
// usual factor is 0.05 - 0.3) means the iterate has reached FP32's floor.
constexpr double kStallRatio = 0.6;
constexpr int kCoarsePasses = 1;   // x 2 sweeps on the coarsest level (sigma >= 2: enough)
constexpr int kTileW = 64, kTileH = 16;
constexpr size_t kAlign = 256;

size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

template <typename T> void key_push(std::vector<unsigned long long> &k, const T &v)
{
    unsigned long long x = 0;
    std::memcpy(&x, &v, std::min(sizeof v, sizeof x));
    k.push_back(x);
}

// ------------------------------------------------------------------ options

struct Opts {
    int prec, max_vc, nu, out_dtype, use_graph, tile_rows, inner, launch, autotune;
    int fsw;   // sweeps of the fused finest pass
    int csw;   // sweeps per smoothing step on the coarse levels
    bool csw_auto;   // csw defaulted: levels with a strong screening term take nu sweeps
    int robust;   // robust cross-slice averaging in fuse_stack
    int sor;      // over-relaxed fused finest passes
};

gdf_status parse_opts(const gdf_solve_opts *o, Opts &r)
{
    gdf_solve_opts z;
    std::memset(&z, 0, sizeof z);
    if (!o) o = &z;
    r.prec = o->precision;
    if (r.prec < GDF_PREC_FP32 || r.prec > GDF_PREC_MIXED)
        return set_err(GDF_EINVAL, "opts.precision must be GDF_PREC_FP32, _FP64 or _MIXED (got %d)", r.prec);
    r.max_vc = o->max_vcycles ? o->max_vcycles : 40;
    if (r.max_vc < 1 || r.max_vc > 100000)
        return set_err(GDF_EINVAL, "opts.max_vcycles must be in [1, 100000] (got %d)", r.max_vc);
    r.nu = o->nu ? o->nu : 2;
    if (r.nu != 1 && r.nu != 2) return set_err(GDF_EINVAL, "opts.nu must be 1 or 2 (got %d)", r.nu);
    r.out_dtype = o->out_dtype ? o->out_dtype : (r.prec == GDF_PREC_FP32 ? GDF_F32 : GDF_F64);
    if (r.out_dtype != GDF_F32 && r.out_dtype != GDF_F64)
        return set_err(GDF_EINVAL, "opts.out_dtype must be GDF_F32 or GDF_F64 (got %d)", r.out_dtype);
    r.use_graph = o->use_graph != 0;
    r.tile_rows = o->tile_rows;
    if (r.tile_rows && (r.tile_rows < 16 || (r.tile_rows & 1) || r.tile_rows > 65536))
        return set_err(GDF_EINVAL, "opts.tile_rows must be 0 or an even number in [16, 65536] (got %d)", r.tile_rows);
    r.inner = o->inner_cycles ? o->inner_cycles : 3;
    if (r.inner < 1 || r.inner > 64)
        return set_err(GDF_EINVAL, "opts.inner_cycles must be in [1, 64] (got %d)", r.inner);
    r.launch = o->launch_mode ? o->launch_mode : GDF_LAUNCH_GRID;
    if (r.launch != GDF_LAUNCH_GRID && r.launch != GDF_LAUNCH_PERSISTENT)
        return set_err(GDF_EINVAL, "opts.launch_mode must be 0, GDF_LAUNCH_GRID or GDF_LAUNCH_PERSISTENT (got %d)",
                       o->launch_mode);
    r.autotune = o->autotune;
    if (r.autotune != 0 && r.autotune != 1)
        return set_err(GDF_EINVAL, "opts.autotune must be 0 or 1 (got %d)", r.autotune);
    r.fsw = o->fine_sweeps ? o->fine_sweeps : 2 * r.nu;
    if (r.fsw < 2 * r.nu || r.fsw > 2 * r.nu + 2)
        return set_err(GDF_EINVAL, "opts.fine_sweeps must be 0 or in [2 nu, 2 nu + 2] (got %d)", o->fine_sweeps);
    // default: one sweep more than nu on the coarse levels, where it buys whole
    // cycles; the inner solves of the mixed scheme run a fixed cycle count, so
    // there the extra sweep only costs
    r.csw = o->coarse_sweeps ? o->coarse_sweeps : (r.prec == GDF_PREC_MIXED ? r.nu : r.nu + 1);
    if (r.csw < 1 || r.csw > 3)
        return set_err(GDF_EINVAL, "opts.coarse_sweeps must be 0 or in [1, 3] (got %d)", o->coarse_sweeps);
    r.csw_auto = o->coarse_sweeps == 0 && r.csw > r.nu;   // (see kSigmaLight)
    r.robust = o->robust;
    if (r.robust != 0 && r.robust != 1) return set_err(GDF_EINVAL, "opts.robust must be 0 or 1 (got %d)", r.robust);
    if (r.robust && r.prec == GDF_PREC_FP64)
        return set_err(GDF_EUNSUPPORTED, "opts.robust: robust averaging runs in the FP32 smoothing (FP32 or MIXED)");
    r.sor = o->sor;
    if (r.sor != 0 && r.sor != 1) return set_err(GDF_EINVAL, "opts.sor must be 0 or 1 (got %d)", r.sor);
    if (r.sor && (r.prec == GDF_PREC_FP64 || (r.fsw != 4 && r.fsw != 5)))
        return set_err(GDF_EUNSUPPORTED, "opts.sor: over-relaxed sweeps are built for FP32 hierarchies (FP32 or "
                                         "MIXED) with 4 or 5 fused finest sweeps (got fine_sweeps %d)", r.fsw);
    return GDF_OK;
}

gdf_status check_common(int bc, double tol)
{
    if (bc == GDF_BC_DIRICHLET)
        return set_err(GDF_EUNSUPPORTED, "Dirichlet boundaries need boundary values the method does not define");
    if (bc != GDF_BC_NEUMANN && bc != GDF_BC_PERIODIC) return set_err(GDF_EINVAL, "unknown boundary condition %d", bc);
    if (!(tol > 0.0 && tol < 1.0)) return set_err(GDF_EINVAL, "tol must be in (0, 1) (got %g)", tol);
    return GDF_OK;
}

// ------------------------------------------------------------------- plan

struct SliceGeom {
    int H, W;
    double alpha;
    int nlev;
    int h[kMaxLevels], w[kMaxLevels], pitch[kMaxLevels];
    double sigma[kMaxLevels];
    double wxL[kMaxLevels], wyL[kMaxLevels];   // last column / row size relative to a full cell
    size_t off_u[kMaxLevels][2], off_b[kMaxLevels];
    size_t off_u64[2];
};

int level_pitch(int W)
{
    const int p = (W & 1) ? W + 1 : W;
    return (p + 63) / 64 * 64;
}

void build_levels(SliceGeom &g)
{
    g.h[0] = g.H;
    g.w[0] = g.W;
    g.sigma[0] = g.alpha;
    int l = 0;
    while (l + 1 < kMaxLevels && g.sigma[l] < kSigmaStop && (g.h[l] > 1 || g.w[l] > 1)) {
        g.h[l + 1] = (g.h[l] + 1) / 2;
        g.w[l + 1] = (g.w[l] + 1) / 2;
        g.sigma[l + 1] = 4.0 * g.sigma[l];
        ++l;
    }
    g.nlev = l + 1;
    for (int i = 0; i < g.nlev; ++i) g.pitch[i] = level_pitch(g.w[i]);
    // extent of the last cell in pixels: a coarse cell takes two children, or
    // one when the finer side is odd; only the last cell can be partial
    double lx = 1.0, ly = 1.0, side = 1.0;
    g.wxL[0] = g.wyL[0] = 1.0;
    for (int i = 1; i < g.nlev; ++i) {
        lx = (g.w[i - 1] & 1) ? lx : side + lx;
        ly = (g.h[i - 1] & 1) ? ly : side + ly;
        side *= 2.0;
        g.wxL[i] = lx / side;
        g.wyL[i] = ly / side;
    }
}

// A work list: items of one pass kind at one level.  Items clear of the
// slices' first and last rows run the unguarded kernel variant (fast part);
// partial-sum slots (pidx) count over both parts with each slice contiguous.
struct List {
    StripKind kind;
    int level;
    int off, count;            // all items: [off, off + count) = interior, column-edge, guarded
    int n_fast, n_rows_in;
    int G, VW, TH;
    int csw;                   // sweeps per smoothing step of this list's passes (coarse levels)
    std::vector<std::pair<int, double>> slice_px;   // (slice, pixels at this level)
};

enum ProfClass { PC_SMOOTH, PC_FINE, PC_FIRST, PC_COARSE, PC_FINALIZE, PC_PREP, PC_REFINE, PC_ADJOINT, PC_FINE0,
                 PC_COUNT };
const char *kProfNames[PC_COUNT] = {"smooth", "vcycle_fine", "restrict_first", "coarse", "finalize",
                                    "prep", "refine", "adjoint", "vcycle_fine_first"};

struct Plan {
    Opts o;
    bool fp64;       // hierarchy element type
    int esz;         // bytes per level-0 element
    int csz;         // bytes per coarse-level element
    int n;
    std::vector<SliceGeom> g;
    std::vector<int> desc_base;
    std::vector<LevelDesc> descs;
    std::vector<Item> items;
    std::vector<List> lists;
    int list_first = -1, list_fine = -1, list_single = -1;
    int list_down[kMaxLevels], list_up[kMaxLevels], list_coarse[kMaxLevels];
    int max_level = 0;
    std::vector<int> ranges_cycle, ranges_tiles, ranges_ftiles, ranges_smooth;
    int n_norm;
    std::vector<SliceIO> io;
    long long n_tiles = 0;
    long long n_ftiles = 0;    // blocks of the row-marching output pass
    long long n_partd = 0;
    bool mixed = false;
    bool need_gs_copy = false;   // fuse_stack MIXED without g_smooth output
    // periodic boundaries: tiles of every level (list l = all slices having
    // level l, the slices with a level below l first: pmid[l] items); level
    // 0's per-slice slot ranges.  Every plan reserves the tables and partial
    // sums they need, so workspace sizes do not depend on the boundary.
    bool periodic = false;
    std::vector<PItem> pitems;
    int poff[kMaxLevels], pcnt[kMaxLevels], pmid[kMaxLevels];
    std::vector<int> ranges_p0;
    long long n_pitems = 0, n_p0 = 0;
    // layout (bytes from the workspace base)
    size_t off_tables, tables_bytes;
    size_t off_state, off_active, off_only, off_done, off_desc, off_items, off_r_cycle, off_r_tiles, off_r_ftiles,
        off_r_smooth, off_io, off_u64tab, off_pitems, off_r_p0;
    size_t off_partf, off_partd, off_partd2, off_partd3, off_gscopy, off_arena, arena_bytes, total;
};

// Rows per work item of a list (TH): 80 on level 0, halved (down to 16) while
// the list would have fewer than two items per wave the device holds at once.
// Taller items waste less on halo rows; more items keep every SIMD busy to the
// end of the pass.  (Measured on 64 x 2048^2 stacks at alpha 0.001, 0.01 and
// 0.1: 80 rows beat 64, 72, 88, 96, 112, 128 and taller on level 0, by 1-4% of
// the whole step against 128.)
int choose_rows(const Plan &P, const std::vector<int> &slices, int level, StripKind kind, int G, int VW, int csw)
{
    if (level == 0 && P.o.tile_rows) return P.o.tile_rows;
    int slots = strip_resident_waves(kind, csw, P.o.fsw, P.fp64);
    if (slots <= 0) slots = 4096;
    const int E = (G + 2) & ~1;
    // Coarse levels start from 64-row items, 32 on levels of at most 256 rows,
    // and are halved only for batches far too small to fill the GPU: their
    // passes are bound by the serial row march of each item, so many short
    // items (each re-walking its halo rows) lose to fewer taller ones (on the
    // 64 x 2048^2 stack 16-row items on levels 2 and 3 make the coarse levels
    // 18% slower, and so do 128-row items everywhere)
    int th = 80;
    double want = 2.0 * slots;   // level 0: items that fill the GPU twice over
    if (level > 0) {
        int hmax = 0;
        for (int s : slices) hmax = std::max(hmax, P.g[s].h[level]);
        th = hmax <= 256 ? 32 : 64;
        want = slots / 16.0;
    }
    for (; th / 2 >= 16; th /= 2) {
        double items = 0.0;
        for (int s : slices) {
            const int H = P.g[s].h[level], W = P.g[s].w[level];
            const int lo = E, hi = (H - E) & ~1;
            const int nb = hi - lo >= th ? 2 + (hi - lo + th - 1) / th : (H + th - 1) / th;
            items += (double)((W + VW - 1) / VW) * nb;
        }
        if (items >= want) break;
    }
    return th;
}

int add_list(Plan &P, StripKind kind, int level, const std::vector<int> &slices)
{
    if (slices.empty()) return -1;
    List L;
    L.kind = kind;
    L.level = level;
    // coarse sweeps by default: nu + 1, and nu on levels where every slice's
    // screening coefficient is at least kSigmaLight (there the extra sweep
    // buys no cycles)
    L.csw = P.o.csw;
    if (P.o.csw_auto && (kind == SK_DOWN || kind == SK_UP)) {
        double smin = 1e300;
        for (int sl : slices) smin = std::min(smin, P.g[sl].sigma[level]);
        if (smin >= kSigmaLight) L.csw = P.o.nu;
    }
    L.G = strip_halo(kind, L.csw, P.o.fsw);
    L.VW = kStripCols - 2 * L.G;
    L.TH = choose_rows(P, slices, level, kind, L.G, L.VW, L.csw);
    // the rows an item touches must span less than 2^31 bytes (the kernel
    // addresses them with 32-bit offsets); with W <= kMaxWidth this leaves at
    // least 16 rows per item
    int maxp = 0;
    for (int s : slices) maxp = std::max(maxp, P.g[s].pitch[level]);
    const long long row_bytes = (long long)maxp * (level == 0 ? P.esz : P.csz);
    const long long rmax = (0x7FFFFFFFLL / row_bytes - 2 * L.G - 4) & ~1LL;
    if (L.TH > rmax) L.TH = (int)std::max<long long>(16, rmax);
    L.off = (int)P.items.size();
    std::vector<Item> fast, edge, guarded;
    int pidx = 0;
    // Row bands: a thin band at the top and at the bottom of a slice (just
    // deep enough for the halo: these items run the guarded code), and bands
    // of TH rows in between, whose items are clear of the top and bottom edges.
    // Band starts are even (the kernel's row parity and restriction pairs).
    const int E = (L.G + 2) & ~1;   // >= G + 1
    std::vector<std::pair<int, int>> bands;
    for (int s : slices) {
        const SliceGeom &g = P.g[s];
        const int H = g.h[level], W = g.w[level];
        L.slice_px.emplace_back(s, (double)H * W);
        bands.clear();
        const int lo = E, hi = (H - E) & ~1;   // interior rows [lo, hi)
        if (hi - lo >= L.TH) {
            bands.emplace_back(0, lo);
            for (int y0 = lo; y0 < hi; y0 += L.TH) bands.emplace_back(y0, std::min(y0 + L.TH, hi));
            bands.emplace_back(hi, H);
        } else {
            for (int y0 = 0; y0 < H; y0 += L.TH) bands.emplace_back(y0, std::min(y0 + L.TH, H));
        }
        for (const auto &band : bands) {
            const int y0 = band.first, y1 = band.second;
            const bool yin = y0 - L.G >= 1 && y1 + L.G <= H - 1;
            for (int x0 = 0; x0 < W; x0 += L.VW) {
                const bool xin = x0 - L.G >= 1 && x0 - L.G + kStripCols - 1 <= W - 2;
                (yin ? (xin ? fast : edge) : guarded).push_back(Item{P.desc_base[s] + level, x0, y0, y1, pidx++});
            }
        }
    }
    P.items.insert(P.items.end(), fast.begin(), fast.end());
    P.items.insert(P.items.end(), edge.begin(), edge.end());
    P.items.insert(P.items.end(), guarded.begin(), guarded.end());
    L.n_fast = (int)fast.size();
    L.n_rows_in = (int)(fast.size() + edge.size());
    L.count = (int)P.items.size() - L.off;
    P.lists.push_back(L);
    return (int)P.lists.size() - 1;
}

// per-slice [begin, end) of a list's partial-sum slots
void list_ranges(const Plan &P, int li, int base, std::vector<int> &r)
{
    if (li < 0) return;
    const List &L = P.lists[li];
    for (int i = 0; i < L.count; ++i) {
        const Item &it = P.items[L.off + i];
        const int s = P.descs[it.lev].slice;
        if (r[2 * s] < 0 || base + it.pidx < r[2 * s]) r[2 * s] = base + it.pidx;
        r[2 * s + 1] = std::max(r[2 * s + 1], base + it.pidx + 1);
    }
}

// Builds geometry, work lists and the workspace layout.  Host only.
gdf_status make_plan(Plan &P, int n, const std::vector<int> &H, const std::vector<int> &W,
                     const std::vector<double> &alpha, const Opts &o, int smooth_S)
{
    P.o = o;
    P.n = n;
    P.mixed = o.prec == GDF_PREC_MIXED;
    P.fp64 = o.prec == GDF_PREC_FP64;
    P.esz = P.fp64 ? 8 : 4;
    P.csz = P.fp64 ? 8 : 2;   // coarse levels of an FP32 hierarchy are stored as bfloat16
    P.g.resize(n);
    P.desc_base.resize(n);
    int nd = 0;
    for (int s = 0; s < n; ++s) {
        SliceGeom &g = P.g[s];
        g.H = H[s];
        g.W = W[s];
        g.alpha = alpha[s];
        build_levels(g);
        P.desc_base[s] = nd;
        nd += g.nlev;
        P.max_level = std::max(P.max_level, g.nlev - 1);
    }
    // arena: per slice, per level u[0], u[1], b; plus the FP64 iterates when mixed
    size_t off = 0;
    for (int s = 0; s < n; ++s) {
        SliceGeom &g = P.g[s];
        for (int l = 0; l < g.nlev; ++l) {
            const size_t bytes = align_up((size_t)g.h[l] * g.pitch[l] * (l == 0 ? P.esz : P.csz));
            g.off_u[l][0] = off; off += bytes;
            g.off_u[l][1] = off; off += bytes;
            g.off_b[l] = off; off += bytes;
        }
        if (P.mixed) {
            const size_t bytes = align_up((size_t)g.h[0] * g.pitch[0] * 8);
            g.off_u64[0] = off; off += bytes;
            g.off_u64[1] = off; off += bytes;
        }
    }
    P.arena_bytes = off;
    // level descriptors (pointers filled at bind time)
    P.descs.resize(nd);
    for (int s = 0; s < n; ++s) {
        const SliceGeom &g = P.g[s];
        for (int l = 0; l < g.nlev; ++l) {
            LevelDesc &d = P.descs[P.desc_base[s] + l];
            std::memset(&d, 0, sizeof d);
            d.H = g.h[l];
            d.W = g.w[l];
            d.pitch = g.pitch[l];
            d.sigma = g.sigma[l];
            d.wxL = g.wxL[l];
            d.wyL = g.wyL[l];
            d.slice = s;
            if (l + 1 < g.nlev) {
                d.Hc = g.h[l + 1];
                d.Wc = g.w[l + 1];
                d.pitch_c = g.pitch[l + 1];
            } else {
                d.Hc = d.Wc = 1;
                d.pitch_c = 0;
            }
        }
    }
    // work lists
    for (int l = 0; l < kMaxLevels; ++l) P.list_down[l] = P.list_up[l] = P.list_coarse[l] = -1;
    std::vector<int> mid0, single0;
    for (int s = 0; s < n; ++s) (P.g[s].nlev > 1 ? mid0 : single0).push_back(s);
    P.list_first = add_list(P, SK_FIRST_RESTRICT, 0, mid0);
    P.list_fine = add_list(P, SK_FINE, 0, mid0);
    P.list_single = add_list(P, SK_SINGLE, 0, single0);
    for (int l = 1; l <= P.max_level; ++l) {
        std::vector<int> mid, coarsest;
        for (int s = 0; s < n; ++s) {
            if (P.g[s].nlev - 1 > l) mid.push_back(s);
            else if (P.g[s].nlev - 1 == l) coarsest.push_back(s);
        }
        P.list_down[l] = add_list(P, SK_DOWN, l, mid);
        P.list_up[l] = add_list(P, SK_UP, l, mid);
        P.list_coarse[l] = add_list(P, SK_COARSE, l, coarsest);
    }
    const int nC = P.list_fine >= 0 ? P.lists[P.list_fine].count : 0;
    const int nS = P.list_single >= 0 ? P.lists[P.list_single].count : 0;
    P.n_norm = nC + nS;   // norm partials: fused finest pass, then single-level slices
    P.ranges_cycle.assign(2 * n, -1);
    list_ranges(P, P.list_fine, 0, P.ranges_cycle);
    list_ranges(P, P.list_single, nC, P.ranges_cycle);
    // tiles for the per-pixel kernels
    P.io.resize(n);
    P.ranges_tiles.resize(2 * n);
    P.ranges_ftiles.resize(2 * n);
    long long tb = 0, fb = 0;
    for (int s = 0; s < n; ++s) {
        SliceIO &io = P.io[s];
        std::memset(&io, 0, sizeof io);
        io.alpha = alpha[s];
        io.H = H[s];
        io.W = W[s];
        io.lev0 = P.desc_base[s];
        io.tiles_x = (W[s] + kTileW - 1) / kTileW;
        io.tile_begin = tb;
        const long long nt = (long long)io.tiles_x * ((H[s] + kTileH - 1) / kTileH);
        P.ranges_tiles[2 * s] = (int)tb;
        tb += nt;
        P.ranges_tiles[2 * s + 1] = (int)tb;
        io.ftiles_x = (W[s] + kFinCols - 1) / kFinCols;
        io.ftile_begin = fb;
        P.ranges_ftiles[2 * s] = (int)fb;
        fb += (long long)io.ftiles_x * ((H[s] + kFinRows - 1) / kFinRows);
        P.ranges_ftiles[2 * s + 1] = (int)fb;
    }
    P.n_tiles = tb;
    P.n_ftiles = fb;
    P.n_partd = tb;
    // periodic tiles (counted for every plan, built for periodic ones)
    auto ptiles = [&](int s, int l) {
        return (long long)((P.g[s].h[l] + kPTileH - 1) / kPTileH) * ((P.g[s].w[l] + kPTileW - 1) / kPTileW);
    };
    for (int s = 0; s < n; ++s)
        for (int l = 0; l < P.g[s].nlev; ++l) {
            P.n_pitems += ptiles(s, l);
            if (l == 0) P.n_p0 += ptiles(s, l);
        }
    P.n_partd = std::max(P.n_partd, P.n_p0);
    P.ranges_p0.assign(2 * n, 0);
    for (int l = 0; l < kMaxLevels; ++l) P.poff[l] = P.pcnt[l] = P.pmid[l] = 0;
    if (P.periodic) {
        std::vector<int> order(n);
        for (int s = 0; s < n; ++s) order[s] = s;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return P.g[a].nlev > P.g[b].nlev; });
        for (int l = 0; l <= P.max_level; ++l) {
            P.poff[l] = (int)P.pitems.size();
            for (int s : order) {
                const SliceGeom &g = P.g[s];
                if (g.nlev <= l) continue;
                if (l == 0) P.ranges_p0[2 * s] = (int)P.pitems.size() - P.poff[0];
                for (int y0 = 0; y0 < g.h[l]; y0 += kPTileH)
                    for (int x0 = 0; x0 < g.w[l]; x0 += kPTileW)
                        P.pitems.push_back(PItem{P.desc_base[s] + l, s, x0, y0});
                if (l == 0) P.ranges_p0[2 * s + 1] = (int)P.pitems.size() - P.poff[0];
                if (g.nlev > l + 1) P.pmid[l] = (int)P.pitems.size() - P.poff[l];
            }
            P.pcnt[l] = (int)P.pitems.size() - P.poff[l];
        }
    }
    if (smooth_S > 0) {
        // smoothing partials: [S][tiles]
        const long long nparts = (long long)((W[0] + kSmoothTileW - 1) / kSmoothTileW) *
                                 ((H[0] + kSmoothTileH - 1) / kSmoothTileH);   // one per tile
        P.ranges_smooth.resize(2 * n);
        for (int s = 0; s < n; ++s) {
            P.ranges_smooth[2 * s] = (int)(s * nparts);
            P.ranges_smooth[2 * s + 1] = (int)((s + 1) * nparts);
        }
        P.n_partd = std::max<long long>(P.n_partd, nparts * n);
    }
    if (P.n_partd > 0x7fffffffLL || P.items.size() > 0x7fffffffULL || P.n_pitems > 0x7fffffffLL)
        return set_err(GDF_EUNSUPPORTED, "problem too large for 32-bit work indices");
    // layout: [tables][partials][gs copy][arena]
    size_t o2 = 0;
    auto take = [&](size_t bytes) { const size_t r = o2; o2 += align_up(bytes); return r; };
    P.off_tables = 0;
    P.off_state = take(sizeof(SliceState) * n);
    P.off_active = take(sizeof(int) * n);
    P.off_only = take(sizeof(int) * n);
    P.off_done = take(sizeof(int));
    P.off_desc = take(sizeof(LevelDesc) * P.descs.size());
    P.off_items = take(sizeof(Item) * std::max<size_t>(1, P.items.size()));
    P.off_r_cycle = take(sizeof(int) * 2 * n);
    P.off_r_tiles = take(sizeof(int) * 2 * n);
    P.off_r_ftiles = take(sizeof(int) * 2 * n);
    P.off_r_smooth = take(sizeof(int) * 2 * n);
    P.off_io = take(sizeof(SliceIO) * n);
    P.off_u64tab = take(sizeof(double *) * 2 * n);
    P.off_r_p0 = take(sizeof(int) * 2 * n);
    P.off_pitems = take(sizeof(PItem) * (size_t)std::max<long long>(1, P.n_pitems));
    P.tables_bytes = o2;
    P.off_partf = take(sizeof(float2) * std::max(1, P.n_norm));
    P.off_partd = take(sizeof(double) * std::max<long long>(1, P.n_partd));
    P.off_partd2 = take(sizeof(double) * std::max<long long>(1, P.n_partd));
    P.off_partd3 = take(sizeof(double) * std::max<long long>(1, P.n_partd));
    P.off_gscopy = o2;
    if (P.need_gs_copy) take((size_t)n * H[0] * W[0] * sizeof(float));
    P.off_arena = take(0);
    P.total = P.off_arena + P.arena_bytes;
    return GDF_OK;
}

// Fills device pointers into the descriptors and returns the host image of
// the tables region.
std::vector<char> bind_tables(const Plan &P, char *ws, const std::vector<SliceIO> &io)
{
    char *arena = ws + P.off_arena;
    SliceState *st_dev = reinterpret_cast<SliceState *>(ws + P.off_state);
    std::vector<LevelDesc> descs = P.descs;
    for (int s = 0; s < P.n; ++s) {
        const SliceGeom &g = P.g[s];
        for (int l = 0; l < g.nlev; ++l) {
            LevelDesc &d = descs[P.desc_base[s] + l];
            d.u[0] = arena + g.off_u[l][0];
            d.u[1] = arena + g.off_u[l][1];
            d.b = arena + g.off_b[l];
            d.bshift = (l == 0 && !P.mixed) ? &st_dev[s].bmean : nullptr;
            d.bshift_fine = (l == 1 && !P.mixed) ? &st_dev[s].bmean : nullptr;
            if (l + 1 < g.nlev) {
                d.bc = arena + g.off_b[l + 1];
                // level l+1's final iterate: buffer 1 after an up pass; the
                // coarsest level ends its kCoarsePasses passes in buffer (passes-1)&1
                const int fin = (l + 1 == g.nlev - 1) ? ((kCoarsePasses - 1) & 1) : 1;
                d.ec = arena + g.off_u[l + 1][fin];
            }
        }
    }
    std::vector<char> img(P.periodic ? P.tables_bytes : P.off_pitems, 0);
    // state zeroed except the per-slice constants; active = 1
    SliceState *st = reinterpret_cast<SliceState *>(img.data() + P.off_state);
    int *act = reinterpret_cast<int *>(img.data() + P.off_active);
    for (int s = 0; s < P.n; ++s) {
        st[s].npx = (double)P.g[s].H * P.g[s].W;
        st[s].alpha = P.g[s].alpha;
        act[s] = 1;
    }
    std::memcpy(img.data() + P.off_desc, descs.data(), sizeof(LevelDesc) * descs.size());
    if (!P.items.empty()) std::memcpy(img.data() + P.off_items, P.items.data(), sizeof(Item) * P.items.size());
    std::memcpy(img.data() + P.off_r_cycle, P.ranges_cycle.data(), sizeof(int) * 2 * P.n);
    std::memcpy(img.data() + P.off_r_tiles, P.ranges_tiles.data(), sizeof(int) * 2 * P.n);
    std::memcpy(img.data() + P.off_r_ftiles, P.ranges_ftiles.data(), sizeof(int) * 2 * P.n);
    if (!P.ranges_smooth.empty())
        std::memcpy(img.data() + P.off_r_smooth, P.ranges_smooth.data(), sizeof(int) * 2 * P.n);
    std::memcpy(img.data() + P.off_io, io.data(), sizeof(SliceIO) * P.n);
    std::memcpy(img.data() + P.off_r_p0, P.ranges_p0.data(), sizeof(int) * 2 * P.n);
    if (!P.pitems.empty())
        std::memcpy(img.data() + P.off_pitems, P.pitems.data(), sizeof(PItem) * P.pitems.size());
    if (P.mixed) {
        double **tab = reinterpret_cast<double **>(img.data() + P.off_u64tab);
        for (int s = 0; s < P.n; ++s) {
            tab[s] = reinterpret_cast<double *>(arena + P.g[s].off_u64[0]);
            tab[P.n + s] = reinterpret_cast<double *>(arena + P.g[s].off_u64[1]);
        }
    }
    return img;
}

// --------------------------------------------------------------- plan cache
//
// A plan is a pure function of the batch shape and the options; for large
// batches it holds hundreds of thousands of work items and takes milliseconds
// to build, so recent plans are kept, read-only, and shared between calls.

std::mutex g_plan_mu;
std::vector<std::pair<std::vector<unsigned long long>, std::shared_ptr<const Plan>>> g_plans;

gdf_status cached_plan(std::shared_ptr<const Plan> &out, int n, const std::vector<int> &H,
                       const std::vector<int> &W, const std::vector<double> &al, const Opts &o, int smooth_S,
                       bool need_gs, bool periodic = false)
{
    std::vector<unsigned long long> key;
    for (int v : {n, smooth_S, need_gs ? 1 : 0, periodic ? 1 : 0, o.prec, o.max_vc, o.nu, o.csw, o.csw_auto ? 1 : 0, o.out_dtype,
                  o.use_graph, o.tile_rows, o.inner, o.launch, o.fsw, o.sor})
        key_push(key, v);
    for (int i = 0; i < n; ++i) {
        key_push(key, H[i]);
        key_push(key, W[i]);
        key_push(key, al[i]);
    }
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        for (size_t i = 0; i < g_plans.size(); ++i)
            if (g_plans[i].first == key) {
                out = g_plans[i].second;
                std::rotate(g_plans.begin() + i, g_plans.begin() + i + 1, g_plans.end());   // most recent last
                return GDF_OK;
            }
    }
    auto p = std::make_shared<Plan>();
    p->need_gs_copy = need_gs;
    p->periodic = periodic;
    const gdf_status r = make_plan(*p, n, H, W, al, o, smooth_S);
    if (r) return r;
    std::lock_guard<std::mutex> lk(g_plan_mu);
    if (g_plans.size() >= 16) g_plans.erase(g_plans.begin());
    g_plans.emplace_back(std::move(key), p);
    out = p;
    return GDF_OK;
}

// ---------------------------------------------------------------- profiling

std::mutex g_prof_mu;
bool g_prof_on = false;
bool g_prof_fine_only = false;   // mode 2: only the fused finest pass is timed
struct ProfRec { int cls; hipEvent_t a, b; double bytes; };
std::vector<ProfRec> g_prof_recs;
std::vector<hipEvent_t> g_prof_pool;
double g_prof_ms[PC_COUNT], g_prof_bytes[PC_COUNT];
int g_prof_n[PC_COUNT];

hipEvent_t prof_event()
{
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void prof_drain()
{
    for (ProfRec &r : g_prof_recs) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            g_prof_ms[r.cls] += ms;
            g_prof_bytes[r.cls] += r.bytes;
            g_prof_n[r.cls] += 1;
        }
        g_prof_pool.push_back(r.a);
        g_prof_pool.push_back(r.b);
    }
    g_prof_recs.clear();
}

struct ProfScope {
    bool on;
    ProfRec rec;
    hipStream_t s;
    ProfScope(int cls, double bytes, hipStream_t st, bool capturing) : on(false), s(st)
    {
        if (!g_prof_on || capturing || (g_prof_fine_only && cls != PC_FINE)) return;
        std::lock_guard<std::mutex> lk(g_prof_mu);
        rec.cls = cls;
        rec.bytes = bytes;
        rec.a = prof_event();
        rec.b = prof_event();
        if (!rec.a || !rec.b) return;
        on = hipEventRecord(rec.a, s) == hipSuccess;
    }
    ~ProfScope()
    {
        if (!on) return;
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (hipEventRecord(rec.b, s) == hipSuccess) g_prof_recs.push_back(rec);
    }
};

// ------------------------------------------------------------------ driver

// Set for the duration of a solve_slices_noalloc call on this thread: host
// reads of device flags then go to pageable memory instead of the page-locked
// buffer below (whose first use allocates it).
thread_local bool t_no_pinned = false;

// Page-locked host buffer for the per-cycle convergence flags (a direct copy,
// no staging through a bounce buffer), one per thread, grown as needed and
// kept until the process ends.
hipError_t pinned_flags(int n, int *&out)
{
    if (t_no_pinned) {
        thread_local std::vector<int> pageable;
        if ((int)pageable.size() < n) pageable.resize(n);
        out = pageable.data();
        return hipSuccess;
    }
    thread_local int *buf = nullptr;
    thread_local int cap = 0;
    if (cap < n) {
        int *nb = nullptr;
        const int want = std::max(n, 1024);
        const hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&nb), sizeof(int) * (size_t)want,
                                           hipHostMallocDefault);
        if (e != hipSuccess) return e;
        if (buf) (void)hipHostFree(buf);
        buf = nb;
        cap = want;
    }
    out = buf;
    return hipSuccess;
}

struct Run {
    const Plan &P;
    char *ws;
    hipStream_t s;
    bool capturing = false;
    SliceState *st;
    int *active;
    int *only;      // slices to re-finalize after a resume
    int *done;      // set when no slice is active (read by the passes of a captured schedule)
    LevelDesc *desc;
    Item *items;
    int *r_cycle, *r_tiles, *r_ftiles, *r_smooth;
    SliceIO *io;
    double **u64tab;
    float2 *partf;
    double *partd, *partd2, *partd3;
    PItem *pitems;
    int *r_p0;
    std::vector<char> active_host;
    double tol;
    int max_cycles;
    double stall_ratio = 0.0;   // FIN_CHECK stall test (FP32 iterates only)
    // the smoothing pass restricted the unshifted b to level 1: the first pass
    // skips its restriction and the next level-1 down pass removes the mean
    bool raw_rhs_l1 = false;

    Run(const Plan &p, char *w, hipStream_t st_) : P(p), ws(w), s(st_)
    {
        st = reinterpret_cast<SliceState *>(ws + P.off_state);
        active = reinterpret_cast<int *>(ws + P.off_active);
        only = reinterpret_cast<int *>(ws + P.off_only);
        done = reinterpret_cast<int *>(ws + P.off_done);
        desc = reinterpret_cast<LevelDesc *>(ws + P.off_desc);
        items = reinterpret_cast<Item *>(ws + P.off_items);
        r_cycle = reinterpret_cast<int *>(ws + P.off_r_cycle);
        r_tiles = reinterpret_cast<int *>(ws + P.off_r_tiles);
        r_ftiles = reinterpret_cast<int *>(ws + P.off_r_ftiles);
        r_smooth = reinterpret_cast<int *>(ws + P.off_r_smooth);
        io = reinterpret_cast<SliceIO *>(ws + P.off_io);
        u64tab = reinterpret_cast<double **>(ws + P.off_u64tab);
        partf = reinterpret_cast<float2 *>(ws + P.off_partf);
        partd = reinterpret_cast<double *>(ws + P.off_partd);
        partd2 = reinterpret_cast<double *>(ws + P.off_partd2);
        partd3 = reinterpret_cast<double *>(ws + P.off_partd3);
        pitems = reinterpret_cast<PItem *>(ws + P.off_pitems);
        r_p0 = reinterpret_cast<int *>(ws + P.off_r_p0);
        active_host.assign(P.n, 1);
    }

    // ---- periodic boundaries
    // launch arguments over level l's tiles (mid: only the slices that have a
    // level below l)
    PLaunch plaunch(int l, bool mid = false) const
    {
        PLaunch a{};
        a.levs = desc;
        a.items = pitems + P.poff[l];
        a.n_items = mid ? P.pmid[l] : P.pcnt[l];
        a.active = active;
        // the per-cycle norms go to their own arrays: the output pass keeps the
        // partial sums of slices it skips in a resume round in partd
        a.part_rr = partd2;
        a.part_r = partd3;
        return a;
    }
    gdf_status psmooth(int l, int half_sweeps, int &cur, bool zero_first, bool fp64)
    {
        for (int h = 0; h < half_sweeps; ++h) {
            PLaunch a = plaunch(l);
            a.colour = h & 1;
            a.in_sel = cur;
            a.out_sel = cur ^ 1;
            a.zero_in = h == 0 && zero_first;
            ProfScope ps(PC_COARSE, 0.0, s, capturing);
            HIP_TRY(launch_psmooth_level(fp64, l == 0, a, s));
            cur ^= 1;
        }
        return GDF_OK;
    }
    // One V-cycle with periodic boundaries: down the levels (pre-smoothing,
    // residual restricted into the next level's right-hand side; coarse levels
    // start from zero), then up (prolongation of the coarser iterate, post-
    // smoothing).  Each slice's coarsest level is smoothed on the way down and
    // on the way up.  Level 0 takes nu sweeps each way, the coarse levels
    // coarse_sweeps; an even number of half-sweeps per cycle leaves the
    // level-0 iterate in buffer 0.
    gdf_status pcycle(bool fp64, bool zero)
    {
        gdf_status r;
        int cur[kMaxLevels] = {0};
        for (int l = 0; l <= P.max_level; ++l) {
            if ((r = psmooth(l, 2 * (l == 0 ? P.o.nu : P.o.csw), cur[l], l > 0 || zero, fp64))) return r;
            if (l < P.max_level) {
                PLaunch a = plaunch(l + 1);
                a.in_sel = cur[l];
                ProfScope ps(PC_COARSE, 0.0, s, capturing);
                HIP_TRY(launch_prestrict_level(fp64, l == 0, a, s));
            }
        }
        for (int l = P.max_level; l >= 0; --l) {
            if (l < P.max_level) {
                PLaunch a = plaunch(l, true);
                a.in_sel = cur[l];
                a.coarse_sel = cur[l + 1];
                ProfScope ps(PC_COARSE, 0.0, s, capturing);
                HIP_TRY(launch_pprolong_level(fp64, l == 0, a, s));
            }
            if ((r = psmooth(l, 2 * (l == 0 ? P.o.nu : P.o.csw), cur[l], false, fp64))) return r;
        }
        return GDF_OK;
    }
    // the in-loop convergence check after a cycle
    gdf_status check_cycle(bool fp64)
    {
        if (!P.periodic) return finish(r_cycle, partf, nullptr, FIN_CHECK, 1);
        PLaunch a = plaunch(0);
        a.in_sel = 0;
        HIP_TRY(launch_pnorm(fp64, a, s));
        return finish(r_p0, nullptr, partd2, FIN_CHECK, 1, partd3);
    }

    // algorithmic bytes of a list's pass over the slices still iterating
    double pass_bytes(int li, double per_px) const
    {
        double px = 0.0;
        for (const auto &e : P.lists[li].slice_px)
            if (active_host[e.first]) px += e.second;
        return px * per_px;
    }

    gdf_status strip(int li, StripKind kind, int in_sel, int out_sel, float2 *partials, bool fp64,
                     int cls, double per_px, bool slice_parity = false, bool raw_rhs = false)
    {
        if (li < 0) return GDF_OK;
        const List &L = P.lists[li];
        if (L.count == 0) return GDF_OK;
        StripLaunch a{};
        a.levs = desc;
        a.in_sel = in_sel;
        a.out_sel = out_sel;
        a.cycles = slice_parity ? &st[0].cycles : nullptr;
        a.cycles_stride = (int)(sizeof(SliceState) / sizeof(int));
        a.active = active;
        a.done = capturing ? done : nullptr;
        a.partials = partials;
        a.raw_rhs = raw_rhs ? 1 : 0;
        const bool timed = g_prof_on && (!g_prof_fine_only || cls == PC_FINE);
        ProfScope ps(cls, timed ? pass_bytes(li, per_px) : 0.0, s, capturing);
        a.items = items + L.off;
        a.n_items = L.count;
        a.n_fast = L.n_fast;
        a.n_rows_in = L.n_rows_in;
        const bool sor = P.o.sor && (kind == SK_FINE || kind == SK_FINE_ZERO);
        HIP_TRY(launch_strip(kind, L.csw, P.o.fsw, fp64, P.o.launch == GDF_LAUNCH_PERSISTENT, a, s, sor));
        return GDF_OK;
    }

    // The in-loop test uses 0.99 tol: the working-precision residual can sit a
    // hair below the exact FP64 residual of the output, which is checked after.
    // (in-loop checks -- strip partials, or FP64 partials with the sums of r --
    // use the working-precision residual)
    gdf_status finish(const int *range, const float2 *pf, const double *pd, int mode, int count,
                      const double *pd2 = nullptr)
    {
        const bool in_loop = mode == FIN_CHECK && (pf || pd2);
        const double t = in_loop ? 0.99 * tol : tol;
        HIP_TRY(launch_finish(P.n, range, pf, pd, pd2, mode, t, max_cycles, count, in_loop ? stall_ratio : 0.0, st,
                              active, s));
        return GDF_OK;
    }

    // one multigrid coarse-grid correction (levels >= 1), hierarchy precision fp64
    gdf_status coarse(bool fp64)
    {
        const double e = fp64 ? 8.0 : 2.0;   // coarse-level element bytes
        gdf_status r;
        const bool raw = raw_rhs_l1;
        raw_rhs_l1 = false;
        for (int l = 1; l <= P.max_level; ++l) {
            if ((r = strip(P.list_down[l], SK_DOWN, 0, 0, nullptr, fp64, PC_COARSE, 2.25 * e, false, raw && l == 1)))
                return r;
            if ((r = strip(P.list_coarse[l], SK_COARSE_ZERO, 0, 0, nullptr, fp64, PC_COARSE, 2 * e))) return r;
            for (int k = 1; k < kCoarsePasses; ++k)
                if ((r = strip(P.list_coarse[l], SK_COARSE, (k - 1) & 1, k & 1, nullptr, fp64, PC_COARSE, 3 * e))) return r;
        }
        for (int l = P.max_level - 1; l >= 1; --l)
            if ((r = strip(P.list_up[l], SK_UP, 0, 1, nullptr, fp64, PC_COARSE, 3.25 * e))) return r;
        return GDF_OK;
    }

    gdf_status first_pass(bool fp64)
    {
        if (P.periodic) return GDF_OK;   // (the first periodic cycle starts from zero)
        const double e = fp64 ? 8.0 : 4.0, ce = fp64 ? 8.0 : 2.0;
        gdf_status r;
        const int nC = P.list_fine >= 0 ? P.lists[P.list_fine].count : 0;
        // read b, write the coarse right-hand side (a quarter per pixel), unless
        // the smoothing pass wrote it
        if (!raw_rhs_l1)
            if ((r = strip(P.list_first, SK_FIRST_RESTRICT, 0, 0, partf, fp64, PC_FIRST, e + 0.25 * ce))) return r;
        if ((r = strip(P.list_single, SK_SINGLE_ZERO, 0, 0, partf + nC, fp64, PC_COARSE, 2 * e))) return r;
        return GDF_OK;
    }

    // slice_par: F/S passes take each slice's buffer parity from its cycle
    // count (plain solve); otherwise from k (the inner solves of the mixed mode)
    // zero: the finest iterate is zero (first cycle after a restricting first pass)
    gdf_status cycle(int k, bool fp64, bool slice_par = true, bool zero = false)
    {
        if (P.periodic) return pcycle(fp64, zero);
        const double e = fp64 ? 8.0 : 4.0, ce = fp64 ? 8.0 : 2.0;
        gdf_status r;
        if ((r = coarse(fp64))) return r;
        const int nC = P.list_fine >= 0 ? P.lists[P.list_fine].count : 0;
        // read b and the black half of u (the red half is dead: the first
        // half-sweep overwrites it unread; none of u when zero), write u; read
        // the coarse correction and write the coarse right-hand side (a quarter
        // per pixel each)
        if ((r = strip(P.list_fine, zero ? SK_FINE_ZERO : SK_FINE, (k - 1) & 1, k & 1, partf, fp64,
                       zero ? PC_FINE0 : PC_FINE, (zero ? 2.0 : 2.5) * e + 0.5 * ce, slice_par)))
            return r;
        if ((r = strip(P.list_single, SK_SINGLE, (k - 1) & 1, k & 1, partf + nC, fp64, PC_COARSE, 3 * e, slice_par))) return r;
        return GDF_OK;
    }

    gdf_status read_active(bool &any)
    {
        int *h = nullptr;
        HIP_TRY(pinned_flags(P.n, h));
        HIP_TRY(hipMemcpyAsync(h, active, sizeof(int) * P.n, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        any = false;
        for (int i = 0; i < P.n; ++i) {
            active_host[i] = h[i] != 0;
            any |= active_host[i];
        }
        return GDF_OK;
    }

    // V-cycles until every slice meets tol (host checks the flags after each
    // cycle).  With first = false, continues from the current iterates.  A
    // captured schedule has no host checks: it holds `captured` cycles, which
    // frozen slices skip on the device.
    gdf_status iterate(bool fp64, bool first = true, int captured = 0)
    {
        gdf_status r;
        if (first) {
            if ((r = first_pass(fp64))) return r;   // (no iterate to check yet)
        }
        const bool z = first;   // first cycle from a zero iterate
        if (capturing) {
            // passes after the last active slice exit at once (the done flag)
            HIP_TRY(launch_done(P.n, active, done, s));
            for (int k = 1; k <= (captured ? captured : max_cycles); ++k) {
                if ((r = cycle(k, fp64, true, z && k == 1))) return r;
                if ((r = check_cycle(fp64))) return r;
                HIP_TRY(launch_done(P.n, active, done, s));
            }
            return GDF_OK;
        }
        bool any = true;
        for (int k = 1; k <= max_cycles; ++k) {
            // (a fresh solve starts its first cycle without reading the flags:
            // slices already converged skip it on the device, and the GPU does
            // not idle while the host waits for the smoothing pass)
            if (!(first && k == 1)) {
                if ((r = read_active(any))) return r;
                if (!any) break;
            }
            if ((r = cycle(k, fp64, true, z && k == 1))) return r;
            if ((r = check_cycle(fp64))) return r;
        }
        return GDF_OK;
    }

    // After the exact FP64 residual of the output: slices that stopped on the
    // in-loop (working-precision) estimate but miss tol resume iterating, as
    // long as each round shrinks their exact residual by the stall factor (a
    // slice that stops improving has reached the working precision's floor and
    // is left to the FP64-refinement re-solve).
    std::vector<double> prev_exact;
    gdf_status resume_missed(bool &any)
    {
        std::vector<SliceState> h(P.n);
        HIP_TRY(hipMemcpyAsync(h.data(), st, sizeof(SliceState) * P.n, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (prev_exact.empty()) prev_exact.assign(P.n, HUGE_VAL);
        std::vector<int> act(P.n, 0);
        any = false;
        for (int i = 0; i < P.n; ++i) {
            const bool progress = stall_ratio <= 0.0 || h[i].rel < stall_ratio * prev_exact[i];
            if (h[i].status == 0 && !h[i].stalled && std::isfinite(h[i].rel) && h[i].rel > tol &&
                h[i].cycles < max_cycles && progress) {
                act[i] = 1;
                any = true;
            }
            prev_exact[i] = h[i].rel;
        }
        if (any) {
            HIP_TRY(hipMemcpyAsync(active, act.data(), sizeof(int) * P.n, hipMemcpyHostToDevice, s));
            HIP_TRY(hipMemcpyAsync(only, act.data(), sizeof(int) * P.n, hipMemcpyHostToDevice, s));
        }
        HIP_TRY(hipStreamSynchronize(s));
        return GDF_OK;
    }
};

// Page-locked staging of the tables image, per thread: two buffers used in
// turn, each with an event recorded after its upload, so an upload never
// waits for the device unless the buffer's previous upload is still in
// flight.  (Without page-locked memory -- solve_slices_noalloc -- the image is
// copied from pageable memory and the stream synchronised, so the image can
// be released.)
struct TableStaging {
    int dev = -1;
    char *buf[2] = {nullptr, nullptr};
    size_t cap[2] = {0, 0};
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool pending[2] = {false, false};
    int next = 0;
};
thread_local TableStaging t_stage;

gdf_status upload_tables(const Plan &P, char *ws, const std::vector<SliceIO> &io, hipStream_t s)
{
    std::vector<char> img = bind_tables(P, ws, io);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    TableStaging &T = t_stage;
    if (t_no_pinned || (T.dev >= 0 && T.dev != dev)) {
        HIP_TRY(hipMemcpyAsync(ws + P.off_tables, img.data(), img.size(), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
        return GDF_OK;
    }
    T.dev = dev;
    const int i = T.next;
    if (T.pending[i]) {
        HIP_TRY(hipEventSynchronize(T.ev[i]));
        T.pending[i] = false;
    }
    if (!T.ev[i]) HIP_TRY(hipEventCreateWithFlags(&T.ev[i], hipEventDisableTiming));
    if (T.cap[i] < img.size()) {
        if (T.buf[i]) HIP_TRY(hipHostFree(T.buf[i]));
        T.buf[i] = nullptr;
        T.cap[i] = 0;
        const size_t want = std::max<size_t>(img.size(), 1 << 16);
        HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&T.buf[i]), want, hipHostMallocDefault));
        T.cap[i] = want;
    }
    std::memcpy(T.buf[i], img.data(), img.size());
    HIP_TRY(hipMemcpyAsync(ws + P.off_tables, T.buf[i], img.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(T.ev[i], s));
    T.pending[i] = true;
    T.next = i ^ 1;
    return GDF_OK;
}

gdf_status collect(const Plan &P, char *ws, hipStream_t s, gdf_slice_report *rep, double tol, int cycles_scale,
                   std::vector<SliceState> *states = nullptr)
{
    std::vector<SliceState> h(P.n);
    HIP_TRY(hipMemcpyAsync(h.data(), ws + P.off_state, sizeof(SliceState) * P.n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (states) *states = h;
    gdf_status worst = GDF_OK;
    for (int i = 0; i < P.n; ++i) {
        int status = GDF_OK;
        if (h[i].status == GDF_ENONFINITE || !std::isfinite(h[i].rel)) status = GDF_ENONFINITE;
        else if (h[i].rel > tol) status = GDF_ENOCONV;
        if (rep) {
            rep[i].vcycles = h[i].cycles * cycles_scale;
            rep[i].status = status;
            rep[i].rel_residual = h[i].rel;
            rep[i].rel_residual_init = h[i].rel_init;
        }
        if (status == GDF_ENONFINITE) worst = GDF_ENONFINITE;
        else if (status == GDF_ENOCONV && worst == GDF_OK) worst = GDF_ENOCONV;
    }
    if (worst == GDF_ENOCONV) set_err(worst, "some slices did not reach tol=%g", tol);
    if (worst == GDF_ENONFINITE) set_err(worst, "non-finite residual in some slices");
    return worst;
}

// -------------------------------------------------------------- graph cache

struct GraphEntry {
    std::vector<unsigned long long> key;
    hipGraphExec_t exec;
};
std::mutex g_graph_mu;
std::vector<GraphEntry> g_graphs;

hipGraphExec_t graph_lookup(const std::vector<unsigned long long> &key)
{
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto &e : g_graphs)
        if (e.key == key) return e.exec;
    return nullptr;
}

void graph_store(const std::vector<unsigned long long> &key, hipGraphExec_t ex)
{
    std::lock_guard<std::mutex> lk(g_graph_mu);
    if (g_graphs.size() >= 16) {
        hipGraphExecDestroy(g_graphs.front().exec);
        g_graphs.erase(g_graphs.begin());
    }
    g_graphs.push_back(GraphEntry{key, ex});
}


// ------------------------------------------------------------ solve body

struct SolveIO {
    int gs_dtype, go_dtype;
    const void *gs, *go;
    void *f;
    bool rows_ok;   // widths and g_o / f offsets fit the row-marching output pass
};

// Every width a multiple of 4 and every g_o / f row start on a four-element
// boundary (the row-marching output pass moves four elements per lane).
static bool fin_rows_ok(const std::vector<SliceIO> &io)
{
    for (const SliceIO &v : io)
        if ((v.W & 3) || (v.off_go & 3) || (v.pitch_go & 3) || (v.off_f & 3) || (v.pitch_f & 3)) return false;
    return true;
}

// FP64 iterative refinement around FP32 V-cycles.  The FP64 iterate u64 starts
// at zero; each step solves A e = r (r the FP64 residual, stored as FP32 in the
// level-0 right-hand side) with inner_cycles FP32 V-cycles from e = 0, then
// u64 += e and the FP64 residual is formed again, until every slice's FP64
// relative residual meets tol.  The right-hand side is alpha (g_s - g_o), or
// `rhs` when given (the adjoint system).
gdf_status mixed_iterate(Run &R, int gs_dtype, const void *gs, int go_dtype, const void *go,
                         const void *rhs)
{
    const Plan &P = R.P;
    gdf_status r;
    RefineArgs ra;
    ra.gs_dtype = gs_dtype;
    ra.go_dtype = go_dtype;
    ra.gs = gs;
    ra.go = go;
    ra.rhs = rhs;
    ra.io = R.io;
    ra.n_slices = P.n;
    ra.n_tiles = P.n_tiles;
    ra.levs = R.desc;
    ra.u64 = R.u64tab;
    ra.active = R.active;
    ra.part_rr = R.partd;
    ra.in_sel = 1;
    ra.e_sel = 0;
    ra.first = 1;
    // (periodic boundaries: tiles of the periodic lists, the inner solve's
    // correction in level-0 buffer 0)
    auto refine = [&]() -> hipError_t {
        ProfScope ps(PC_REFINE, 0.0, R.s, R.capturing);
        return P.periodic ? launch_prefine(ra, R.plaunch(0), R.s) : launch_refine(ra, R.s);
    };
    const int *rr_range = P.periodic ? R.r_p0 : R.r_tiles;
    HIP_TRY(refine());
    if ((r = R.finish(rr_range, nullptr, R.partd, FIN_CHECK, 0))) return r;
    const int steps = std::max(1, P.o.max_vc / P.o.inner);
    const int saved_max = R.max_cycles;
    R.max_cycles = steps;
    for (int k = 1; k <= steps; ++k) {
        if (!R.capturing) {
            bool any = true;
            if ((r = R.read_active(any))) return r;
            if (!any) break;
        }
        if ((r = R.first_pass(false))) return r;
        for (int c = 1; c <= P.o.inner; ++c)
            if ((r = R.cycle(c, false, false, c == 1))) return r;
        ra.first = 0;
        ra.in_sel = (k - 1) & 1;
        ra.e_sel = P.periodic ? 0 : P.o.inner & 1;
        HIP_TRY(refine());
        if ((r = R.finish(rr_range, nullptr, R.partd, FIN_CHECK, 1))) return r;
    }
    R.max_cycles = saved_max;
    return GDF_OK;
}

// Prepared right-hand side (prep kernel or smoothing) -> iterate -> output.
gdf_status solve_body(Run &R, const SolveIO &x)
{
    const Plan &P = R.P;
    gdf_status r;
    // algorithmic bytes per pixel of the output pass: iterate and b (or the
    // FP64 iterate), g_o, f
    const double go_b = x.go_dtype == GDF_U8 ? 1.0 : (x.go_dtype == GDF_F32 ? 4.0 : 8.0);
    const double f_b = P.o.out_dtype == GDF_F64 ? 8.0 : 4.0;
    double all_px = 0.0;
    for (int i = 0; i < P.n; ++i) all_px += (double)P.g[i].H * P.g[i].W;
    // the row-marching output pass reads g_o and writes f four elements at a time
    const size_t go_e = x.go_dtype == GDF_U8 ? 1 : (x.go_dtype == GDF_F32 ? 4 : 8);
    const bool rows = x.rows_ok && (reinterpret_cast<uintptr_t>(x.go) % (4 * go_e)) == 0 &&
                      (reinterpret_cast<uintptr_t>(x.f) % (size_t)(4 * f_b)) == 0;
    if (!P.mixed) {
        // rounds after the first resume slices whose exact residual missed tol
        // (decided on the host, or on the device inside a captured graph, which
        // holds two such rounds of two cycles each)
        for (int round = 0; round < 4; ++round) {
            if ((r = R.iterate(P.fp64, round == 0, round ? 2 : 0))) return r;
            {
                // (later rounds touch only the resumed slices: not counted)
                ProfScope ps(PC_FINALIZE, round ? 0.0 : all_px * (2.0 * P.esz + go_b + f_b), R.s, R.capturing);
                if (P.periodic) {
                    PLaunch a = R.plaunch(0);
                    a.in_sel = 0;
                    a.part_rr = R.partd;
                    HIP_TRY(launch_pfinalize(P.fp64, x.go_dtype, x.go, P.o.out_dtype, x.f, R.io, a, R.st,
                                             round ? R.only : nullptr, R.s));
                } else {
                    HIP_TRY(launch_finalize(P.fp64, rows, x.go_dtype, x.go, P.o.out_dtype, x.f, R.io, P.n,
                                            rows ? P.n_ftiles : P.n_tiles, R.desc, R.st, round ? R.only : nullptr,
                                            R.partd, R.s));
                }
            }
            if ((r = R.finish(P.periodic ? R.r_p0 : (rows ? R.r_ftiles : R.r_tiles), nullptr, R.partd, FIN_FINAL, 0)))
                return r;
            if (R.capturing) {
                if (round == 2) break;
                HIP_TRY(launch_resume_flags(P.n, R.st, R.tol, R.max_cycles, R.active, R.only, R.s));
                continue;
            }
            bool again = false;
            if ((r = R.resume_missed(again))) return r;
            if (!again) break;
        }
        return GDF_OK;
    }
    gdf_status q;
    if ((q = mixed_iterate(R, x.gs_dtype, x.gs, x.go_dtype, x.go, nullptr))) return q;
    {
        ProfScope ps(PC_FINALIZE, all_px * (8.0 + go_b + f_b), R.s, R.capturing);
        HIP_TRY(launch_finalize64(x.go_dtype, x.go, P.o.out_dtype, x.f, R.io, P.n, P.n_tiles,
                                  R.u64tab, R.st, R.desc, R.s));
    }
    return GDF_OK;
}

// ------------------------------------------------------------- autotuning
//
// A call with opts.autotune = 1 times whole solves of its own batch under
// candidate settings and keeps the fastest: first the sweep count nu per
// smoothing step (fewer sweeps per pass against more V-cycles), then every
// pairing of the fused-pass sweeps (plain or over-relaxed) with the rows per
// strip work item (tile_rows: halo overhead against the number of items in
// flight), then the coarse sweeps, the launch mode (one wave per item against
// a persistent grid) and the rows once more.  Fields the caller set
// explicitly are not tuned.  The result is
// cached per batch signature (sizes, screening weights, tolerances, precision
// and dtypes; not the data or the pointers) until gdf_release.

struct Tuned { int nu, fine_sweeps, coarse_sweeps, tile_rows, launch, sor; };
std::mutex g_tune_mu;
std::vector<std::pair<std::vector<unsigned long long>, Tuned>> g_tuned;
thread_local gdf_solve_opts g_last_tuned;
thread_local bool g_last_tuned_ok = false;

std::vector<int> tune_nus(const gdf_solve_opts &b)
{
    return b.nu ? std::vector<int>{b.nu} : std::vector<int>{2, 1};
}
std::vector<int> tune_fine_sweeps(const gdf_solve_opts &b, int nu)
{
    return b.fine_sweeps ? std::vector<int>{b.fine_sweeps} : std::vector<int>{0, 2 * nu + 1, 2 * nu + 2};
}
std::vector<int> tune_coarse_sweeps(const gdf_solve_opts &b, int nu)
{
    return b.coarse_sweeps ? std::vector<int>{b.coarse_sweeps} : std::vector<int>{0, nu};
}
std::vector<int> tune_tiles(const gdf_solve_opts &b)
{
    return b.tile_rows ? std::vector<int>{b.tile_rows} : std::vector<int>{0, 32, 64, 128, 256};
}
std::vector<int> tune_launches(const gdf_solve_opts &b)
{
    return b.launch_mode ? std::vector<int>{b.launch_mode}
                         : std::vector<int>{GDF_LAUNCH_GRID, GDF_LAUNCH_PERSISTENT};
}

gdf_solve_opts opts_or_zero(const gdf_solve_opts *o)
{
    gdf_solve_opts z;
    std::memset(&z, 0, sizeof z);
    return o ? *o : z;
}

// Largest workspace over the candidate settings (size_of(opts) per candidate),
// memoised per signature: each candidate size builds a full plan.
std::mutex g_wsz_mu;
std::vector<std::pair<std::vector<unsigned long long>, size_t>> g_wsz;

template <class SizeOf>
size_t tuned_workspace(const std::vector<unsigned long long> &key, const gdf_solve_opts &base, SizeOf size_of)
{
    {
        std::lock_guard<std::mutex> lk(g_wsz_mu);
        for (auto &e : g_wsz)
            if (e.first == key) return e.second;
    }
    size_t m = 0;
    for (int nu : tune_nus(base))
        for (int fs : tune_fine_sweeps(base, nu))
            for (int cs : tune_coarse_sweeps(base, nu))
                for (int tr : tune_tiles(base)) {
                    gdf_solve_opts c = base;
                    c.autotune = 0;
                    c.nu = nu;
                    c.fine_sweeps = fs;
                    c.coarse_sweeps = cs;
                    c.tile_rows = tr;
                    const size_t b = size_of(&c);
                    if (b == 0) return 0;
                    m = std::max(m, b);
                }
    std::lock_guard<std::mutex> lk(g_wsz_mu);
    if (g_wsz.size() >= 64) g_wsz.erase(g_wsz.begin());
    g_wsz.emplace_back(key, m);
    return m;
}

template <class Call>
gdf_status autotuned(const std::vector<unsigned long long> &key, const gdf_solve_opts &base, Call call)
{
    gdf_solve_opts best = base;
    best.autotune = 0;
    Tuned t{0, 0, 0, 0, 0, 0};
    bool have = false;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (auto &e : g_tuned)
            if (e.first == key) { t = e.second; have = true; break; }
    }
    if (!have) {
        const double inf = HUGE_VAL;
        auto timeit = [&](const gdf_solve_opts &c) -> double {
            double tmin = inf;
            for (int rep = 0; rep < 2; ++rep) {   // the first run also captures a graph
                const auto t0 = std::chrono::steady_clock::now();
                if (call(&c) != GDF_OK) return inf;
                const auto t1 = std::chrono::steady_clock::now();
                tmin = std::min(tmin, std::chrono::duration<double>(t1 - t0).count());
            }
            return tmin;
        };
        const std::vector<int> nus = tune_nus(base), tiles = tune_tiles(base), ls = tune_launches(base);
        gdf_solve_opts cur = best;
        cur.nu = nus[0];
        cur.fine_sweeps = base.fine_sweeps;
        cur.coarse_sweeps = base.coarse_sweeps;
        cur.tile_rows = tiles[0];
        cur.launch_mode = ls[0];
        double tcur = timeit(cur);
        auto try_field = [&](int gdf_solve_opts::*field, const std::vector<int> &vals) {
            for (int v : vals) {
                if (cur.*field == v) continue;
                gdf_solve_opts c = cur;
                c.*field = v;
                const double tc = timeit(c);
                if (tc < tcur) { cur = c; tcur = tc; }
            }
        };
        try_field(&gdf_solve_opts::nu, nus);
        // the fused-pass sweeps (plain counts, then 4 or 5 over-relaxed ones:
        // fewer over-relaxed sweeps can match more plain ones, so count and
        // mode change together) jointly with the item height: the best of each
        // depends on the other, and one field at a time stops short of it
        struct Sweeps { int fs, sor; };
        std::vector<Sweeps> sw;
        for (int fs : tune_fine_sweeps(base, cur.nu)) sw.push_back({fs, base.sor});
        if (!base.sor && base.precision != GDF_PREC_FP64)
            for (int fs : {4, 5})
                if (fs >= 2 * cur.nu && fs <= 2 * cur.nu + 2 && (!base.fine_sweeps || base.fine_sweeps == fs))
                    sw.push_back({fs, 1});
        for (const Sweeps &w : sw)
            for (int tr : tiles) {
                if (w.fs == cur.fine_sweeps && w.sor == cur.sor && tr == cur.tile_rows) continue;
                gdf_solve_opts c = cur;
                c.fine_sweeps = w.fs;
                c.sor = w.sor;
                c.tile_rows = tr;
                const double tc = timeit(c);
                if (tc < tcur) { cur = c; tcur = tc; }
            }
        try_field(&gdf_solve_opts::coarse_sweeps, tune_coarse_sweeps(base, cur.nu));
        try_field(&gdf_solve_opts::launch_mode, ls);
        try_field(&gdf_solve_opts::tile_rows, tiles);   // (under the launch mode picked)
        if (!(tcur < inf)) return call(&best);   // no candidate ran cleanly: report the plain call
        t = Tuned{cur.nu, cur.fine_sweeps, cur.coarse_sweeps, cur.tile_rows, cur.launch_mode, cur.sor};
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (g_tuned.size() >= 64) g_tuned.erase(g_tuned.begin());
        g_tuned.emplace_back(key, t);
    }
    best.nu = t.nu;
    best.fine_sweeps = t.fine_sweeps;
    best.coarse_sweeps = t.coarse_sweeps;
    best.tile_rows = t.tile_rows;
    best.launch_mode = t.launch;
    best.sor = t.sor;
    g_last_tuned = best;
    g_last_tuned_ok = true;
    return call(&best);
}

}  // namespace

// ===================================================================== ABI

extern "C" {

const char *gdf_last_error(void) { return g_err.c_str(); }

const char *gdf_version(void) { return "gdf-mi355x 0.1 (gfx950)"; }

void gdf_release(void)
{
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        for (auto &e : g_graphs) hipGraphExecDestroy(e.exec);
        g_graphs.clear();
    }
    {
        std::lock_guard<std::mutex> lk(g_wsz_mu);
        g_wsz.clear();
    }
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        g_plans.clear();
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned.clear();
}

int gdf_autotune_last(gdf_solve_opts *opts_host)
{
    if (!g_last_tuned_ok) return 0;
    if (opts_host) *opts_host = g_last_tuned;
    return 1;
}

void gdf_profile_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    g_prof_fine_only = on == 2;
}

void gdf_profile_reset(void)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_drain();
    for (int i = 0; i < PC_COUNT; ++i) g_prof_ms[i] = g_prof_bytes[i] = 0.0, g_prof_n[i] = 0;
}

int gdf_profile_read(const char *cls, double *ms, double *bytes)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_drain();
    for (int i = 0; i < PC_COUNT; ++i)
        if (cls && std::strcmp(cls, kProfNames[i]) == 0) {
            if (ms) *ms = g_prof_ms[i];
            if (bytes) *bytes = g_prof_bytes[i];
            return g_prof_n[i];
        }
    return -1;
}

// ---------------------------------------------------------------- fuse_stack

// Opts of the FP64-refinement re-solve of slices that stall in FP32
static Opts escalation_opts(const Opts &o)
{
    Opts m = o;
    m.prec = GDF_PREC_MIXED;
    m.max_vc = 40;
    m.inner = 3;
    m.use_graph = 0;
    m.autotune = 0;
    return m;
}

// FP32 solves reserve room to re-solve their largest slice with FP64 refinement
static size_t escalation_bytes(const Opts &o, int H, int W, double alpha)
{
    if (o.prec != GDF_PREC_FP32) return 0;
    std::shared_ptr<const Plan> Q;
    if (cached_plan(Q, 1, {H}, {W}, {alpha}, escalation_opts(o), 0, false)) return 0;
    return Q->total;
}

static gdf_status escalate(int n, const gdf_slice_desc *d, int gs_dtype, const void *gs, int go_dtype,
                           const void *go, int bc, double tol, void *f, const Opts &o, void *ws,
                           size_t ws_bytes, const std::vector<SliceState> &h, gdf_slice_report *report,
                           void *stream);
static std::vector<int> escalation_list(int n, const std::vector<SliceState> &h, double tol, int max_vc);
static std::vector<int> slice_status(int n, const std::vector<SliceState> &h, double tol);
static gdf_status worst_status(const std::vector<int> &status, double tol);
static gdf_status escalate_slices(const std::vector<int> &todo, const gdf_slice_desc *d, int gs_dtype,
                                  const void *gs, int go_dtype, const void *go, int bc, double tol, void *f,
                                  const Opts &o, void *ws, size_t ws_bytes, std::vector<int> &status,
                                  gdf_slice_report *report, void *stream);


// The slices fuse_stack solves: [z_begin, z_end) of the S (0, 0: all of them).
static gdf_status out_range(const gdf_solve_opts *opts, int S, int &z0, int &z1)
{
    z0 = opts ? opts->z_begin : 0;
    z1 = opts ? opts->z_end : 0;
    if (z0 == 0 && z1 == 0) z1 = S;
    if (z0 < 0 || z1 > S || z0 >= z1)
        return set_err(GDF_EINVAL, "z_begin, z_end must satisfy 0 <= z_begin < z_end <= S (got %d, %d, S = %d)", z0,
                       z1, S);
    return GDF_OK;
}

static gdf_status fuse_validate(const uint8_t *stack, int S, int H, int W, long long pr, long long ps,
                                double alpha, int bc, double tol, double sxy, double sz,
                                const void *f, const gdf_solve_opts *opts, Opts &o)
{
    gdf_status r;
    if ((r = parse_opts(opts, o))) return r;
    if (S < 1 || H < 1 || W < 1) return set_err(GDF_EINVAL, "S, H, W must be >= 1 (got %d, %d, %d)", S, H, W);
    if (W > kMaxWidth) return set_err(GDF_EINVAL, "W must be <= %d (got %d)", kMaxWidth, W);
    if (!stack || !f) return set_err(GDF_EINVAL, "stack and f must be non-null");
    if (pr < W || ps < (long long)H * pr)
        return set_err(GDF_EINVAL, "pitch_row must be >= W and pitch_slice >= H * pitch_row");
    if (!(alpha > 0.0) || !std::isfinite(alpha)) return set_err(GDF_EINVAL, "alpha must be finite and > 0 (got %g)", alpha);
    if ((r = check_common(bc, tol))) return r;
    if (o.sor && bc == GDF_BC_PERIODIC)
        return set_err(GDF_EUNSUPPORTED, "opts.sor: the periodic multigrid has no over-relaxed sweeps");
    if (!(sxy >= 0.0) || !(sz >= 0.0) || !std::isfinite(sxy) || !std::isfinite(sz))
        return set_err(GDF_EINVAL, "sigma_xy and sigma_z must be finite and >= 0");
    if (std::floor(3.0 * sxy) > 7 || std::floor(3.0 * sz) > 12)
        return set_err(GDF_EUNSUPPORTED, "smoothing radius beyond 7 (xy) or 12 (z) taps is not supported");
    return GDF_OK;
}

static gdf_status fuse_plan(std::shared_ptr<const Plan> &P, int S, int H, int W, double alpha, const Opts &o,
                            bool need_gs, bool periodic = false)
{
    std::vector<int> Hs(S, H), Ws(S, W);
    std::vector<double> al(S, alpha);
    return cached_plan(P, S, Hs, Ws, al, o, S, need_gs, periodic);
}

static size_t fuse_workspace_plain(int S_all, int H, int W, const gdf_solve_opts *opts)
{
    Opts o;
    if (parse_opts(opts, o)) return 0;
    if (S_all < 1 || H < 1 || W < 1) return 0;
    int z0, z1;
    if (out_range(opts, S_all, z0, z1)) return 0;
    const int S = z1 - z0;   // the slices solved
    std::shared_ptr<const Plan> P, Q;
    if (fuse_plan(P, S, H, W, 1.0, o, o.prec == GDF_PREC_MIXED)) return 0;
    // the hierarchy depth depends on alpha; size for the deepest (smallest alpha)
    if (fuse_plan(Q, S, H, W, 1e-12, o, o.prec == GDF_PREC_MIXED)) return 0;
    // FP32: room to re-solve one slice with FP64 refinement, beside that
    // slice's smoothed values (re-computed for the re-solve)
    const size_t esc = o.prec == GDF_PREC_FP32 ? align_up((size_t)H * W * sizeof(float)) + escalation_bytes(o, H, W, 1e-12)
                                               : 0;
    return std::max({P->total, Q->total, esc});
}

// ------------------------------------------------- gradient through smoothing

static size_t transpose_tmp_bytes(int S, int H, int W)
{
    return ((size_t)S * H * W * sizeof(float) + 255) / 256 * 256;
}

size_t gdf_smooth_transpose_workspace_size(int S, int H, int W)
{
    if (S < 1 || H < 1 || W < 1) return 0;
    return 2 * transpose_tmp_bytes(S, H, W) + sizeof(float) * ((size_t)S + H + W);
}

gdf_status smooth_transpose(const float *grad_dev, int S, int H, int W, double sigma_xy, double sigma_z,
                            float *out_dev, const float *add_dev, void *workspace, size_t ws_bytes, void *stream)
{
    if (S < 1 || H < 1 || W < 1) return set_err(GDF_EINVAL, "S, H, W must be >= 1 (got %d, %d, %d)", S, H, W);
    if (!grad_dev || !out_dev || !workspace) return set_err(GDF_EINVAL, "grad, out and workspace must be non-null");
    if (grad_dev == out_dev || grad_dev == add_dev) return set_err(GDF_EINVAL, "out and add must not alias grad");
    if (!(sigma_xy >= 0.0) || !(sigma_z >= 0.0) || !std::isfinite(sigma_xy) || !std::isfinite(sigma_z))
        return set_err(GDF_EINVAL, "sigma_xy and sigma_z must be finite and >= 0");
    const int rxy = sigma_xy > 0 ? (int)std::floor(3.0 * sigma_xy) : 0;
    const int rz = sigma_z > 0 ? (int)std::floor(3.0 * sigma_z) : 0;
    if (rxy > 7 || rz > 12)
        return set_err(GDF_EUNSUPPORTED, "smoothing radius beyond 7 (xy) or 12 (z) taps is not supported");
    const size_t need = gdf_smooth_transpose_workspace_size(S, H, W);
    if (ws_bytes < need) return set_err(GDF_ENOMEM, "workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
    // taps exp(-d^2 / 2 sigma^2) and the per-axis in-range weight sums
    double wxy[8] = {0}, wz[16] = {0};
    for (int d = 0; d <= rxy; ++d) wxy[d] = sigma_xy > 0 ? std::exp(-(double)d * d / (2 * sigma_xy * sigma_xy)) : 1.0;
    for (int d = 0; d <= rz; ++d) wz[d] = sigma_z > 0 ? std::exp(-(double)d * d / (2 * sigma_z * sigma_z)) : 1.0;
    float wxyf[8], wzf[16];
    for (int d = 0; d < 8; ++d) wxyf[d] = (float)wxy[d];
    for (int d = 0; d < 16; ++d) wzf[d] = (float)wz[d];
    char *ws = static_cast<char *>(workspace);
    float *tmp = reinterpret_cast<float *>(ws);
    float *tmp2 = reinterpret_cast<float *>(ws + transpose_tmp_bytes(S, H, W));
    float *inv_d = reinterpret_cast<float *>(ws + 2 * transpose_tmp_bytes(S, H, W));
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(launch_transpose_tables(inv_d, S, H, W, rxy, rz, wxy, wz, s));
    HIP_TRY(launch_smooth_transpose(grad_dev, out_dev, add_dev, tmp, tmp2, inv_d, S, H, W, rxy, rz, wxyf, wzf, s));
    return GDF_OK;
}

// Runs body (the whole device schedule of a call) as a graph: captured on
// the stream the first time for this key (sizes, pointers, stream and
// options), then replayed.  Convergence is decided on the device inside the
// graph (per-slice flags); the host reads the states once, afterwards.
static gdf_status run_captured(const std::vector<unsigned long long> &key, Run &R, const Opts &o,
                               const std::function<gdf_status()> &body)
{
    hipStream_t s = R.s;
    hipGraphExec_t ex = graph_lookup(key);
    if (!ex) {
        if (o.launch == GDF_LAUNCH_PERSISTENT) {
            strip_prepare(o.csw, o.fsw, R.P.fp64);
            if (o.csw_auto) strip_prepare(o.nu, o.fsw, R.P.fp64);
        }
        R.capturing = true;
        HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        gdf_status q = body();
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(s, &g);
        R.capturing = false;
        if (q) {
            if (g) hipGraphDestroy(g);
            return q;
        }
        if (ec != hipSuccess) return set_err(GDF_EDEVICE, "graph capture failed: %s", hipGetErrorString(ec));
        const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (ei != hipSuccess) return set_err(GDF_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(ei));
        graph_store(key, ex);
    }
    HIP_TRY(hipGraphLaunch(ex, s));
    return GDF_OK;
}

size_t gdf_fuse_workspace_size(int S, int H, int W, const gdf_solve_opts *opts)
{
    const gdf_solve_opts b = opts_or_zero(opts);
    if (b.autotune != 1) return fuse_workspace_plain(S, H, W, opts);
    std::vector<unsigned long long> key;
    key_push(key, 0);
    for (int v : {S, H, W, b.precision, b.max_vcycles, b.out_dtype, b.use_graph, b.inner_cycles, b.nu, b.fine_sweeps, b.coarse_sweeps, b.tile_rows,
                  b.launch_mode, b.robust, b.z_begin, b.z_end, b.sor})
        key_push(key, v);
    return tuned_workspace(key, b, [&](const gdf_solve_opts *c) { return fuse_workspace_plain(S, H, W, c); });
}

static gdf_status fuse_stack_plain(const uint8_t *stack, int S, int H, int W, long long pitch_row,
                                   long long pitch_slice, double alpha, int bc, double tol, double sigma_xy,
                                   double sigma_z, void *f, void *g_smooth, const gdf_solve_opts *opts,
                                   void *workspace, size_t ws_bytes, gdf_slice_report *report, void *stream);

gdf_status fuse_stack(const uint8_t *stack, int S, int H, int W, long long pitch_row,
                      long long pitch_slice, double alpha, int bc, double tol, double sigma_xy,
                      double sigma_z, void *f, void *g_smooth, const gdf_solve_opts *opts,
                      void *workspace, size_t ws_bytes, gdf_slice_report *report, void *stream)
{
    const gdf_solve_opts b = opts_or_zero(opts);
    if (b.autotune != 1)
        return fuse_stack_plain(stack, S, H, W, pitch_row, pitch_slice, alpha, bc, tol, sigma_xy, sigma_z, f,
                                g_smooth, opts, workspace, ws_bytes, report, stream);
    Opts o;
    gdf_status r;
    if ((r = fuse_validate(stack, S, H, W, pitch_row, pitch_slice, alpha, bc, tol, sigma_xy, sigma_z, f, opts, o)))
        return r;
    std::vector<unsigned long long> key;
    key_push(key, 0);
    for (int v : {S, H, W, bc, b.precision, b.max_vcycles, b.out_dtype, b.use_graph, b.inner_cycles, b.nu, b.fine_sweeps, b.coarse_sweeps,
                  b.tile_rows, b.launch_mode, g_smooth ? 1 : 0, b.robust, b.z_begin, b.z_end, b.sor})
        key_push(key, v);
    for (double v : {alpha, tol, sigma_xy, sigma_z}) key_push(key, v);
    return autotuned(key, b, [&](const gdf_solve_opts *c) {
        return fuse_stack_plain(stack, S, H, W, pitch_row, pitch_slice, alpha, bc, tol, sigma_xy, sigma_z, f,
                                g_smooth, c, workspace, ws_bytes, report, stream);
    });
}

// Smoothing arguments of a stack (taps, renormalisation tables, tiling); the
// caller sets the outputs (b_u, level-1 right-hand side, g_s, partial sums).
static SmoothArgs smooth_args(const uint8_t *stack, int S, int H, int W, long long pitch_row, long long pitch_slice,
                              double sigma_xy, double sigma_z, double alpha, int robust)
{
    SmoothArgs a;
    std::memset(&a, 0, sizeof a);
    a.stack = stack;
    a.pitch_row = pitch_row;
    a.pitch_slice = pitch_slice;
    a.S = S;
    a.H = H;
    a.W = W;
    a.rxy = sigma_xy > 0 ? (int)std::floor(3.0 * sigma_xy) : 0;
    a.rz = sigma_z > 0 ? (int)std::floor(3.0 * sigma_z) : 0;
    for (int d = 0; d <= a.rxy; ++d)
        a.wxy[d] = sigma_xy > 0 ? std::exp(-(double)d * d / (2 * sigma_xy * sigma_xy)) : 1.0;
    for (int d = 0; d <= a.rz; ++d)
        a.wz[d] = sigma_z > 0 ? std::exp(-(double)d * d / (2 * sigma_z * sigma_z)) : 1.0;
    a.alpha = alpha;
    for (int d = 0; d < 8; ++d) a.wxy_f[d] = (float)a.wxy[d];
    for (int d = 0; d < 16; ++d) a.wz_f[d] = (float)a.wz[d];
    a.alpha_f = (float)alpha;
    a.robust = robust;
    for (int lo = 0; lo <= 12; ++lo)
        for (int hi = 0; hi <= 12; ++hi) {
            double w = 0.0;
            for (int d = -lo; d <= hi; ++d)
                if (d >= -a.rz && d <= a.rz) w += a.wz[d < 0 ? -d : d];
            a.inv_wz[lo][hi] = 1.0 / w;
            a.inv_wz_f[lo][hi] = (float)(1.0 / w);
        }
    a.tiles_x = (W + kSmoothTileW - 1) / kSmoothTileW;
    a.tiles_y = (H + kSmoothTileH - 1) / kSmoothTileH;
    a.z_lo = 0;
    a.z_hi = S;
    return a;
}

static gdf_status fuse_stack_plain(const uint8_t *stack_all, int S_all, int H, int W, long long pitch_row,
                                   long long pitch_slice, double alpha, int bc, double tol, double sigma_xy,
                                   double sigma_z, void *f, void *g_smooth, const gdf_solve_opts *opts,
                                   void *workspace, size_t ws_bytes, gdf_slice_report *report, void *stream)
{
    Opts o;
    gdf_status r;
    if ((r = fuse_validate(stack_all, S_all, H, W, pitch_row, pitch_slice, alpha, bc, tol, sigma_xy, sigma_z, f, opts,
                           o)))
        return r;
    if (!workspace) return set_err(GDF_EINVAL, "workspace must be non-null");
    // The slices solved, [z0, z1): S of them at stack (the first).  The
    // smoothing reads the stack from zv0, the first slice in their windows.
    int z0, z1;
    if ((r = out_range(opts, S_all, z0, z1))) return r;
    const int S = z1 - z0;
    const int rz = sigma_z > 0 ? (int)std::floor(3.0 * sigma_z) : 0;
    const int zv0 = std::max(0, z0 - rz), zv1 = std::min(S_all, z1 + rz);
    const uint8_t *stack = stack_all + (long long)z0 * pitch_slice;
    const bool mixed = o.prec == GDF_PREC_MIXED;
    std::shared_ptr<const Plan> PP;
    const bool periodic = bc == GDF_BC_PERIODIC;
    if ((r = fuse_plan(PP, S, H, W, alpha, o, mixed && !g_smooth, periodic))) return r;
    const Plan &P = *PP;
    if (ws_bytes < P.total)
        return set_err(GDF_ENOMEM, "workspace too small: %zu bytes given, %zu needed", ws_bytes, P.total);
    // g_o is the stack itself; f (and the FP32 copy of g_s when kept) are contiguous
    std::vector<SliceIO> io = P.io;
    for (int z = 0; z < S; ++z) {
        io[z].off_go = (long long)z * pitch_slice;
        io[z].pitch_go = pitch_row;
        io[z].off_f = (long long)z * H * W;
        io[z].pitch_f = W;
        io[z].off_gs = (long long)z * H * W;
        io[z].pitch_gs = W;
    }
    char *ws = static_cast<char *>(workspace);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((r = upload_tables(P, ws, io, s))) return r;
    Run R(P, ws, s);
    R.tol = tol;
    R.max_cycles = o.max_vc;
    R.stall_ratio = o.prec == GDF_PREC_FP32 ? kStallRatio : 0.0;

    // smoothing writes the level-0 right-hand side of every slice
    SmoothArgs a = smooth_args(stack_all + (long long)zv0 * pitch_slice, zv1 - zv0, H, W, pitch_row, pitch_slice,
                               sigma_xy, sigma_z, alpha, o.robust);
    a.z_lo = z0 - zv0;
    a.z_hi = z1 - zv0;
    void *gs_used = g_smooth ? g_smooth : (mixed ? (void *)(ws + P.off_gscopy) : nullptr);
    a.gs_out = gs_used;
    a.gs_zlo = a.z_lo;
    a.gs_zhi = a.z_hi;
    // a uniform stack: every slice has the same arena block, so the level-0
    // right-hand sides are equally spaced
    a.b0 = ws + P.off_arena + P.g[0].off_b[0];
    a.b_slice_stride = S > 1 ? (long long)((P.g[1].off_b[0] - P.g[0].off_b[0]) / P.esz) : 0;
    for (int z = 1; z < S; ++z)
        if ((long long)(P.g[z].off_b[0] - P.g[0].off_b[0]) != a.b_slice_stride * z * P.esz)
            return set_err(GDF_EDEVICE, "internal: non-uniform arena layout of a stack");
    a.b_pitch = P.g[0].pitch[0];
    // FP32 hierarchy: the smoothing pass also restricts b_u to level 1, so the
    // solve's first pass has nothing left to do
    if (!P.fp64 && !mixed && !periodic && P.g[0].nlev >= 2 && P.csz == 2) {
        a.bc0 = ws + P.off_arena + P.g[0].off_b[1];
        a.bc_slice_stride = S > 1 ? (long long)((P.g[1].off_b[1] - P.g[0].off_b[1]) / P.csz) : 0;
        a.bc_pitch = P.g[0].pitch[1];
        for (int z = 1; z < S; ++z)
            if ((long long)(P.g[z].off_b[1] - P.g[0].off_b[1]) != a.bc_slice_stride * z * P.csz) a.bc0 = nullptr;
    }
    a.part_bb = R.partd;
    a.part_b0 = R.partd2;
    a.part_bs = R.partd3;
    SolveIO x;
    x.gs_dtype = P.fp64 ? GDF_F64 : GDF_F32;
    x.gs = gs_used;
    x.go_dtype = GDF_U8;
    x.go = stack;
    x.f = f;
    x.rows_ok = fin_rows_ok(io);

    auto body = [&]() -> gdf_status {
        {
            ProfScope ps(PC_SMOOTH,
                         (double)H * W * ((zv1 - zv0) + S * (P.esz + (gs_used ? P.esz : 0) + (a.bc0 ? 0.25 * P.csz : 0.0))),
                         s, R.capturing);
            HIP_TRY(launch_smooth(P.fp64, a, s));
        }
        R.raw_rhs_l1 = a.bc0 != nullptr;
        if (periodic) {
            // the norms of Eq. (1)'s right-hand side with the periodic Laplacian,
            // from the b_u the smoothing wrote and the stack
            HIP_TRY(launch_pprep(P.fp64, P.fp64 ? GDF_F64 : GDF_F32, nullptr, GDF_U8, stack, R.io, R.plaunch(0),
                                 R.partd, R.partd2, R.partd3, s));
            HIP_TRY(launch_finish_rhs(P.n, R.r_p0, R.partd, R.partd2, R.partd3, R.st, s));
        } else {
            HIP_TRY(launch_finish_rhs(P.n, R.r_smooth, R.partd, R.partd2, R.partd3, R.st, s));
        }
        return solve_body(R, x);
    };
    if (!o.use_graph) {
        if ((r = body())) return r;
    } else {
        std::vector<unsigned long long> key;
        key_push(key, 3);
        for (int v : {S_all, H, W, z0, z1, bc, o.prec, o.max_vc, o.nu, o.csw, o.csw_auto ? 1 : 0, o.out_dtype, o.tile_rows, o.inner, o.launch,
                      o.fsw, o.robust, o.sor})
            key_push(key, v);
        for (double v : {alpha, tol, sigma_xy, sigma_z}) key_push(key, v);
        key_push(key, pitch_row);
        key_push(key, pitch_slice);
        for (const void *p : {(const void *)stack_all, (const void *)f, (const void *)g_smooth, (const void *)ws,
                              (const void *)s})
            key_push(key, p);
        if ((r = run_captured(key, R, o, body))) return r;
        if (!report) return GDF_OK;   // asynchronous: nothing waits for the device
    }
    std::vector<SliceState> h;
    const gdf_status st = collect(P, ws, s, report, tol, mixed ? o.inner : 1, &h);
    if (st != GDF_ENOCONV || o.prec != GDF_PREC_FP32) return st;
    // Slices left above tol at the FP32 floor are re-solved by FP64 refinement
    // from their g_s (FP32) and the stack: from the returned g_s when there is
    // one, else one slice at a time from g_s smoothed again into the front of
    // the workspace (the re-solve uses the rest of it).
    std::vector<gdf_slice_desc> d(S);
    for (int z = 0; z < S; ++z) {
        d[z].H = H;
        d[z].W = W;
        d[z].alpha = alpha;
        d[z].off_gs = g_smooth ? (long long)z * H * W : 0;
        d[z].pitch_gs = W;
        d[z].off_go = (long long)z * pitch_slice;
        d[z].pitch_go = pitch_row;
        d[z].off_f = (long long)z * H * W;
        d[z].pitch_f = W;
    }
    if (g_smooth)
        return escalate(S, d.data(), GDF_F32, g_smooth, GDF_U8, stack, bc, tol, f, o, workspace, ws_bytes, h, report,
                        stream);
    std::vector<int> status = slice_status(S, h, tol);
    const size_t gs1 = align_up((size_t)H * W * sizeof(float));
    if (ws_bytes <= gs1) return worst_status(status, tol);
    SmoothArgs a1 = a;   // g_s of one slice only: no b_u, no level-1 restriction, no partial sums
    a1.b0 = nullptr;
    a1.bc0 = nullptr;
    a1.part_bb = a1.part_b0 = a1.part_bs = nullptr;
    a1.gs_out = ws;
    for (int z : escalation_list(S, h, tol, o.max_vc)) {
        a1.z_lo = a1.gs_zlo = z + z0 - zv0;
        a1.z_hi = a1.gs_zhi = z + z0 - zv0 + 1;
        HIP_TRY(launch_smooth(false, a1, s));
        if ((r = escalate_slices({z}, d.data(), GDF_F32, ws, GDF_U8, stack, bc, tol, f, o, ws + gs1, ws_bytes - gs1,
                                 status, report, stream)))
            return r;
    }
    return worst_status(status, tol);
}

// -------------------------------------------------------------- solve_slices

static gdf_status slices_validate(int n, const gdf_slice_desc *d, double tol, int bc,
                                  const gdf_solve_opts *opts, Opts &o, std::vector<int> &H,
                                  std::vector<int> &W, std::vector<double> &al)
{
    gdf_status r;
    if ((r = parse_opts(opts, o))) return r;
    if (n < 1 || !d) return set_err(GDF_EINVAL, "n must be >= 1 and desc non-null");
    if ((r = check_common(bc, tol))) return r;
    if (o.sor && bc == GDF_BC_PERIODIC)
        return set_err(GDF_EUNSUPPORTED, "opts.sor: the periodic multigrid has no over-relaxed sweeps");
    H.resize(n);
    W.resize(n);
    al.resize(n);
    for (int i = 0; i < n; ++i) {
        const gdf_slice_desc &s = d[i];
        if (s.H < 1 || s.W < 1) return set_err(GDF_EINVAL, "slice %d: H, W must be >= 1", i);
        if (s.W > kMaxWidth) return set_err(GDF_EINVAL, "slice %d: W must be <= %d (got %d)", i, kMaxWidth, s.W);
        if (!(s.alpha > 0.0) || !std::isfinite(s.alpha))
            return set_err(GDF_EINVAL, "slice %d: alpha must be finite and > 0 (got %g)", i, s.alpha);
        if (s.off_gs < 0 || s.off_go < 0 || s.off_f < 0)
            return set_err(GDF_EINVAL, "slice %d: offsets must be >= 0", i);
        if (s.pitch_gs < s.W || s.pitch_go < s.W || s.pitch_f < s.W)
            return set_err(GDF_EINVAL, "slice %d: row pitches must be >= W", i);
        H[i] = s.H;
        W[i] = s.W;
        al[i] = s.alpha;
    }
    return GDF_OK;
}

static std::vector<SliceIO> slice_io(const Plan &P, const gdf_slice_desc *d)
{
    std::vector<SliceIO> io = P.io;
    for (int i = 0; i < P.n; ++i) {
        io[i].off_gs = d[i].off_gs;
        io[i].pitch_gs = d[i].pitch_gs;
        io[i].off_go = d[i].off_go;
        io[i].pitch_go = d[i].pitch_go;
        io[i].off_f = d[i].off_f;
        io[i].pitch_f = d[i].pitch_f;
    }
    return io;
}

static size_t solve_workspace_plain(int n, const gdf_slice_desc *d, const gdf_solve_opts *opts)
{
    Opts o;
    std::vector<int> H, W;
    std::vector<double> al;
    if (slices_validate(n, d, 0.5, GDF_BC_NEUMANN, opts, o, H, W, al)) return 0;
    std::shared_ptr<const Plan> P;
    if (cached_plan(P, n, H, W, al, o, 0, false)) return 0;
    int big = 0;
    for (int i = 1; i < n; ++i)
        if ((long long)H[i] * W[i] > (long long)H[big] * W[big]) big = i;
    return std::max(P->total, escalation_bytes(o, H[big], W[big], al[big]));
}

size_t gdf_solve_workspace_size(int n, const gdf_slice_desc *d, const gdf_solve_opts *opts)
{
    const gdf_solve_opts b = opts_or_zero(opts);
    if (b.autotune != 1) return solve_workspace_plain(n, d, opts);
    if (n < 1 || !d) return 0;
    std::vector<unsigned long long> key;
    key_push(key, 1);
    for (int v : {n, b.precision, b.max_vcycles, b.out_dtype, b.use_graph, b.inner_cycles, b.nu, b.fine_sweeps, b.coarse_sweeps, b.tile_rows,
                  b.launch_mode, b.sor})
        key_push(key, v);
    for (int i = 0; i < n; ++i) {
        key_push(key, d[i].H);
        key_push(key, d[i].W);
        key_push(key, d[i].alpha);
    }
    return tuned_workspace(key, b, [&](const gdf_solve_opts *c) { return solve_workspace_plain(n, d, c); });
}

size_t gdf_backward_workspace_size(int n, const gdf_slice_desc *d, const gdf_solve_opts *opts)
{
    // FP32 adjoints run inside FP64 refinement (see solve_slices_backward)
    gdf_solve_opts o;
    std::memset(&o, 0, sizeof o);
    if (opts) o = *opts;
    if (o.precision != GDF_PREC_FP64) o.precision = GDF_PREC_MIXED;
    return gdf_solve_workspace_size(n, d, &o);
}

static gdf_status solve_slices_plain(int n, const gdf_slice_desc *d, int gs_dtype, const void *gs,
                                     int go_dtype, const void *go, int bc, double tol, void *f,
                                     const gdf_solve_opts *opts, void *workspace, size_t ws_bytes,
                                     gdf_slice_report *report, void *stream);

// Slices to re-solve with FP64 refinement after an FP32 solve: finite, above
// tol, and stopped before the cycle cap (stalled at the FP32 floor, or resumed
// without progress).  A slice that used up max_vcycles keeps GDF_ENOCONV: the
// caller's cap holds.
static std::vector<int> escalation_list(int n, const std::vector<SliceState> &h, double tol, int max_vc)
{
    std::vector<int> todo;
    for (int i = 0; i < n; ++i) {
        const bool bad = h[i].status == GDF_ENONFINITE || !std::isfinite(h[i].rel);
        if (!bad && h[i].rel > tol && (h[i].stalled || h[i].cycles < max_vc)) todo.push_back(i);
    }
    return todo;
}

static std::vector<int> slice_status(int n, const std::vector<SliceState> &h, double tol)
{
    std::vector<int> status(n);
    for (int i = 0; i < n; ++i) {
        const bool bad = h[i].status == GDF_ENONFINITE || !std::isfinite(h[i].rel);
        status[i] = bad ? GDF_ENONFINITE : (h[i].rel > tol ? GDF_ENOCONV : GDF_OK);
    }
    return status;
}

static gdf_status worst_status(const std::vector<int> &status, double tol)
{
    gdf_status worst = GDF_OK;
    for (int v : status) {
        if (v == GDF_ENONFINITE) worst = GDF_ENONFINITE;
        else if (v == GDF_ENOCONV && worst == GDF_OK) worst = GDF_ENOCONV;
    }
    if (worst == GDF_ENOCONV) set_err(worst, "some slices did not reach tol=%g", tol);
    else if (worst == GDF_ENONFINITE) set_err(worst, "non-finite residual in some slices");
    else g_err.clear();
    return worst;
}

static gdf_solve_opts escalation_call_opts(const Opts &o)
{
    const Opts mo = escalation_opts(o);
    gdf_solve_opts m;
    std::memset(&m, 0, sizeof m);
    m.precision = mo.prec;
    m.max_vcycles = mo.max_vc;
    m.nu = mo.nu;
    m.fine_sweeps = mo.fsw;
    m.coarse_sweeps = mo.csw;
    m.out_dtype = mo.out_dtype;
    m.tile_rows = mo.tile_rows;
    m.inner_cycles = mo.inner;
    m.launch_mode = mo.launch;
    return m;
}

// Re-solves the slices `todo` from zero by FP32 V-cycles inside FP64
// iterative refinement, in groups that fit the workspace, writing their f in
// place and updating status[] and the report.
static gdf_status escalate_slices(const std::vector<int> &todo, const gdf_slice_desc *d, int gs_dtype,
                                  const void *gs, int go_dtype, const void *go, int bc, double tol, void *f,
                                  const Opts &o, void *ws, size_t ws_bytes, std::vector<int> &status,
                                  gdf_slice_report *report, void *stream)
{
    const gdf_solve_opts m = escalation_call_opts(o);
    size_t k = 0;
    while (k < todo.size()) {
        std::vector<gdf_slice_desc> g;
        std::vector<int> idx;
        for (; k < todo.size(); ++k) {
            g.push_back(d[todo[k]]);
            const size_t need = solve_workspace_plain((int)g.size(), g.data(), &m);
            if (need == 0 || need > ws_bytes) {
                g.pop_back();
                break;
            }
            idx.push_back(todo[k]);
        }
        if (g.empty()) {   // this slice alone does not fit: it keeps GDF_ENOCONV
            ++k;
            continue;
        }
        std::vector<gdf_slice_report> sub(g.size());
        const gdf_status r = solve_slices_plain((int)g.size(), g.data(), gs_dtype, gs, go_dtype, go, bc, tol, f,
                                                &m, ws, ws_bytes, sub.data(), stream);
        if (r != GDF_OK && r != GDF_ENOCONV && r != GDF_ENONFINITE) return r;
        for (size_t j = 0; j < idx.size(); ++j) {
            const int i = idx[j];
            status[i] = sub[j].status;
            if (report) {
                report[i].vcycles += sub[j].vcycles;
                report[i].status = sub[j].status;
                report[i].rel_residual = sub[j].rel_residual;
            }
        }
    }
    return GDF_OK;
}

static gdf_status escalate(int n, const gdf_slice_desc *d, int gs_dtype, const void *gs, int go_dtype,
                           const void *go, int bc, double tol, void *f, const Opts &o, void *ws,
                           size_t ws_bytes, const std::vector<SliceState> &h, gdf_slice_report *report,
                           void *stream)
{
    std::vector<int> status = slice_status(n, h, tol);
    const gdf_status r = escalate_slices(escalation_list(n, h, tol, o.max_vc), d, gs_dtype, gs, go_dtype, go, bc,
                                         tol, f, o, ws, ws_bytes, status, report, stream);
    if (r) return r;
    return worst_status(status, tol);
}

gdf_status solve_slices(int n, const gdf_slice_desc *d, int gs_dtype, const void *gs, int go_dtype,
                        const void *go, int bc, double tol, void *f, const gdf_solve_opts *opts,
                        void *workspace, size_t ws_bytes, gdf_slice_report *report, void *stream)
{
    const gdf_solve_opts b = opts_or_zero(opts);
    if (b.autotune != 1)
        return solve_slices_plain(n, d, gs_dtype, gs, go_dtype, go, bc, tol, f, opts, workspace, ws_bytes,
                                  report, stream);
    Opts o;
    std::vector<int> H, W;
    std::vector<double> al;
    gdf_status r;
    if ((r = slices_validate(n, d, tol, bc, opts, o, H, W, al))) return r;
    std::vector<unsigned long long> key;
    key_push(key, 1);
    for (int v : {n, bc, gs_dtype, go_dtype, b.precision, b.max_vcycles, b.out_dtype, b.use_graph,
                  b.inner_cycles, b.nu, b.fine_sweeps, b.coarse_sweeps, b.tile_rows, b.launch_mode, b.sor})
        key_push(key, v);
    key_push(key, tol);
    for (int i = 0; i < n; ++i) {
        key_push(key, d[i].H);
        key_push(key, d[i].W);
        key_push(key, d[i].alpha);
    }
    return autotuned(key, b, [&](const gdf_solve_opts *c) {
        return solve_slices_plain(n, d, gs_dtype, gs, go_dtype, go, bc, tol, f, c, workspace, ws_bytes, report,
                                  stream);
    });
}

static gdf_status solve_slices_plain(int n, const gdf_slice_desc *d, int gs_dtype, const void *gs,
                                     int go_dtype, const void *go, int bc, double tol, void *f,
                                     const gdf_solve_opts *opts, void *workspace, size_t ws_bytes,
                                     gdf_slice_report *report, void *stream)
{
    Opts o;
    std::vector<int> H, W;
    std::vector<double> al;
    gdf_status r;
    if ((r = slices_validate(n, d, tol, bc, opts, o, H, W, al))) return r;
    if (gs_dtype != GDF_F32 && gs_dtype != GDF_F64) return set_err(GDF_EINVAL, "gs_dtype must be GDF_F32 or GDF_F64");
    if (go_dtype != GDF_U8 && go_dtype != GDF_F32 && go_dtype != GDF_F64)
        return set_err(GDF_EINVAL, "go_dtype must be GDF_U8, GDF_F32 or GDF_F64");
    if (!gs || !go || !f) return set_err(GDF_EINVAL, "gs, go and f must be non-null");
    if (!workspace) return set_err(GDF_EINVAL, "workspace must be non-null");
    std::shared_ptr<const Plan> PP;
    if ((r = cached_plan(PP, n, H, W, al, o, 0, false, bc == GDF_BC_PERIODIC))) return r;
    const Plan &P = *PP;
    if (ws_bytes < P.total)
        return set_err(GDF_ENOMEM, "workspace too small: %zu bytes given, %zu needed", ws_bytes, P.total);
    char *ws = static_cast<char *>(workspace);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const std::vector<SliceIO> io = slice_io(P, d);
    if ((r = upload_tables(P, ws, io, s))) return r;
    Run R(P, ws, s);
    R.tol = tol;
    R.max_cycles = o.max_vc;
    R.stall_ratio = o.prec == GDF_PREC_FP32 ? kStallRatio : 0.0;
    SolveIO x{gs_dtype, go_dtype, gs, go, f, fin_rows_ok(io)};

    auto body = [&]() -> gdf_status {
        {
            ProfScope ps(PC_PREP, 0.0, s, R.capturing);
            if (P.periodic)
                HIP_TRY(launch_pprep(P.fp64, gs_dtype, gs, go_dtype, go, R.io, R.plaunch(0), R.partd, R.partd2,
                                     R.partd3, s));
            else
                HIP_TRY(launch_prep(P.fp64, gs_dtype, gs, go_dtype, go, R.io, n, P.n_tiles, R.desc, R.partd,
                                    R.partd2, R.partd3, s));
        }
        HIP_TRY(launch_finish_rhs(n, P.periodic ? R.r_p0 : R.r_tiles, R.partd, R.partd2, R.partd3, R.st, s));
        return solve_body(R, x);
    };

    if (!o.use_graph) {
        if ((r = body())) return r;
    } else {
        std::vector<unsigned long long> key;
        key_push(key, n);
        key_push(key, (const void *)ws);
        key_push(key, gs);
        key_push(key, go);
        key_push(key, (const void *)f);
        key_push(key, (const void *)s);
        key_push(key, gs_dtype);
        key_push(key, go_dtype);
        key_push(key, tol);
        key_push(key, o.prec);
        key_push(key, o.max_vc);
        key_push(key, o.nu);
        key_push(key, o.csw);
        key_push(key, o.csw_auto ? 1 : 0);
        key_push(key, o.out_dtype);
        key_push(key, o.tile_rows);
        key_push(key, o.inner);
        key_push(key, o.launch);
        key_push(key, o.fsw);
        key_push(key, o.sor);
        for (int i = 0; i < n; ++i) {
            key_push(key, d[i].H);
            key_push(key, d[i].W);
            key_push(key, d[i].alpha);
            key_push(key, d[i].off_gs);
            key_push(key, d[i].off_go);
            key_push(key, d[i].off_f);
            key_push(key, d[i].pitch_gs);
            key_push(key, d[i].pitch_go);
            key_push(key, d[i].pitch_f);
        }
        if ((r = run_captured(key, R, o, body))) return r;
        if (!report) return GDF_OK;   // asynchronous: nothing waits for the device
    }
    std::vector<SliceState> h;
    const gdf_status st = collect(P, ws, s, report, tol, o.prec == GDF_PREC_MIXED ? o.inner : 1, &h);
    if (st == GDF_ENOCONV && o.prec == GDF_PREC_FP32)
        return escalate(n, d, gs_dtype, gs, go_dtype, go, bc, tol, f, o, workspace, ws_bytes, h, report, stream);
    return st;
}

// ----------------------------------------------------- solve_slices_backward

static gdf_status backward_plain(int n, const gdf_slice_desc *d, int dtype, const void *grad_f,
                                 const void *f, const void *gs, int bc, double tol, void *grad_gs,
                                 void *grad_go, double *grad_alpha, double *grad_alpha_sum, const gdf_solve_opts *opts,
                                 void *workspace, size_t ws_bytes, gdf_slice_report *report,
                                 void *stream);

gdf_status solve_slices_backward(int n, const gdf_slice_desc *d, int dtype, const void *grad_f,
                                 const void *f, const void *gs, int bc, double tol, void *grad_gs,
                                 void *grad_go, double *grad_alpha, double *grad_alpha_sum,
                                 const gdf_solve_opts *opts, void *workspace, size_t ws_bytes,
                                 gdf_slice_report *report, void *stream)
{
    const gdf_solve_opts b = opts_or_zero(opts);
    if (b.autotune != 1)
        return backward_plain(n, d, dtype, grad_f, f, gs, bc, tol, grad_gs, grad_go, grad_alpha, grad_alpha_sum, opts,
                              workspace, ws_bytes, report, stream);
    Opts o;
    std::vector<int> H, W;
    std::vector<double> al;
    gdf_status r;
    if ((r = slices_validate(n, d, tol, bc, opts, o, H, W, al))) return r;
    std::vector<unsigned long long> key;
    key_push(key, 2);
    for (int v : {n, bc, dtype, b.precision, b.max_vcycles, b.inner_cycles, b.nu, b.fine_sweeps, b.coarse_sweeps, b.tile_rows, b.launch_mode, b.sor})
        key_push(key, v);
    key_push(key, tol);
    for (int i = 0; i < n; ++i) {
        key_push(key, d[i].H);
        key_push(key, d[i].W);
        key_push(key, d[i].alpha);
    }
    return autotuned(key, b, [&](const gdf_solve_opts *c) {
        return backward_plain(n, d, dtype, grad_f, f, gs, bc, tol, grad_gs, grad_go, grad_alpha, grad_alpha_sum, c,
                              workspace, ws_bytes, report, stream);
    });
}

static gdf_status backward_plain(int n, const gdf_slice_desc *d, int dtype, const void *grad_f,
                                 const void *f, const void *gs, int bc, double tol, void *grad_gs,
                                 void *grad_go, double *grad_alpha, double *grad_alpha_sum, const gdf_solve_opts *opts,
                                 void *workspace, size_t ws_bytes, gdf_slice_report *report,
                                 void *stream)
{
    Opts o;
    std::vector<int> H, W;
    std::vector<double> al;
    gdf_status r;
    if ((r = slices_validate(n, d, tol, bc, opts, o, H, W, al))) return r;
    if (dtype != GDF_F32 && dtype != GDF_F64) return set_err(GDF_EINVAL, "dtype must be GDF_F32 or GDF_F64");
    if ((dtype == GDF_F64) != (o.prec == GDF_PREC_FP64))
        return set_err(GDF_EINVAL, "dtype must match opts.precision (F32 <-> FP32 or MIXED, F64 <-> FP64)");
    // FP32 data: the adjoint right-hand side grad_f is typically rough and its
    // solution has large smooth components, beyond what an FP32 iterate can
    // resolve to tol; it is solved with FP32 V-cycles inside FP64 refinement
    if (dtype == GDF_F32) o.prec = GDF_PREC_MIXED;
    if (!grad_f || !f || !gs) return set_err(GDF_EINVAL, "grad_f, f and gs must be non-null");
    if (!workspace) return set_err(GDF_EINVAL, "workspace must be non-null");
    std::shared_ptr<const Plan> PP;
    if ((r = cached_plan(PP, n, H, W, al, o, 0, false, bc == GDF_BC_PERIODIC))) return r;
    const Plan &P = *PP;
    if (ws_bytes < P.total)
        return set_err(GDF_ENOMEM, "workspace too small: %zu bytes given, %zu needed", ws_bytes, P.total);
    char *ws = static_cast<char *>(workspace);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((r = upload_tables(P, ws, slice_io(P, d), s))) return r;
    Run R(P, ws, s);
    R.tol = tol;
    R.max_cycles = o.max_vc;
    {
        ProfScope ps(PC_PREP, 0.0, s, false);
        HIP_TRY(launch_prep_adjoint(P.fp64, grad_f, R.io, n, P.n_tiles, R.desc, R.partd, R.partd3, s));
    }
    HIP_TRY(launch_finish_rhs(n, R.r_tiles, R.partd, R.partd, R.partd3, R.st, s));
    if (P.mixed) {
        if ((r = mixed_iterate(R, dtype, nullptr, GDF_F32, nullptr, grad_f))) return r;
    } else {
        if ((r = R.iterate(P.fp64))) return r;
    }
    {
        ProfScope ps(PC_ADJOINT, 0.0, s, false);
        if (P.periodic) {
            PLaunch a = R.plaunch(0);
            a.in_sel = 0;
            HIP_TRY(launch_padjoint(P.fp64, gs, f, grad_gs, grad_go, R.io, n, a, R.st, P.mixed ? R.u64tab : nullptr,
                                    R.partd, s));
        } else {
            HIP_TRY(launch_adjoint_assemble(P.fp64, gs, f, grad_gs, grad_go, R.io, n, P.n_tiles, R.desc, R.st,
                                            P.mixed ? R.u64tab : nullptr, R.partd, s));
        }
    }
    if ((r = R.finish(P.periodic ? R.r_p0 : R.r_tiles, nullptr, R.partd, FIN_SUM, 0))) return r;
    if (grad_alpha_sum) HIP_TRY(launch_sum_aux(n, R.st, grad_alpha_sum, s));
    std::vector<SliceState> h(n);
    HIP_TRY(hipMemcpyAsync(h.data(), R.st, sizeof(SliceState) * n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (grad_alpha)
        for (int i = 0; i < n; ++i) grad_alpha[i] = h[i].aux;
    return collect(P, ws, s, report, tol, 1);
}

// ------------------------------------------------------ solve_slices_noalloc

}  // extern "C"

// Device scratch of solve_slices_noalloc: one array per GPU (the runtime
// places it when the library's code object is loaded on that GPU) and held
// until the process ends.  Host code never passes `gdf_scratch` itself to the
// device (on the host the name is only a stand-in for the symbol): its device
// address on each GPU comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char gdf_scratch[GDF_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu[kMaxDevices];   // one call at a time per device (they share its scratch)
void *g_scratch_ptr[kMaxDevices];       // device address per device, set under that device's lock

}  // namespace

extern "C" {

gdf_status solve_slices_noalloc(int n, const gdf_slice_desc *d, int gs_dtype, const void *gs, int go_dtype,
                                const void *go, int bc, double tol, void *f, const gdf_solve_opts *opts,
                                gdf_slice_report *report, void *stream)
{
    const gdf_solve_opts b = opts_or_zero(opts);
    if (b.use_graph)
        return set_err(GDF_EUNSUPPORTED, "solve_slices_noalloc: use_graph is not available (instantiating a graph "
                                         "allocates device memory)");
    // argument checks and the scratch size come first, on the host
    Opts o;
    std::vector<int> H, W;
    std::vector<double> al;
    gdf_status r;
    if ((r = slices_validate(n, d, tol, bc, opts, o, H, W, al))) return r;
    const size_t need = gdf_solve_workspace_size(n, d, opts);
    if (need == 0) return set_err(GDF_EINVAL, "solve_slices_noalloc: invalid batch");
    if (need > (size_t)GDF_NOALLOC_SCRATCH_BYTES)
        return set_err(GDF_ENOMEM, "solve_slices_noalloc: the batch needs %zu bytes of scratch, the static scratch "
                                   "holds %zu (use solve_slices with a workspace)",
                       need, (size_t)GDF_NOALLOC_SCRATCH_BYTES);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0;
    if (s) HIP_TRY(hipStreamGetDevice(s, &dev));
    else HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return set_err(GDF_EDEVICE, "solve_slices_noalloc: device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu[dev]);
    if (!g_scratch_ptr[dev]) {
        // once per device, with that device current
        int cur = 0;
        HIP_TRY(hipGetDevice(&cur));
        if (cur != dev) HIP_TRY(hipSetDevice(dev));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(gdf_scratch));
        if (cur != dev) HIP_TRY(hipSetDevice(cur));
        if (e != hipSuccess || !p)
            return set_err(GDF_EDEVICE, "solve_slices_noalloc: hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    t_no_pinned = true;
    r = solve_slices(n, d, gs_dtype, gs, go_dtype, go, bc, tol, f, opts, g_scratch_ptr[dev],
                     (size_t)GDF_NOALLOC_SCRATCH_BYTES, report, stream);
    t_no_pinned = false;
    return r;
}

}  // extern "C"
