// Internal declarations shared by the host driver and the HIP kernels of the
// gradient-domain fusion library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace gdf {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kStripCols = 128;    // columns covered by one wave (2 per lane)
constexpr int kWavesPerBlock = 4;  // independent waves per workgroup
constexpr int kMaxLevels = 16;
constexpr int kMaxWidth = 1 << 22;  // widest slice (keeps an item's rows within 32-bit offsets)

#ifdef __HIPCC__
// Logical tile of this workgroup in a 1-D grid of nb workgroups.  The hardware
// hands workgroup b to XCD b % 8; remapping gives each XCD a contiguous range of
// tiles, so tiles that share halo rows and columns run on the same XCD at about
// the same time and meet in its L2.  A tail of fewer than 8 groups keeps its
// order.
__device__ __forceinline__ long long xcd_tile(long long b, long long nb)
{
    const long long nb8 = nb >> 3;
    if (b >= nb8 * 8) return b;
    return (b & 7) * nb8 + (b >> 3);
}

// ------------------------------------------------------- buffer access ---

// Raw buffer resource over `bytes` bytes from `base` (no stride or swizzle;
// dword 3 selects plain dword access on this GPU family).  The address of an
// access is base + row offset (a scalar) + lane offset; a lane offset at or
// past `bytes` reads zero and drops a store.  So a lane is masked by its
// offset and a whole row by a zero-sized resource, without a branch.
typedef __amdgpu_buffer_rsrc_t Rsrc;
__device__ __forceinline__ Rsrc make_rsrc(const void *base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
// a lane offset past every window (the host keeps an item's rows below 2^31 bytes)
constexpr unsigned kNoLane = 0x80000000u;

template <typename X> struct Buf;
template <> struct Buf<unsigned short> {
    __device__ static unsigned short ld(Rsrc r, unsigned vo, unsigned so)
    {
        return __builtin_amdgcn_raw_buffer_load_b16(r, (int)vo, (int)so, 0);
    }
    __device__ static void st(unsigned short v, Rsrc r, unsigned vo, unsigned so)
    {
        __builtin_amdgcn_raw_buffer_store_b16(v, r, (int)vo, (int)so, 0);
    }
};
template <> struct Buf<unsigned> {
    __device__ static unsigned ld(Rsrc r, unsigned vo, unsigned so)
    {
        return __builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, 0);
    }
    __device__ static void st(unsigned v, Rsrc r, unsigned vo, unsigned so)
    {
        __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)vo, (int)so, 0);
    }
};
template <> struct Buf<float> {
    __device__ static float ld(Rsrc r, unsigned vo, unsigned so) { return __uint_as_float(Buf<unsigned>::ld(r, vo, so)); }
    __device__ static void st(float v, Rsrc r, unsigned vo, unsigned so) { Buf<unsigned>::st(__float_as_uint(v), r, vo, so); }
};
typedef unsigned U2 __attribute__((ext_vector_type(2)));
typedef unsigned U4 __attribute__((ext_vector_type(4)));
template <typename X, typename R> struct BufBits {   // 8- and 16-byte values
    __device__ static X ld(Rsrc r, unsigned vo, unsigned so)
    {
        if constexpr (sizeof(X) == 8) return __builtin_bit_cast(X, __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, 0));
        else return __builtin_bit_cast(X, __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, (int)so, 0));
    }
    __device__ static void st(X v, Rsrc r, unsigned vo, unsigned so)
    {
        if constexpr (sizeof(X) == 8) __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(R, v), r, (int)vo, (int)so, 0);
        else __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(R, v), r, (int)vo, (int)so, 0);
    }
};
template <> struct Buf<double> : BufBits<double, U2> {};
#endif  // __HIPCC__

// One multigrid level of one slice.  Arrays are row-major with row pitch
// `pitch` (elements, even, >= W + 1 for odd W) so that a lane's two-column
// vector access never leaves the allocation.  Exception: the iterate of
// level 0 (outside the periodic multigrid) stores each row by colour, pixel
// (x, y) at element x / 2 of the half (x + y) & 1 of row y, each half pitch / 2
// elements long: a red-black sweep pass then reads the one colour it needs as
// contiguous runs.
struct LevelDesc {
    void *u[2];      // iterate ping-pong buffers at this level
    void *b;         // right-hand side at this level (scaled units, see below)
    void *ec;        // coarse correction to prolongate (level+1 iterate), or null
    void *bc;        // coarse right-hand side to restrict into (level+1), or null
    int H, W, pitch;
    int Hc, Wc, pitch_c;
    double sigma;    // alpha * h^2 with h = 2^level: the level's scaled screening term
    double wxL, wyL; // width of the last column / height of the last row relative to a full
                     // cell (ceil-halving leaves a partial last cell when a side is odd)
    const double *bshift;  // level 0: per-slice mean of b subtracted on load (null: none)
    int slice;       // slice index (flags, partial sums)
    int pad_;
    // level 1: the level-0 mean; a right-hand side restricted from the unshifted
    // level-0 one (StripLaunch::raw_rhs) has each cell's children's share of it
    // subtracted on load
    const double *bshift_fine;
};

// A strip work item: one wave processes columns [x0 - G, x0 - G + 128) of
// rows [y0 - G, y1 + G) and owns output columns [x0, x0 + 128 - 2G) x rows [y0, y1).
struct Item {
    int lev;   // index into the LevelDesc table
    int x0;
    int y0;
    int y1;
    int pidx;  // slot of this item's partial sums (a slice's slots are contiguous)
};

enum ResidMode { RES_NONE = 0, RES_NORM = 1, RES_RESTRICT = 2, RES_BOTH = 3 };

// Launch parameters of one strip pass.
struct StripLaunch {
    const LevelDesc *levs;
    const Item *items;
    int n_items;
    int n_fast;              // items [0, n_fast) run the interior variant
    int n_rows_in;           // items [n_fast, n_rows_in) the column-edge variant, the rest the guarded one
    int in_sel, out_sel;     // which u buffer is read / written
    const int *cycles;       // if non-null: read buffer (cycles[slice] & 1), write the other
    int cycles_stride;       // ints between consecutive slices' counters
    const int *active;       // per-slice "still iterating" flags
    const int *done;         // if non-null and set: no slice is iterating (every wave exits at once)
    float2 *partials;        // per-item partial sums (r^2, r) (RES_NORM / RES_BOTH)
    int raw_rhs;             // level 1: b holds sums of unshifted level-0 values (see LevelDesc)
};

// Strip kernel variants (template instances live in mg_kernels.hip).
enum StripKind {
    SK_FIRST_RESTRICT,  // finest, first pass of a solve from zero: restrict b (no sweeps)
    SK_FINE,         // prolongate, fsw sweeps, residual -> norm + restrict (finest, fused up+down)
    SK_DOWN,         // zero start, csw sweeps, restrict (coarse levels, down leg)
    SK_UP,           // prolongate, csw sweeps (coarse levels, up leg)
    SK_COARSE_ZERO,  // zero start, 2 sweeps (coarsest level)
    SK_COARSE,       // 2 sweeps (coarsest level)
    SK_SINGLE_ZERO,  // zero start, 2 sweeps, residual -> norm (single-level slices)
    SK_SINGLE,       // 2 sweeps, residual -> norm
    SK_FINE_ZERO,    // as SK_FINE from a zero iterate (the first cycle after SK_FIRST_RESTRICT)
    SK_COUNT
};

// Halo (G) of a strip kind: stages after the load, plus one for prolongation,
// rounded up to even.  Valid output width per strip is 128 - 2G.
int strip_halo(StripKind k, int csw, int fsw);

// Enqueue one strip pass (one launch).  Items [0, a.n_fast) stay clear of
// the slice's edges (rows y0 - G .. y1 + G in [1, H - 2], columns x0 - G ..
// x0 - G + 127 in [1, W - 2]) and run the code without row guards and edge
// masks; items [a.n_fast, a.n_rows_in) have such rows but touch a column edge
// (no row guards, per-lane masks); the others run the guarded code.  csw: sweeps per smoothing step of
// the coarse passes; fsw: sweeps of the fused finest pass
// (SK_FINE).  fp64 selects double precision.  persistent: the grid is capped
// at the workgroups resident on the device at once and each wave loops over
// the list's items; otherwise one wave per item.  sor: the over-relaxed
// instances of SK_FINE / SK_FINE_ZERO (FP32, fsw 4 or 5; any other pass or
// setting is an error).
hipError_t launch_strip(StripKind k, int csw, int fsw, bool fp64, bool persistent, const StripLaunch &a,
                        hipStream_t s, bool sor = false);

// Waves of a strip kernel variant that the device holds at once (occupancy x
// SIMDs); 0 if the runtime cannot tell (no device).
int strip_resident_waves(StripKind k, int csw, int fsw, bool fp64);

// Resolves the persistent grid sizes of every strip kernel variant for nu,
// fsw and the precision (device queries; call before a stream capture begins).
void strip_prepare(int csw, int fsw, bool fp64);

// ---- per-slice reductions and flags ------------------------------------

struct SliceState {
    double bb;          // ||b||^2 of Eq. (1) (f-form right-hand side)
    double rr;          // ||r||^2 at the last check
    double rel;         // sqrt(rr / bb)
    double rel_init;    // residual of f = g_o relative to b
    double aux;         // FIN_SUM result
    double npx;         // pixels in the slice (set by the host)
    double alpha;       // screening weight (set by the host)
    double shift;       // constant-mode correction mean(r) / alpha of the last check
    double bmean;       // mean of the level-0 right-hand side (subtracted on load)
    double uoff;        // bmean / alpha: the solution's mean, added back at the end
    int cycles;         // coarse-grid corrections applied
    int status;         // 0 ok / iterating, GDF_ENONFINITE ...
    int stalled;        // 1: stopped because a cycle no longer reduced the residual
    int pad_;
};

enum FinishMode {
    FIN_BB = 0,       // store the sum as ||b||^2
    FIN_CHECK = 1,    // in-loop residual: store rr/rel, count the cycle, clear `active` when done
    FIN_FINAL = 2,    // residual of the returned f: store rr/rel
    FIN_INIT = 3,     // ||b_u||^2: rel_init = sqrt(sum / bb)
    FIN_SUM = 4,      // plain sum into state.aux (e.g. dLoss/dalpha)
    FIN_MEAN = 5      // sum of b: bmean = sum / npx, uoff = bmean / alpha
};

// Sum the partials of each slice over [range[2s], range[2s+1]) in a fixed
// order (deterministic) and update the slice state and flags.
// partials_f: strip partials (r^2, r); partials_d: FP64 tile partials.
// FIN_CHECK with strip partials also records the constant-mode correction.
// FIN_CHECK with stall_ratio > 0: from the second counted cycle on, a slice
// whose residual shrank by less than that factor in one cycle (while still
// above tol) stops with state.stalled = 1 (the working precision's floor).
// partials_d2 (with partials_d, FIN_CHECK): FP64 partial sums of r, giving
// the constant-mode correction as the strip partials do.
hipError_t launch_finish(int n_slices, const int *range, const float2 *partials_f,
                         const double *partials_d, const double *partials_d2, int mode, double tol,
                         int max_cycles, int count_cycle, double stall_ratio, SliceState *state, int *active,
                         hipStream_t s);

// FIN_BB, FIN_INIT and FIN_MEAN of one right-hand side in one launch.
hipError_t launch_finish_rhs(int n_slices, const int *range, const double *pbb, const double *pb0,
                             const double *pbs, SliceState *state, hipStream_t s);

// After the exact residual of the output (FIN_FINAL): slices whose FP64
// relative residual still exceeds tol, with cycles left and finite state,
// get active = only = 1 (resume iterating, re-form f); others get 0.
// done = 1 when no slice's active flag is set, else 0 (one workgroup).  Lets
// the passes of a captured schedule that outlast the last active slice exit
// at their first instruction.
hipError_t launch_done(int n_slices, const int *active, int *done, hipStream_t s);

hipError_t launch_resume_flags(int n_slices, const SliceState *state, double tol, int max_cycles,
                               int *active, int *only, hipStream_t s);

// ---- elementwise / simple stencil kernels --------------------------------

struct SliceIO {        // per-slice user-buffer view (element offsets/pitches)
    long long off_gs, pitch_gs;
    long long off_go, pitch_go;
    long long off_f, pitch_f;
    double alpha;
    int H, W;
    int lev0;           // LevelDesc index of the slice's finest level
    int tiles_x;        // 64-wide tiles per row (for the simple 2D kernels)
    long long tile_begin;  // first tile index of this slice
    int ftiles_x;       // blocks per row of the row-marching output pass
    int pad_;
    long long ftile_begin;  // first such block of this slice
};

// b_u = alpha (g_s - g_o) into level 0 b, and FP64 partials of
// ||alpha g_s + L g_o||^2, ||b_u||^2 and sum(b_u) per tile.
hipError_t launch_prep(bool fp64, int gs_dtype, const void *gs, int go_dtype, const void *go,
                       const SliceIO *io_dev, int n_slices, long long n_tiles,
                       const LevelDesc *levs, double *part_bb, double *part_b0, double *part_bs,
                       hipStream_t s);

// f = g_o + u (out dtype), FP64 partials of ||b_u - A u||^2 per tile.  The
// level-0 iterate of slice s is buffer (state[s].cycles & 1).
// With `only` non-null, tiles of slices with only[s] == 0 are skipped.
// rows: the row-marching kernel over blocks of kFinCols x kFinRows (n_tiles
// of those; every width a multiple of 4 and the g_o and f rows aligned to four
// elements), else the quad kernel over 64 x 16 tiles.
constexpr int kFinCols = 256, kFinRows = 64;
hipError_t launch_finalize(bool fp64, bool rows, int go_dtype, const void *go, int out_dtype, void *f,
                           const SliceIO *io_dev, int n_slices, long long n_tiles,
                           const LevelDesc *levs, const SliceState *state, const int *only,
                           double *part_rr, hipStream_t s);

// Adjoint right-hand side: b = grad_f (converted), partials of ||grad_f||^2 and sum(grad_f).
hipError_t launch_prep_adjoint(bool fp64, const void *grad_f, const SliceIO *io_dev, int n_slices,
                               long long n_tiles, const LevelDesc *levs, double *part_bb,
                               double *part_bs, hipStream_t s);

// From lambda (level-0 iterate): grad_gs = alpha lambda, grad_go = L lambda,
// partials of lambda . (g_s - f).  Buffers share the dtype of the solve.
// With u64 non-null, lambda is the FP64 iterate of the mixed solve (buffer
// state[s].cycles & 1) instead of the level-0 working-precision iterate.
hipError_t launch_adjoint_assemble(bool fp64, const void *gs, const void *f, void *grad_gs,
                                   void *grad_go, const SliceIO *io_dev, int n_slices,
                                   long long n_tiles, const LevelDesc *levs,
                                   const SliceState *state, double *const *u64, double *part_da,
                                   hipStream_t s);

// Mixed precision refinement step: u64_out = u64_in + e (e = level-0 FP32
// iterate, buffer e_sel; skipped when first), r = alpha (g_s - g_o) - A u64_out
// in FP64, written as FP32 into level-0 b, partials of ||r||^2.
struct RefineArgs {
    int gs_dtype, go_dtype;
    const void *gs, *go;
    const void *rhs;         // if non-null: b = rhs (dtype gs_dtype, indexed like f) instead of
                             // alpha (g_s - g_o) -- the adjoint system A lambda = grad_f
    const SliceIO *io;
    int n_slices;
    long long n_tiles;
    const LevelDesc *levs;   // FP32 hierarchy
    double *const *u64;      // [2][n_slices] device table of FP64 iterates (pitch = level-0 pitch)
    int in_sel, e_sel;       // which FP64 buffer is read; which FP32 level-0 buffer holds e
    int first;               // 1: no correction to add (u64_in = 0)
    const int *active;
    double *part_rr;
};
hipError_t launch_refine(const RefineArgs &a, hipStream_t s);

// Mixed precision output: f = g_o + u64 (buffer state[s].cycles & 1).
hipError_t launch_finalize64(int go_dtype, const void *go, int out_dtype, void *f,
                             const SliceIO *io_dev, int n_slices, long long n_tiles,
                             double *const *u64, const SliceState *state, const LevelDesc *levs,
                             hipStream_t s);

// ---- periodic boundaries ---------------------------------------------------
//
// Slices with wrap-around (periodic) boundaries run a plain multigrid of their
// own (periodic_kernels.hip): the same levels and finite-volume operators as
// the Neumann hierarchy, with the neighbours of the first and last row and
// column taken across the wrap, one launch per half-sweep (red-black, from one
// buffer into the other, so cells of one colour that meet across the wrap of
// an odd side read each other's previous values), a residual and restriction
// pass, and a prolongation pass.  Every level is stored in the arithmetic
// type.  Work is split into tiles of kPTileW x kPTileH cells of one level of
// one slice (items); a list holds one level's items of every slice, slice by
// slice, so per-slice partial sums occupy contiguous slots.
constexpr int kPTileW = 64, kPTileH = 16;
struct PItem {
    int lev;     // LevelDesc index
    int slice;   // slice index (SliceIO, flags)
    int x0, y0;  // tile origin at that level
};
struct PLaunch {
    const LevelDesc *levs;
    const PItem *items;
    int n_items;
    const int *active;
    int in_sel, out_sel;   // u buffers read and written (smoothing); the buffer used (others)
    int colour;            // smoothing: cells with (x + y) % 2 == colour are updated
    int zero_in;           // smoothing: the input iterate is zero (not read)
    int coarse_sel;        // prolongation: the coarse level's buffer
    double *part_rr, *part_r;   // level-0 residual: per-item sums of r^2 and r
};
// Buffer element types (gdf_dtype values of the public header).
enum { GDF_DT_U8 = 0, GDF_DT_F32 = 1, GDF_DT_F64 = 2 };
// One red-black half-sweep of a level (items of that level); level0: the
// items are on level 0 (stored in the arithmetic type, coarse levels of an
// FP32 hierarchy in bfloat16).
hipError_t launch_psmooth_level(bool fp64, bool level0, const PLaunch &a, hipStream_t s);
// residual of a level restricted into the next level's right-hand side
// (items of the coarser level: each coarse cell sums its children's
// residuals); from_level0: the finer level is level 0
hipError_t launch_prestrict_level(bool fp64, bool from_level0, const PLaunch &a, hipStream_t s);
// level-0 residual norms (r^2 and r per item; items of level 0)
hipError_t launch_pnorm(bool fp64, const PLaunch &a, hipStream_t s);
// u (buffer in_sel) += bilinear prolongation of the next level's iterate
// (buffer coarse_sel); items of the finer level; into_level0: that is level 0
hipError_t launch_pprolong_level(bool fp64, bool into_level0, const PLaunch &a, hipStream_t s);
// b_u = alpha (g_s - g_o) into level-0 b, partials of ||alpha g_s + L g_o||^2,
// ||b_u||^2, sum(b_u), with the periodic L; items of level 0
hipError_t launch_pprep(bool fp64, int gs_dtype, const void *gs, int go_dtype, const void *go, const SliceIO *io,
                        const PLaunch &a, double *part_bb, double *part_b0, double *part_bs, hipStream_t s);
// f = g_o + u (+ uoff + shift) from the level-0 buffer a.in_sel, FP64 partials
// of the residual ||b_u - A u||^2; slices with only[s] == 0 skipped (only non-null)
hipError_t launch_pfinalize(bool fp64, int go_dtype, const void *go, int out_dtype, void *f, const SliceIO *io,
                            const PLaunch &a, const SliceState *st, const int *only, hipStream_t s);
// mixed refinement step with the periodic operator (as launch_refine; the
// FP32 correction is in level-0 buffer e_sel)
hipError_t launch_prefine(const RefineArgs &r, const PLaunch &a, hipStream_t s);
// adjoint assembly with the periodic L (as launch_adjoint_assemble; lambda in
// level-0 buffer a.in_sel, or the FP64 iterate u64[(cycles & 1) * n + s] when
// u64 is non-null)
hipError_t launch_padjoint(bool fp64, const void *gs, const void *f, void *grad_gs, void *grad_go,
                           const SliceIO *io, int n_slices, const PLaunch &a, const SliceState *st,
                           double *const *u64, double *part_da, hipStream_t s);

// ---- smoothing ------------------------------------------------------------

constexpr int kSmoothWaves = 8;   // waves per smoothing workgroup (one partial-sum slot each)
#ifndef GDF_SMOOTH_TILE_H
#define GDF_SMOOTH_TILE_H 24
#endif
// smoothing tile: one workgroup per kSmoothTileW x kSmoothTileH tile of every slice
constexpr int kSmoothTileW = 64, kSmoothTileH = GDF_SMOOTH_TILE_H;
static_assert(kSmoothTileH % kSmoothWaves == 0, "whole rows per thread");

struct SmoothArgs {
    const uint8_t *stack;
    long long pitch_row, pitch_slice;
    int S, H, W;
    int rxy, rz;
    double wxy[8];        // in-plane taps (0..rxy)
    double wz[16];        // cross-slice taps (0..rz)
    double alpha;
    float wxy_f[8];       // the same taps rounded to FP32 (FP32 kernel: kept in scalar registers)
    float wz_f[16];
    float alpha_f;
    int z_lo, z_hi;       // the output slices: [z_lo, z_hi) of the S (the others only feed
                          // their cross-slice windows); b_u, the level-1 right-hand side and
                          // the partial sums of slice z go to index z - z_lo
    void *gs_out;         // optional smoothed slices (contiguous [gs_zhi - gs_zlo][H][W])
    int gs_zlo, gs_zhi;   // output slices [gs_zlo, gs_zhi) are stored into gs_out (slice z at z - gs_zlo)
    void *b0;                 // level-0 right-hand side of slice 0 (b_u is written there);
                              // null: neither b_u nor the partial sums are stored
    long long b_slice_stride; // elements between consecutive slices' level-0 right-hand sides
    int b_pitch;              // its row pitch (elements)
    // 1 / (sum of the z taps inside the stack) for an output slice with lo
    // taps below it and hi above it inside the stack: inv_wz[lo][hi], lo, hi <= rz
    double inv_wz[13][13];
    float inv_wz_f[13][13];
    double *part_bb;      // [z_hi - z_lo][tiles] partial ||alpha g_s + L g_o||^2
    double *part_b0;      // [z_hi - z_lo][tiles] partial ||b_u||^2
    double *part_bs;      // [z_hi - z_lo][tiles] partial sum(b_u)
    int tiles_x, tiles_y;
    // optional (FP32): level-1 right-hand side (bfloat16) of slice 0, written as
    // the sum of each coarse cell's children's b_u (no mean removed); slices are
    // bc_slice_stride elements apart, rows bc_pitch
    void *bc0;
    long long bc_slice_stride;
    int bc_pitch;
    int robust;           // robust cross-slice averaging (FP32 only)
};

hipError_t launch_smooth(bool fp64, const SmoothArgs &a, hipStream_t s);

// Transpose of the smoothing for FP32 gradients: out = K (g / D) (see
// smooth_transpose.hip); tmp holds S H W floats, inv_d the tables 1 / Dz (S),
// 1 / Dy (H), 1 / Dx (W) in that order; wxy[0..7] and wz[0..15] the taps.
// 1 / D tables of the smoothing transpose (W + H + S floats at inv_d), from
// the in-plane (radius rxy <= 7) and cross-slice (rz <= 15) taps in FP64.
hipError_t launch_transpose_tables(float *inv_d, int S, int H, int W, int rxy, int rz, const double *wxy,
                                   const double *wz, hipStream_t s);
// add (nullable, may be out itself): out = K (g / D) + add.  tmp2: a second
// S H W buffer for the one-voxel passes.
hipError_t launch_smooth_transpose(const float *g, float *out, const float *add, float *tmp, float *tmp2,
                                   const float *inv_d, int S, int H, int W, int rxy, int rz, const float *wxy,
                                   const float *wz, hipStream_t s);
// dst[0] = sum of state[i].aux over the slices, in slice order (one thread)
hipError_t launch_sum_aux(int n_slices, const SliceState *state, double *dst, hipStream_t s);

}  // namespace gdf
