// Anisotropic Gaussian smoothing of a uint8 stack across slices (Section
// III-A), truncated at three standard deviations per axis (Implementation
// subsection), renormalised over the taps that fall inside the stack.  The
// kernel and the in-stack box are both products over the axes, so the
// renormalised 3D sum factors into three 1D passes, each divided by its own
// in-range weight sum.
//
// One workgroup of 8 waves owns a 64 x 24 tile of every slice (three rows per
// thread) and marches through the stack.  While it blurs slice z along x and
// y, the raw tile of slice z + 1 (with an in-plane halo) is already in flight
// as 4-byte loads held in registers, waited for only when it is written to
// LDS at the end of the step; the raw tiles of the slices between the current output and input
// slice stay in an LDS byte ring (they also give the Laplacian of the original
// slice at output time, with no second read from HBM).  Blurred planes go into
// a register ring of 2 rz + 1 planes; the z blur of an output slice is a
// weighted sum over that ring.  The output is written straight into the
// right-hand side of the solve, b_u = alpha (I1 - I0), together with per-tile
// partial sums of ||alpha I1 + L I0||^2 (the norm of Eq. (1)'s right-hand
// side), ||b_u||^2 and sum(b_u).  The smoothed stack is written only when asked.
#pragma once
#include "internal.h"

namespace gdf {

constexpr int kSTX = kSmoothTileW, kSTY = kSmoothTileH, kMaxRxy = 7;
constexpr int kRawW = 80;                 // bytes per raw row: x in [X0 - 8, X0 + 72)
constexpr int kRawDw = kRawW / 4;         // 20 dwords per raw row
constexpr int kRawHMax = kSTY + 2 * kMaxRxy;
constexpr int kSThreads = 64 * kSmoothWaves;               // threads per workgroup
constexpr int kSRows = kSTY / kSmoothWaves;                 // output rows per thread
constexpr int kPrefetch = (kRawHMax * kRawDw + kSThreads - 1) / kSThreads;   // dwords per thread

// Sum over the 64 lanes of a wave, returned to every lane: row sums with
// four full-row DPP adds (pair and quad swaps, half-row and row mirrors; each
// folds into one add), then the rows combined with the lane-swap moves
// (16-lane rows, then 32-lane halves): after a swap of v with itself one result
// holds the even row (lower half) and the other the odd row (upper half) of
// every pair, so their sum is the pair's total in all its lanes.
template <int CTRL> __device__ __forceinline__ float dpp_row(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
__device__ __forceinline__ float wave_sum(float v)
{
    v += dpp_row<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_row<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_row<0x141>(v);   // row_half_mirror
    v += dpp_row<0x140>(v);   // row_mirror
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    const auto h = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(h[0]) + __uint_as_float(h[1]);
}
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// One raw dword (pixels gx .. gx + 3 of row gy), zero outside the slice.
__device__ __forceinline__ uint32_t load_raw_dword(const uint8_t *src, long long pitch, int H, int W,
                                                   int gy, int gx, bool aligned)
{
    if (gy < 0 || gy >= H || gx + 3 < 0 || gx >= W) return 0u;
    const uint8_t *row = src + (long long)gy * pitch;
    if (aligned && gx >= 0 && gx + 3 < W) return *reinterpret_cast<const uint32_t *>(row + gx);
    uint32_t v = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (gx + i >= 0 && gx + i < W) v |= (uint32_t)row[gx + i] << (8 * i);
    return v;
}

// Whether a stack takes the fixed-offset dword loads: rows 4-byte aligned and a
// multiple of 4 wide (every dword whole), and a raw tile window small enough
// for 32-bit offsets.
inline bool smooth_fast_loads(const SmoothArgs &a)
{
    const bool aligned = ((a.pitch_row & 3) == 0) && ((a.pitch_slice & 3) == 0) &&
                         ((reinterpret_cast<uintptr_t>(a.stack) & 3) == 0);
    return aligned && (a.W & 3) == 0 && a.pitch_row * kRawHMax < 0x7fffffffLL;
}

// RT: compile-time in-plane tap radius (>= the true radius; taps beyond it
// carry zero weight), RZ: cross-slice tap radius.  FAST: the stack takes the
// fixed-offset dword loads (smooth_fast_loads); otherwise raw tiles are read
// byte by byte where a dword is not whole.  ROBUST (FP32): the robust
// cross-slice average of "Extensions and Applications" (values more than two
// weighted standard deviations from the window's weighted mean left out).
// Plain FP32 instances keep four waves per SIMD (two workgroups per CU); FP64
// and robust ones need more registers than that allows.  RANGE: only the
// output slices [a.z_lo, a.z_hi) are computed and stored (a uniform test per
// step; without it the march has none).
template <typename T, int RZ, int RT, bool FAST, bool ROBUST, bool RANGE>
__global__ __launch_bounds__(kSThreads, ((sizeof(T) == 4 && !ROBUST) ? 4 : 1)) void smooth_kernel(SmoothArgs a)
{
    constexpr int NZ = 2 * RZ + 1;     // register ring of blurred planes
    constexpr int NRAW = RZ + 3;       // LDS ring of raw tiles: slices zo .. zi + 1
    constexpr int RH = RT > 0 ? RT : 1;   // raw halo rows (>= 1 for the Laplacian of I0)
    __shared__ uint32_t ring_raw[NRAW][kRawHMax * kRawDw];
    __shared__ T hb[2][kRawHMax * kSTX];   // x-blurred rows of the last two input slices
    __shared__ double red_s[2][kSmoothWaves][3];   // per-wave partial sums, by output slice parity
    __shared__ float xs[2][kSmoothWaves / 2][64];   // restriction: row shared by two waves, by slice parity

    const int tid = threadIdx.x;
    const int tx = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // (wave-uniform)
    const int tile = (int)xcd_tile(blockIdx.x, gridDim.x);   // neighbouring tiles share an XCD
    const int tile_x = tile % a.tiles_x, tile_y = tile / a.tiles_x;
    const int X0 = tile_x * kSTX, Y0 = tile_y * kSTY;
    const int S = a.S, H = a.H, W = a.W, R = a.rxy;
    // output slices (RANGE: [a.z_lo, a.z_hi); otherwise all, with no test in the march)
    const int z_lo = RANGE ? a.z_lo : 0, z_hi = RANGE ? a.z_hi : S;
    constexpr int rawH = kSTY + 2 * RH;
    const int n_dw = rawH * kRawDw;
    const bool aligned = ((a.pitch_row & 3) == 0) && ((a.pitch_slice & 3) == 0) &&
                         ((reinterpret_cast<uintptr_t>(a.stack) & 3) == 0);
    const int x = X0 + tx;
    const int yb = wv * kSRows;        // this thread's output rows (tile-local)

    // taps are uniform: for FP32 they come from FP32 copies, so they stay in
    // scalar registers (a conversion would place them in vector registers)
    T wxy[RT + 1];
#pragma unroll
    for (int d = 0; d <= RT; ++d) {
        if constexpr (sizeof(T) == 4) wxy[d] = d <= R ? a.wxy_f[d] : 0.f;
        else wxy[d] = d <= R ? a.wxy[d] : 0.0;
    }
    T wz[RZ + 1];
#pragma unroll
    for (int d = 0; d <= RZ; ++d) {
        if constexpr (sizeof(T) == 4) wz[d] = a.wz_f[d];
        else wz[d] = a.wz[d];
    }

    // in-plane renormalisation 1 / (sum_x w * sum_y w) per output pixel
    T wsx = T(0);
    for (int d = -R; d <= R; ++d)
        if (x + d >= 0 && x + d < W) wsx += wxy[d < 0 ? -d : d];
    T inv_xy[kSRows];
#pragma unroll
    for (int i = 0; i < kSRows; ++i) {
        const int y = Y0 + yb + i;
        T wsy = T(0);
        for (int d = -R; d <= R; ++d)
            if (y + d >= 0 && y + d < H) wsy += wxy[d < 0 ? -d : d];
        inv_xy[i] = T(1) / (wsx * wsy);
    }

    T ring[NZ][kSRows];
#pragma unroll
    for (int k = 0; k < NZ; ++k)
#pragma unroll
        for (int i = 0; i < kSRows; ++i) ring[k][i] = T(0);

    T alT;
    if constexpr (sizeof(T) == 4) alT = a.alpha_f;
    else alT = a.alpha;
    const long long nparts = (long long)a.tiles_x * a.tiles_y;   // one partial per tile

    uint32_t pf[kPrefetch];   // raw tile of the next input slice, in flight
    // FAST: each thread loads the same raw dwords of every slice; their offsets
    // in the tile's row window are fixed per thread (kNoLane outside the slice:
    // the load reads zero).
    const int gy0 = max(Y0 - RH, 0), gy1 = min(Y0 + kSTY + RH, H);   // the window's rows
    unsigned voff[kPrefetch];
#pragma unroll
    for (int q = 0; q < kPrefetch; ++q) {
        const int e = tid + q * kSThreads;
        const int r = e / kRawDw, c = e - r * kRawDw;
        const int gy = Y0 - RH + r, gx = X0 - 8 + 4 * c;   // gx: a multiple of 4
        const bool in = e < n_dw && gy >= 0 && gy < H && gx >= 0 && gx < W;
        voff[q] = in ? (unsigned)((gy - gy0) * a.pitch_row + gx) : kNoLane;
    }
    auto issue = [&](int zi) {
        if constexpr (FAST) {
            // unconditional: a load under a branch would be waited for where the
            // paths join, right after its issue.  Past the stack the window is
            // empty (the loads read zero, and the slot is never read).
            const int zc = min(zi, S - 1);
            // (the size goes through readfirstlane: a select the compiler places in
            // vector registers would wrap every load in a per-lane loop)
            const unsigned nb = (unsigned)__builtin_amdgcn_readfirstlane(zi < S ? (int)((gy1 - gy0) * a.pitch_row) : 0);
            const Rsrc rs = make_rsrc(a.stack + (long long)zc * a.pitch_slice + (long long)gy0 * a.pitch_row, nb);
#pragma unroll
            for (int q = 0; q < kPrefetch; ++q) pf[q] = Buf<unsigned>::ld(rs, voff[q], 0);
            return;
        }
#pragma unroll
        for (int q = 0; q < kPrefetch; ++q) {
            const int e = tid + q * kSThreads;
            pf[q] = 0u;
            if (zi < S && e < n_dw) {
                const int r = e / kRawDw, c = e - r * kRawDw;
                pf[q] = load_raw_dword(a.stack + (long long)zi * a.pitch_slice, a.pitch_row, H, W,
                                       Y0 - RH + r, X0 - 8 + 4 * c, aligned);
            }
        }
    };
    auto commit = [&](int zi) {
#pragma unroll
        for (int q = 0; q < kPrefetch; ++q) {
            const int e = tid + q * kSThreads;
            if (e < n_dw) ring_raw[zi % NRAW][e] = pf[q];
        }
    };
    // raw byte at tile-local raw row r (row 0 = Y0 - RH) and byte column c (x = X0 - 8 + c)
    // (a byte load from LDS: no shift-and-mask on the vector unit)
    auto raw_at = [&](int slot, int r, int c) -> float {
        return (float)reinterpret_cast<const uint8_t *>(ring_raw[slot])[r * kRawW + c];
    };
    // output offsets: the thread's column (kNoLane outside the slice, so the
    // stores need no branch) plus each row's offset in the tile's rows of a
    // slice's b (and of g_s), uniform across the wave like the rows' in-slice
    // flags and the masks of the Laplacian's vertical neighbours
    // (the row goes in the scalar offset; rows outside the slice are dropped
    // through the vector offset, kNoLane, like columns outside it)
    const unsigned vx = x < W ? (unsigned)x * (unsigned)sizeof(T) : kNoLane;
    unsigned sb[kSRows];
    bool rin[kSRows], oin[kSRows];
    float myu[kSRows], myd[kSRows];
#pragma unroll
    for (int i = 0; i < kSRows; ++i) {
        const int y = Y0 + yb + i;
        rin[i] = y < H;
        oin[i] = y < H && x < W;
        sb[i] = (unsigned)((yb + i) * a.b_pitch) * (unsigned)sizeof(T);
        myu[i] = y > 0 ? 1.f : 0.f;
        myd[i] = y < H - 1 ? 1.f : 0.f;
    }
    const float mxl = x > 0 ? 1.f : 0.f, mxr = x < W - 1 ? 1.f : 0.f;

    // One partial per tile and slice: the waves' sums of slice z in a fixed
    // order.  They are complete after the barrier that ends slice z's output
    // step, and reduced in the next step, after the raw tile's commit (the next
    // write to that buffer half comes before the barrier after that).  Lane
    // 3 s + q of wave 0 holds quantity q of slice kPB m + s; each group of kPB
    // slices is stored at once.  (A register that held store data or address
    // is rewritten only after a wait for the store: a store per step would
    // stall wave 0, and with it the barrier, once per step.)
    constexpr int kPB = 21;
    double pbuf = 0.0;
    const int pq = tid % 3, ps = tid / 3;
    // (groups count from the first output slice; partial sums are indexed by
    // output slice, z - z_lo)
    auto partial = [&](int z) {
        const int zl = z - z_lo;
        const int zs = zl % kPB;   // uniform
        if (tid < 3 * kPB && ps == zs) {
            double v = 0.0;
#pragma unroll
            for (int w = 0; w < kSmoothWaves; ++w) v += red_s[z & 1][w][pq];
            pbuf = v;
        }
        if ((zs == kPB - 1 || z == z_hi - 1) && a.b0) {
            if (tid < 3 * (zs + 1)) {
                double *dst = pq == 0 ? a.part_bb : (pq == 1 ? a.part_b0 : a.part_bs);
                dst[(long long)(zl - zs + ps) * nparts + tile] = pbuf;
            }
        }
    };
    // Restriction of b_u to level 1 (a.bc0, FP32 hierarchy): a coarse cell's
    // right-hand side is the sum of its children's b_u (zero outside the slice).
    // Lane pairs give the column sums, a thread's rows the row sums; with an odd
    // number of rows per thread, the row pair split between waves 2m and 2m + 1
    // meets in LDS and is stored by wave 2m + 1 in the next step.
    const bool rst = sizeof(T) == 4 && a.bc0 != nullptr;   // (FP64 hierarchies restrict in the solve)
    const unsigned vcol = ((tx & 1) == 0 && X0 + tx < W) ? (unsigned)((X0 + tx) >> 1) * 2u : kNoLane;
    float hx = 0.f;   // odd waves: column sum of their first row (the pair's second row)
    auto cstore = [&](int z, int ty, float v) {   // ty: tile row of the cell's first child (even)
        if (Y0 + ty >= H) return;
        const Rsrc rc = make_rsrc(static_cast<unsigned short *>(a.bc0) + (long long)(z - z_lo) * a.bc_slice_stride +
                                      (long long)((Y0 + ty) >> 1) * a.bc_pitch,
                                  (unsigned)a.bc_pitch * 2u);
        Buf<unsigned short>::st(__builtin_bit_cast(unsigned short, (__bf16)v), rc, vcol, 0);   // nearest even
    };

    // the last step's output values stay in their registers until the next
    // step's commit has waited for every load and store: rewritten earlier,
    // they would need a wait for their stores right there
    T hold[kSRows];
#pragma unroll
    for (int i = 0; i < kSRows; ++i) hold[i] = T(0);

    issue(0);
    commit(0);
    __syncthreads();

    // Step zi (software-pipelined, one barrier per step): x blur of input slice
    // zi into hb[zi & 1]; y blur of slice zi - 1 (x-blurred in the previous
    // step) into register ring slot (zi - 1) mod NZ; z blur and output of slice
    // zo = zi - 1 - RZ; the raw tile of slice zi + 1 enters the LDS ring.
    // (called only for zi < z_hi + RZ + 1; k = zi mod NZ, a constant once unrolled)
    auto step = [&](const int zi, const int k) __attribute__((always_inline)) {
        const int islot = zi % NRAW;
        issue(zi + 1);       // next raw tile: its latency is hidden by this step
        // ------------- x blur of every raw row, 4 consecutive outputs per work item
        if (zi < S) {
            T *hbz = hb[zi & 1];
            for (int wi = tid; wi < rawH * 16; wi += kSThreads) {
                const int r = wi >> 4, seg = (wi & 15) * 4;
                const uint32_t *rowp = &ring_raw[islot][r * kRawDw + (seg >> 2)];
                T v[20];   // v[j] = pixel X0 + seg - 8 + j
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    const uint32_t w = rowp[q];
#pragma unroll
                    for (int i = 0; i < 4; ++i) v[4 * q + i] = (T)((w >> (8 * i)) & 0xffu);
                }
                typedef T T4 __attribute__((ext_vector_type(4)));
                T4 out4;
#pragma unroll
                for (int o = 0; o < 4; ++o) {
                    T acc = wxy[0] * v[8 + o];
#pragma unroll
                    for (int d = 1; d <= RT; ++d) acc += wxy[d] * (v[8 + o - d] + v[8 + o + d]);
                    out4[o] = acc;
                }
                // one vector store per item (strided scalar stores would conflict on banks)
                *reinterpret_cast<T4 *>(&hbz[r * kSTX + seg]) = out4;
            }
        }
        // ------------- y blur of slice zi - 1 into the register ring
        const int ks = (k + NZ - 1) % NZ;   // its ring slot (static once unrolled)
        const int zy = zi - 1;
        if (zy >= 0 && zy < S) {
            const T *hby = hb[zy & 1];
            T col[kSRows + 2 * RT];   // col[j]: x-blurred raw row yb + RH - RT + j
#pragma unroll
            for (int j = 0; j < kSRows + 2 * RT; ++j) col[j] = hby[(yb + RH - RT + j) * kSTX + tx];
#pragma unroll
            for (int i = 0; i < kSRows; ++i) {
                T acc = wxy[0] * col[i + RT];
#pragma unroll
                for (int d = 1; d <= RT; ++d) acc += wxy[d] * (col[i + RT - d] + col[i + RT + d]);
                ring[ks][i] = acc * inv_xy[i];
            }
        } else {
#pragma unroll
            for (int i = 0; i < kSRows; ++i) ring[ks][i] = T(0);
        }
        // ------------- output slice zo = zi - 1 - RZ (the first test is static in
        // the peeled steps)
        const int zo = zi - 1 - RZ;
        if (zo >= 0 && (!RANGE || (zo >= z_lo && zo < z_hi))) {
            const int zlo = min(RZ, zo), zhi = min(RZ, S - 1 - zo);   // in-stack taps
            T iz;
            if constexpr (sizeof(T) == 4) iz = a.inv_wz_f[zlo][zhi];
            else iz = a.inv_wz[zlo][zhi];
            const int oslot = zo % NRAW;
            // this slice's tile rows of b (and of g_s): windows of kSTY rows
            // (a resource of size zero drops the stores: no b_u without a.b0, and
            // g_s only for the output slices asked for)
            const Rsrc rbw = make_rsrc(static_cast<T *>(a.b0) + (long long)(zo - z_lo) * a.b_slice_stride +
                                           (long long)Y0 * a.b_pitch,
                                       a.b0 ? (unsigned)(kSTY * a.b_pitch * (int)sizeof(T)) : 0u);
            const bool gsz = a.gs_out && zo >= a.gs_zlo && zo < a.gs_zhi;   // uniform
            const Rsrc rgw = a.gs_out ? make_rsrc(static_cast<T *>(a.gs_out) + ((long long)(zo - a.gs_zlo) * H + Y0) * W,
                                                  gsz ? (unsigned)(kSTY * W * (int)sizeof(T)) : 0u)
                                      : rbw;
            T sbb = T(0), sb0 = T(0), sbs = T(0);
            // original slice around this thread's column
            float oc[kSRows + 2], ol[kSRows], orr[kSRows];
#pragma unroll
            for (int j = 0; j < kSRows + 2; ++j) oc[j] = raw_at(oslot, yb + RH - 1 + j, tx + 8);
#pragma unroll
            for (int i = 0; i < kSRows; ++i) {
                ol[i] = raw_at(oslot, yb + RH + i, tx + 7);
                orr[i] = raw_at(oslot, yb + RH + i, tx + 9);
            }
            T bus[kSRows], gvs[kSRows];
            float bms[kSRows];   // b_u, zero outside the slice
#pragma unroll
            for (int i = 0; i < kSRows; ++i) {
                // register slot of zo is k - 1 - RZ (mod NZ): static for each k
                T acc = wz[0] * ring[((k - 1 - RZ) % NZ + NZ) % NZ][i];
#pragma unroll
                for (int d = 1; d <= RZ; ++d)
                    acc += wz[d] * (ring[((k - 1 - RZ - d) % NZ + NZ) % NZ][i] +
                                    ring[((k - 1 - RZ + d) % NZ + NZ) % NZ][i]);
                T g = acc * iz;
                if constexpr (ROBUST) {
                    // robust cross-slice average: the window's in-stack values
                    // (taps -zlo .. zhi) within two weighted standard deviations of
                    // their weighted mean g, re-averaged with their weights
                    auto tap = [&](int d) -> T { return ring[((k - 1 - RZ + d) % NZ + NZ) % NZ][i]; };
                    auto wt = [&](int d) -> T { return (d >= -zlo && d <= zhi) ? wz[d < 0 ? -d : d] : T(0); };
                    T var = T(0);
#pragma unroll
                    for (int d = -RZ; d <= RZ; ++d) {
                        const T e = tap(d) - g;
                        var = fma(wt(d) * e, e, var);
                    }
                    const T thr = T(4) * var * iz;
                    T num = T(0), den = T(0);
#pragma unroll
                    for (int d = -RZ; d <= RZ; ++d) {
                        const T e = tap(d) - g;
                        const T w = e * e <= thr ? wt(d) : T(0);
                        num = fma(w, tap(d), num);
                        den += w;
                    }
                    g = num / den;   // (den > 0: the value nearest the mean always stays)
                }
                const float o = oc[i + 1];
                // (L g_o)_p over in-slice neighbours
                float lap = mxl * (o - ol[i]);
                lap = fmaf(mxr, o - orr[i], lap);
                lap = fmaf(myu[i], o - oc[i], lap);
                lap = fmaf(myd[i], o - oc[i + 2], lap);
                const T bu = alT * (g - (T)o);
                const T bf = alT * g + (T)lap;
                bus[i] = bu;
                gvs[i] = g;
                // (selects: outside the slice the values may not be finite)
                const T bum = oin[i] ? bu : T(0), bfm = oin[i] ? bf : T(0);
                bms[i] = (float)bum;
                sbb = fma(bfm, bfm, sbb);
                sb0 = fma(bum, bum, sb0);
                sbs += bum;
            }
            // the next raw tile goes into its slot (no reader of it in this
            // step) before the stores: its wait would otherwise also wait
            // for them
            commit(zi + 1);
#pragma unroll
            for (int i = 0; i < kSRows; ++i) asm volatile("" ::"v"(hold[i]));
            if (zo - 1 >= z_lo) partial(zo - 1);
            if (rst) {
                if constexpr (kSRows % 2 == 1)
                    if ((wv & 1) && zo - 1 >= z_lo) cstore(zo - 1, yb - 1, xs[(zo - 1) & 1][wv >> 1][tx] + hx);
                float cs[kSRows];
#pragma unroll
                for (int i = 0; i < kSRows; ++i) cs[i] = bms[i] + dpp_row<0xB1>(bms[i]);   // lane pairs
                if constexpr (kSRows % 2 == 0) {
#pragma unroll
                    for (int i = 0; i < kSRows; i += 2) cstore(zo, yb + i, cs[i] + cs[i + 1]);
                } else if ((wv & 1) == 0) {
#pragma unroll
                    for (int i = 0; i + 1 < kSRows; i += 2) cstore(zo, yb + i, cs[i] + cs[i + 1]);
                    xs[zo & 1][wv >> 1][tx] = cs[kSRows - 1];
                } else {
#pragma unroll
                    for (int i = 1; i + 1 < kSRows; i += 2) cstore(zo, yb + i, cs[i] + cs[i + 1]);
                    hx = cs[0];
                }
            }
#pragma unroll
            for (int i = 0; i < kSRows; ++i) {
                const unsigned vo = rin[i] ? vx : kNoLane;
                Buf<T>::st(bus[i], rbw, vo, sb[i]);
                if (a.gs_out) Buf<T>::st(gvs[i], rgw, vo, (unsigned)((yb + i) * W) * (unsigned)sizeof(T));
                hold[i] = bus[i];
            }
            const double tbb = (double)wave_sum(sbb), tb0 = (double)wave_sum(sb0),
                         tbs = (double)wave_sum(sbs);
            if ((tid & 63) == 0) {
                red_s[zo & 1][wv][0] = tbb;
                red_s[zo & 1][wv][1] = tb0;
                red_s[zo & 1][wv][2] = tbs;
            }
        } else {
            commit(zi + 1);
        }
        __syncthreads();
    };
    // The first block of NZ steps is peeled: there every slice index is a
    // constant, so the steps before the first output carry no output code.
    // In the others every step has an output slice (zo >= NZ - 1 - RZ = RZ).
    // (the march ends with the last output slice)
    const int zend = z_hi + RZ + 1;
#pragma unroll
    for (int k = 0; k < NZ; ++k)
        if (k < zend) step(k, k);
    for (int zb = NZ; zb < zend; zb += NZ) {
        __builtin_assume(zb >= NZ);
#pragma unroll
        for (int k = 0; k < NZ; ++k)
            if (zb + k < zend) step(zb + k, k);   // uniform across the block
    }
    partial(z_hi - 1);   // the last slice's sums are complete after the last barrier
    if constexpr (kSRows % 2 == 1)
        if (rst && (wv & 1)) cstore(z_hi - 1, yb - 1, xs[(z_hi - 1) & 1][wv >> 1][tx] + hx);
}

// Launch one (precision, radius) instance; defined per cross-slice radius in
// the smooth_rz*.hip translation units so they compile in parallel.
template <typename T, int RZ, int RT, bool ROBUST, bool RANGE>
hipError_t smooth_launch_r(const SmoothArgs &a, hipStream_t s)
{
    if (smooth_fast_loads(a))
        hipLaunchKernelGGL((smooth_kernel<T, RZ, RT, true, ROBUST, RANGE>), dim3(a.tiles_x * a.tiles_y),
                           dim3(kSThreads), 0, s, a);
    else
        hipLaunchKernelGGL((smooth_kernel<T, RZ, RT, false, ROBUST, RANGE>), dim3(a.tiles_x * a.tiles_y),
                           dim3(kSThreads), 0, s, a);
    return hipGetLastError();
}
template <typename T, int RZ, int RT, bool ROBUST>
hipError_t smooth_launch(const SmoothArgs &a, hipStream_t s)
{
    if (a.z_lo == 0 && a.z_hi == a.S) return smooth_launch_r<T, RZ, RT, ROBUST, false>(a, s);
    return smooth_launch_r<T, RZ, RT, ROBUST, true>(a, s);
}

// All instances for one cross-slice radius RZ.
#define GDF_SMOOTH_RZ(RZ)                                                                  \
    hipError_t smooth_rz_##RZ(bool fp64, const SmoothArgs &a, hipStream_t s)               \
    {                                                                                      \
        if (fp64) return a.robust ? hipErrorInvalidValue : smooth_launch<double, RZ, kMaxRxy, false>(a, s); \
        if (a.robust)                                                                      \
            return a.rxy == 3 ? smooth_launch<float, RZ, 3, true>(a, s)                    \
                              : smooth_launch<float, RZ, kMaxRxy, true>(a, s);             \
        return a.rxy == 3 ? smooth_launch<float, RZ, 3, false>(a, s)                       \
                          : smooth_launch<float, RZ, kMaxRxy, false>(a, s);                \
    }

}  // namespace gdf
