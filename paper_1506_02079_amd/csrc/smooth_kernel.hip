// Anisotropic Gaussian smoothing of a uint8 stack across slices (Section
// III-A), truncated at three standard deviations per axis (Implementation
// subsection), renormalised over the taps that fall inside the stack.  The
// kernel and the in-stack box are both products over the axes, so the
// renormalised 3D sum factors into three 1D passes, each divided by its own
// in-range weight sum.
//
// One workgroup owns a 64 x 16 tile of every slice and marches through the
// stack.  Per input slice it stages the raw tile plus an in-plane halo in
// LDS, blurs along x then y, and pushes the blurred plane into a ring of
// 2 rz + 1 planes held in registers; the z blur of an output slice is a
// weighted sum over the ring.  The output is written straight into the
// right-hand side of the solve, b_u = alpha (I1 - I0), together with FP64
// partial sums of ||alpha I1 + L I0||^2 (the norm of Eq. (1)'s right-hand
// side) and ||b_u||^2.  The smoothed stack itself is written only when asked.
#include "internal.h"

namespace gdf {

constexpr int kSTX = 64, kSTY = 16, kMaxRxy = 7;
constexpr int kRawW = kSTX + 2 * kMaxRxy, kRawH = kSTY + 2 * kMaxRxy;

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

template <typename T, int RZ>
__global__ __launch_bounds__(256) void smooth_kernel(SmoothArgs a)
{
    constexpr int NZ = 2 * RZ + 1;
    __shared__ T raw[kRawH * kRawW];
    __shared__ T hb[kRawH * kSTX];

    const int tid = threadIdx.x;
    const int tx = tid & 63, wv = tid >> 6;
    const int tile = blockIdx.x;
    const int tile_x = tile % a.tiles_x, tile_y = tile / a.tiles_x;
    const int X0 = tile_x * kSTX, Y0 = tile_y * kSTY;
    const int S = a.S, H = a.H, W = a.W, R = a.rxy;
    const int rawW = kSTX + 2 * R, rawH = kSTY + 2 * R;
    const int x = X0 + tx;
    const int yb = Y0 + wv * 4;   // this thread's 4 output rows yb..yb+3

    T wxy[kMaxRxy + 1];
#pragma unroll
    for (int d = 0; d <= kMaxRxy; ++d) wxy[d] = (T)a.wxy[d];
    T wz[RZ + 1];
#pragma unroll
    for (int d = 0; d <= RZ; ++d) wz[d] = (T)a.wz[d];

    // in-plane renormalisation 1 / (sum_x w * sum_y w) per output pixel
    T wsx = T(0);
    for (int d = -R; d <= R; ++d)
        if (x + d >= 0 && x + d < W) wsx += wxy[d < 0 ? -d : d];
    T inv_xy[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int y = yb + i;
        T wsy = T(0);
        for (int d = -R; d <= R; ++d)
            if (y + d >= 0 && y + d < H) wsy += wxy[d < 0 ? -d : d];
        inv_xy[i] = T(1) / (wsx * wsy);
    }

    T ring[NZ][4];
#pragma unroll
    for (int k = 0; k < NZ; ++k)
#pragma unroll
        for (int i = 0; i < 4; ++i) ring[k][i] = T(0);

    const double al = a.alpha;
    const int nparts = a.tiles_x * a.tiles_y * 4;

    for (int zb = 0; zb < S + RZ; zb += NZ) {
#pragma unroll
        for (int k = 0; k < NZ; ++k) {
            const int zi = zb + k;
            // ---------------- blurred plane of input slice zi into ring[k]
            // (steps past the last output, zi >= S + RZ, do nothing: zo >= S below)
            if (zi < S) {
                const uint8_t *src = a.stack + (long long)zi * a.pitch_slice;
                for (int e = tid; e < rawH * rawW; e += 256) {
                    const int r = e / rawW, c = e - r * rawW;
                    const int gy = Y0 - R + r, gx = X0 - R + c;
                    T v = T(0);
                    if (gy >= 0 && gy < H && gx >= 0 && gx < W) v = (T)src[(long long)gy * a.pitch_row + gx];
                    raw[r * kRawW + c] = v;
                }
                __syncthreads();
                for (int r = wv; r < rawH; r += 4) {
                    T acc = T(0);
                    for (int d = -R; d <= R; ++d) acc += wxy[d < 0 ? -d : d] * raw[r * kRawW + tx + R + d];
                    hb[r * kSTX + tx] = acc;
                }
                __syncthreads();
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = wv * 4 + i;
                    T acc = T(0);
                    for (int d = -R; d <= R; ++d) acc += wxy[d < 0 ? -d : d] * hb[(r + R + d) * kSTX + tx];
                    ring[k][i] = acc * inv_xy[i];
                }
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i) ring[k][i] = T(0);
            }
            // ---------------- output slice zo = zi - RZ
            const int zo = zi - RZ;
            if (zo >= 0 && zo < S) {
                T wsz = T(0);
#pragma unroll
                for (int d = -RZ; d <= RZ; ++d)
                    if (zo + d >= 0 && zo + d < S) wsz += wz[d < 0 ? -d : d];
                const T iz = T(1) / wsz;
                const LevelDesc &L = a.levs[(long long)zo * a.lev_stride];
                T *bdst = static_cast<T *>(L.b);
                const uint8_t *og = a.stack + (long long)zo * a.pitch_slice;
                double sbb = 0.0, sb0 = 0.0, sbs = 0.0;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    T acc = T(0);
#pragma unroll
                    for (int d = -RZ; d <= RZ; ++d) {
                        // plane of slice zo + d = zi - RZ + d sits in slot (k - RZ + d) mod NZ
                        const int slot = ((k - RZ + d) % NZ + NZ) % NZ;
                        acc += wz[d < 0 ? -d : d] * ring[slot][i];
                    }
                    const int y = yb + i;
                    if (y < H && x < W) {
                        const T g = acc * iz;
                        const long long ro = (long long)y * a.pitch_row;
                        const double o = (double)og[ro + x];
                        double lap = 0.0;
                        if (x > 0) lap += o - (double)og[ro + x - 1];
                        if (x < W - 1) lap += o - (double)og[ro + x + 1];
                        if (y > 0) lap += o - (double)og[ro - a.pitch_row + x];
                        if (y < H - 1) lap += o - (double)og[ro + a.pitch_row + x];
                        const double bf = al * (double)g + lap;
                        const T bu = (T)(al * ((double)g - o));
                        bdst[(size_t)y * L.pitch + x] = bu;
                        if (a.gs_out) static_cast<T *>(a.gs_out)[((long long)zo * H + y) * W + x] = g;
                        sbb += bf * bf;
                        sb0 += (double)bu * (double)bu;
                        sbs += (double)bu;
                    }
                }
                sbb = wave_sum_d(sbb);
                sb0 = wave_sum_d(sb0);
                sbs = wave_sum_d(sbs);
                if ((tid & 63) == 0) {
                    const long long pi = (long long)zo * nparts + tile * 4 + wv;
                    a.part_bb[pi] = sbb;
                    a.part_b0[pi] = sb0;
                    a.part_bs[pi] = sbs;
                }
            }
        }
    }
}

template <typename T>
static hipError_t smooth_t(const SmoothArgs &a, hipStream_t s)
{
    const dim3 g(a.tiles_x * a.tiles_y), b(256);
    switch (a.rz) {
#define GDF_RZ(n) case n: hipLaunchKernelGGL((smooth_kernel<T, n>), g, b, 0, s, a); break;
        GDF_RZ(0) GDF_RZ(1) GDF_RZ(2) GDF_RZ(3) GDF_RZ(4) GDF_RZ(5) GDF_RZ(6) GDF_RZ(7)
        GDF_RZ(8) GDF_RZ(9) GDF_RZ(10) GDF_RZ(11) GDF_RZ(12)
#undef GDF_RZ
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_smooth(bool fp64, const SmoothArgs &a, hipStream_t s)
{
    if (a.rxy > kMaxRxy || a.rz > 12) return hipErrorInvalidValue;
    return fp64 ? smooth_t<double>(a, s) : smooth_t<float>(a, s);
}

}  // namespace gdf
