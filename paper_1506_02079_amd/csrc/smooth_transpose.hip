// Transpose of the smoothing operator (the gradient of a loss on the smoothed
// stack with respect to the stack; derived, the paper does not differentiate).
// The smoothing is I1(p) = sum_q K(q - p) I0(q) / D(p) over the in-stack taps of
// p's window (Section III-A; 3-sigma support from the Implementation
// subsection), with K the truncated anisotropic Gaussian and D(p) =
// Dx(x) Dy(y) Dz(z) the product of the per-axis in-range weight sums.  Its
// transpose is G0 = K (G1 / D): scale by 1 / D at every voxel, then correlate
// with K over in-range taps, one axis at a time (K is symmetric and separable).
#include "internal.h"

#include <algorithm>
#include <cstdint>

namespace gdf {

namespace {

struct XArgs {
    const float *in;
    float *out;
    const float *inv_d;   // 1 / Dx, 1 / Dy, 1 / Dz tables (W, H, S)
    int S, H, W;
    int r;                // in-plane tap radius
    float w[8];           // taps w[0..r]
};

// x pass with the 1 / D scaling at the source: one thread per voxel of a row
// (its taps are neighbours in the same cache lines), rows over the grid's y
// and z dimensions.
__global__ __launch_bounds__(256) void transpose_x_kernel(XArgs a)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= a.W) return;
    const float *ix = a.inv_d, *iy = a.inv_d + a.W, *iz = a.inv_d + a.W + a.H;
    const int lo = max(-a.r, -x), hi = min(a.r, a.W - 1 - x);
    for (int z = blockIdx.z; z < a.S; z += gridDim.z)
        for (int y = blockIdx.y; y < a.H; y += gridDim.y) {
            const long long i = ((long long)z * a.H + y) * a.W + x;
            const float izy = iz[z] * iy[y];   // Dz Dy are fixed along the row, Dx changes per tap
            float acc = 0.f;
            for (int d = lo; d <= hi; ++d) acc = fmaf(a.w[d < 0 ? -d : d] * (izy * ix[x + d]), a.in[i + d], acc);
            a.out[i] = acc;
        }
}

// Element arithmetic of the ring passes, for one column (float) or four
// neighbouring columns (float4).
typedef float vec4f __attribute__((ext_vector_type(4)));   // a register vector, 16-byte aligned

__device__ inline float vzero(float) { return 0.f; }
__device__ inline vec4f vzero(vec4f) { return vec4f{0.f, 0.f, 0.f, 0.f}; }
__device__ inline float vmul(float w, float a) { return w * a; }
__device__ inline vec4f vmul(float w, vec4f a) { return vec4f{w * a.x, w * a.y, w * a.z, w * a.w}; }
__device__ inline float vadd(float a, float b) { return a + b; }
__device__ inline vec4f vadd(vec4f a, vec4f b) { return vec4f{a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w}; }
__device__ inline float vfma(float w, float a, float b, float c) { return fmaf(w, a + b, c); }
__device__ inline vec4f vfma(float w, vec4f a, vec4f b, vec4f c)
{
    return vec4f{fmaf(w, a.x + b.x, c.x), fmaf(w, a.y + b.y, c.y), fmaf(w, a.z + b.z, c.z), fmaf(w, a.w + b.w, c.w)};
}

// z pass with a register ring: one thread per (y, x) column (or 4 columns) marches down the
// slices holding in[z - R .. z + R]; each input is read once.  Values outside
// the stack are zero in the ring, which drops their taps (the transpose's
// correlation has no renormalisation).  The march is unrolled by the ring
// length, so ring slots are static.
struct Taps {
    float w[16];
};

// add (may alias out, or be null): out = (z pass) + add, element by element,
// each element read before the same thread writes it
template <int R, typename V>
__global__ __launch_bounds__(256) void transpose_z_ring(const V *in, V *out, const V *add, int S, long long plane,
                                                        Taps t)
{
    // plane: elements of V per slice
    constexpr int N = 2 * R + 1;
    const long long col = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= plane) return;
    const V zero = vzero(V{});
    V ring[N];
#pragma unroll
    for (int j = 0; j < N; ++j) ring[j] = zero;
    // slot of slice z' is (z' + R) mod N; preload slices 0 .. R - 1
#pragma unroll
    for (int zz = 0; zz < R; ++zz) ring[(zz + R) % N] = zz < S ? in[(long long)zz * plane + col] : zero;
    for (int zb = 0; zb < S; zb += N) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const int z = zb + k;
            if (z < S) {   // uniform
                const int zl = z + R;   // slice entering the ring
                ring[(k + 2 * R) % N] = zl < S ? in[(long long)zl * plane + col] : zero;
                V acc = vmul(t.w[0], ring[(k + R) % N]);
#pragma unroll
                for (int d = 1; d <= R; ++d) acc = vfma(t.w[d], ring[(k + R - d) % N], ring[(k + R + d) % N], acc);
                if (add) acc = vadd(acc, add[(long long)z * plane + col]);
                out[(long long)z * plane + col] = acc;
            }
        }
    }
}

// y pass with a register ring: one thread per (z, x) and segment of kYSeg rows,
// holding in[y - R .. y + R] (the segment's first 2R rows are read twice:
// once by this segment, once by the one above).
constexpr int kYSeg = 64;

template <int R, typename V>
__global__ __launch_bounds__(256) void transpose_y_ring(const V *in, V *out, int S, int H, int W, Taps t)
{
    // W: elements of V per row
    constexpr int N = 2 * R + 1;
    const V zero = vzero(V{});
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= W) return;
    const int y0 = blockIdx.y * kYSeg;
    if (y0 >= H) return;
    const int y1 = min(y0 + kYSeg, H);
    for (int z = blockIdx.z; z < S; z += gridDim.z) {
        const V *col = in + (long long)z * H * W + x;
        V *ocol = out + (long long)z * H * W + x;
        V ring[N];
        // slot of row y' is (y' - y0 + R) mod N; preload rows y0 - R .. y0 + R - 1
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) {
            const int yy = y0 - R + j;
            ring[j] = (yy >= 0 && yy < H) ? col[(long long)yy * W] : zero;
        }
        for (int yb = y0; yb < y1; yb += N) {
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const int y = yb + k;
                if (y < y1) {   // uniform
                    const int yl = y + R;   // row entering the ring
                    ring[(k + 2 * R) % N] = yl < H ? col[(long long)yl * W] : zero;
                    V acc = vmul(t.w[0], ring[(k + R) % N]);
#pragma unroll
                    for (int d = 1; d <= R; ++d) acc = vfma(t.w[d], ring[(k + R - d) % N], ring[(k + R + d) % N], acc);
                    ocol[(long long)y * W] = acc;
                }
            }
        }
    }
}

// x and y passes in one kernel for rows of a multiple of 4 voxels (16-byte
// aligned): a thread owns 4 neighbouring columns of a segment of kYSeg rows
// and marches down it with a register ring of the x pass's results for rows
// y - R .. y + R.  Each incoming row's x pass takes the 4 + 2R sources it
// needs as 2K + 1 aligned float4 loads (K = ceil(R / 4)); a float4 is wholly
// inside or outside the row, and one outside is zero, which drops its taps.
// The 1 / Dx factors of those sources stay in registers, and the x pass's
// results never go through memory.  The rows above and below a segment are
// x-passed by both segments that need them.
template <int R>
__global__ __launch_bounds__(256) void transpose_xy_ring(XArgs a)
{
    constexpr int K = (R + 3) / 4;
    constexpr int NV = 4 * (2 * K + 1);
    constexpr int N = 2 * R + 1;
    const int x0 = (blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (x0 >= a.W) return;
    const int y0 = blockIdx.y * kYSeg;
    if (y0 >= a.H) return;
    const int y1 = min(y0 + kYSeg, a.H);
    const float *iy = a.inv_d + a.W, *iz = a.inv_d + a.W + a.H;
    float sx[NV];
#pragma unroll
    for (int g = -K; g <= K; ++g) {
        const int xg = x0 + 4 * g;
        float4 t = make_float4(0.f, 0.f, 0.f, 0.f);
        if (xg >= 0 && xg < a.W) t = *reinterpret_cast<const float4 *>(a.inv_d + xg);
        const int j = 4 * (g + K);
        sx[j] = t.x;
        sx[j + 1] = t.y;
        sx[j + 2] = t.z;
        sx[j + 3] = t.w;
    }
    for (int z = blockIdx.z; z < a.S; z += gridDim.z) {
        const float *plane = a.in + (long long)z * a.H * a.W;
        const float izz = iz[z];
        // the x pass (with the 1 / D scaling) of row y; zero outside the slice
        auto xrow = [&](int y) -> vec4f {
            if (y < 0 || y >= a.H) return vec4f{0.f, 0.f, 0.f, 0.f};
            const float *row = plane + (long long)y * a.W;
            float v[NV];
#pragma unroll
            for (int g = -K; g <= K; ++g) {
                const int xg = x0 + 4 * g;
                float4 t = make_float4(0.f, 0.f, 0.f, 0.f);
                if (xg >= 0 && xg < a.W) t = *reinterpret_cast<const float4 *>(row + xg);
                const int j = 4 * (g + K);
                v[j] = t.x * sx[j];
                v[j + 1] = t.y * sx[j + 1];
                v[j + 2] = t.z * sx[j + 2];
                v[j + 3] = t.w * sx[j + 3];
            }
            const float izy = izz * iy[y];
            float o[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                float acc = 0.f;
#pragma unroll
                for (int d = -R; d <= R; ++d) acc = fmaf(a.w[d < 0 ? -d : d], v[4 * K + t + d], acc);
                o[t] = acc * izy;
            }
            return vec4f{o[0], o[1], o[2], o[3]};
        };
        vec4f ring[N];
        // slot of row y' is (y' - y0 + R) mod N; preload rows y0 - R .. y0 + R - 1
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) ring[j] = xrow(y0 - R + j);
        vec4f *ocol = reinterpret_cast<vec4f *>(a.out + (long long)z * a.H * a.W + x0);
        const int wv = a.W / 4;
        for (int yb = y0; yb < y1; yb += N) {
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const int y = yb + k;
                if (y < y1) {   // uniform
                    ring[(k + 2 * R) % N] = xrow(y + R);
                    vec4f acc = vmul(a.w[0], ring[(k + R) % N]);
#pragma unroll
                    for (int d = 1; d <= R; ++d) acc = vfma(a.w[d], ring[(k + R - d) % N], ring[(k + R + d) % N], acc);
                    ocol[(long long)y * wv] = acc;
                }
            }
        }
    }
}

bool aligned16(const void *a, const void *b)
{
    return ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) & 15) == 0;
}

hipError_t launch_y_ring(const float *in, float *out, int S, int H, int W, int rxy, const float *wxy, hipStream_t s)
{
    Taps t{};
    for (int d = 0; d < 8; ++d) t.w[d] = wxy[d];
    if ((H + kYSeg - 1) / kYSeg > 65535) return hipErrorInvalidValue;   // (H <= 4 M rows)
    const bool vec = aligned16(in, out) && W % 4 == 0;
    const int wv = vec ? W / 4 : W;
    const dim3 grid((unsigned)((wv + 255) / 256), (unsigned)((H + kYSeg - 1) / kYSeg), (unsigned)std::min(S, 65535));
    const vec4f *in4 = reinterpret_cast<const vec4f *>(in);
    vec4f *out4 = reinterpret_cast<vec4f *>(out);
    switch (rxy) {
#define GDF_YR(R) \
    case R: \
        if (vec) hipLaunchKernelGGL((transpose_y_ring<R, vec4f>), grid, dim3(256), 0, s, in4, out4, S, H, wv, t); \
        else hipLaunchKernelGGL((transpose_y_ring<R, float>), grid, dim3(256), 0, s, in, out, S, H, W, t); \
        break;
        GDF_YR(0) GDF_YR(1) GDF_YR(2) GDF_YR(3) GDF_YR(4) GDF_YR(5) GDF_YR(6) GDF_YR(7)
#undef GDF_YR
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_z_ring(const float *in, float *out, const float *add, int S, int H, int W, int rz,
                         const float *wz, hipStream_t s)
{
    Taps t{};
    for (int d = 0; d < 16; ++d) t.w[d] = wz[d];
    const long long plane = (long long)H * W;
    const bool vec = aligned16(in, out) && (!add || aligned16(add, add)) && plane % 4 == 0;
    const long long pv = vec ? plane / 4 : plane;
    const dim3 grid((unsigned)((pv + 255) / 256));
    const vec4f *in4 = reinterpret_cast<const vec4f *>(in);
    vec4f *out4 = reinterpret_cast<vec4f *>(out);
    const vec4f *add4 = reinterpret_cast<const vec4f *>(add);
    switch (rz) {
#define GDF_ZR(R) \
    case R: \
        if (vec) hipLaunchKernelGGL((transpose_z_ring<R, vec4f>), grid, dim3(256), 0, s, in4, out4, add4, S, pv, t); \
        else hipLaunchKernelGGL((transpose_z_ring<R, float>), grid, dim3(256), 0, s, in, out, add, S, plane, t); \
        break;
        GDF_ZR(0) GDF_ZR(1) GDF_ZR(2) GDF_ZR(3) GDF_ZR(4) GDF_ZR(5) GDF_ZR(6) GDF_ZR(7) GDF_ZR(8) GDF_ZR(9)
        GDF_ZR(10) GDF_ZR(11) GDF_ZR(12)
#undef GDF_ZR
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

// The per-axis factors 1 / D: entry c of an axis of n samples is one over the
// sum of the taps w[|d|], |d| <= r, whose sample c + d lies in [0, n), summed
// in FP64 from d = -r up.  Layout: W entries (x), H (y), S (z).
struct TapsD {
    double wxy[8], wz[16];
};

__global__ __launch_bounds__(256) void transpose_tables_kernel(float *inv_d, int S, int H, int W, int rxy, int rz,
                                                               TapsD t)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= W + H + S) return;
    int n, c, r;
    const double *w;
    if (i < W) {
        n = W, c = i, r = rxy, w = t.wxy;
    } else if (i < W + H) {
        n = H, c = i - W, r = rxy, w = t.wxy;
    } else {
        n = S, c = i - W - H, r = rz, w = t.wz;
    }
    double sum = 0.0;
    for (int d = -r; d <= r; ++d)
        if (c + d >= 0 && c + d < n) sum += w[d < 0 ? -d : d];
    inv_d[i] = (float)(1.0 / sum);
}

hipError_t launch_transpose_tables(float *inv_d, int S, int H, int W, int rxy, int rz, const double *wxy,
                                   const double *wz, hipStream_t s)
{
    if (rxy < 0 || rxy > 7 || rz < 0 || rz > 15) return hipErrorInvalidValue;
    TapsD t{};
    for (int d = 0; d < 8; ++d) t.wxy[d] = wxy[d];
    for (int d = 0; d < 16; ++d) t.wz[d] = wz[d];
    const long long n = (long long)W + H + S;
    hipLaunchKernelGGL(transpose_tables_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, inv_d, S, H, W,
                       rxy, rz, t);
    return hipGetLastError();
}

hipError_t launch_smooth_transpose(const float *g, float *out, const float *add, float *tmp, float *tmp2,
                                   const float *inv_d, int S, int H, int W, int rxy, int rz, const float *wxy,
                                   const float *wz, hipStream_t s)
{
    const long long n = (long long)S * H * W;
    if (n == 0) return hipSuccess;
    // x (with the 1 / D scaling at the source), y, z
    XArgs a{};
    a.in = g;
    a.out = out;
    a.inv_d = inv_d;
    a.S = S;
    a.H = H;
    a.W = W;
    a.r = rxy;
    for (int d = 0; d < 8; ++d) a.w[d] = wxy[d];
    const bool vec = W % 4 == 0 && aligned16(g, out) && aligned16(inv_d, tmp);
    if (vec) {
        // x and y in one pass: g -> tmp; z: tmp -> out
        if ((H + kYSeg - 1) / kYSeg > 65535) return hipErrorInvalidValue;   // (H <= 4 M rows)
        a.out = tmp;
        const dim3 grid((unsigned)((W / 4 + 255) / 256), (unsigned)((H + kYSeg - 1) / kYSeg), (unsigned)std::min(S, 65535));
        switch (rxy) {
#define GDF_XYR(R) \
    case R: hipLaunchKernelGGL(transpose_xy_ring<R>, grid, dim3(256), 0, s, a); break;
            GDF_XYR(0) GDF_XYR(1) GDF_XYR(2) GDF_XYR(3) GDF_XYR(4) GDF_XYR(5) GDF_XYR(6) GDF_XYR(7)
#undef GDF_XYR
        default: return hipErrorInvalidValue;
        }
        const hipError_t exy = hipGetLastError();
        if (exy != hipSuccess) return exy;
        return launch_z_ring(tmp, out, add, S, H, W, rz, wz, s);
    }
    // one-voxel x pass: g -> tmp2; y: tmp2 -> tmp; z: tmp -> out
    a.out = tmp2;
    {
        const dim3 grid((unsigned)((W + 255) / 256), (unsigned)std::min(H, 65535), (unsigned)std::min(S, 65535));
        hipLaunchKernelGGL(transpose_x_kernel, grid, dim3(256), 0, s, a);
    }
    hipError_t e0 = hipGetLastError();
    if (e0 != hipSuccess) return e0;
    const hipError_t e = launch_y_ring(tmp2, tmp, S, H, W, rxy, wxy, s);
    if (e != hipSuccess) return e;
    return launch_z_ring(tmp, out, add, S, H, W, rz, wz, s);
}

}  // namespace gdf
