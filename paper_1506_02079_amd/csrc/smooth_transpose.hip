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

namespace gdf {

namespace {

struct XArgs {
    const float *in;
    float *out;
    const float *inv_d;   // 1 / Dz, 1 / Dy, 1 / Dx tables (S, H, W)
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
    const float *iz = a.inv_d, *iy = a.inv_d + a.S, *ix = a.inv_d + a.S + a.H;
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

// z pass with a register ring: one thread per (y, x) column marches down the
// slices holding in[z - R .. z + R]; each input is read once.  Values outside
// the stack are zero in the ring, which drops their taps (the transpose's
// correlation has no renormalisation).  The march is unrolled by the ring
// length, so ring slots are static.
struct Taps {
    float w[16];
};

template <int R>
__global__ __launch_bounds__(256) void transpose_z_ring(const float *in, float *out, int S, long long plane, Taps t)
{
    constexpr int N = 2 * R + 1;
    const long long col = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= plane) return;
    float ring[N];
#pragma unroll
    for (int j = 0; j < N; ++j) ring[j] = 0.f;
    // slot of slice z' is (z' + R) mod N; preload slices 0 .. R - 1
#pragma unroll
    for (int zz = 0; zz < R; ++zz) ring[(zz + R) % N] = zz < S ? in[(long long)zz * plane + col] : 0.f;
    for (int zb = 0; zb < S; zb += N) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const int z = zb + k;
            if (z < S) {   // uniform
                const int zl = z + R;   // slice entering the ring
                ring[(k + 2 * R) % N] = zl < S ? in[(long long)zl * plane + col] : 0.f;
                float acc = t.w[0] * ring[(k + R) % N];
#pragma unroll
                for (int d = 1; d <= R; ++d) acc = fmaf(t.w[d], ring[(k + R - d) % N] + ring[(k + R + d) % N], acc);
                out[(long long)z * plane + col] = acc;
            }
        }
    }
}

// y pass with a register ring: one thread per (z, x) and segment of kYSeg rows,
// holding in[y - R .. y + R] (the segment's first 2R rows are read twice:
// once by this segment, once by the one above).
constexpr int kYSeg = 64;

template <int R>
__global__ __launch_bounds__(256) void transpose_y_ring(const float *in, float *out, int S, int H, int W, Taps t)
{
    constexpr int N = 2 * R + 1;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= W) return;
    const int y0 = blockIdx.y * kYSeg;
    if (y0 >= H) return;
    const int y1 = min(y0 + kYSeg, H);
    for (int z = blockIdx.z; z < S; z += gridDim.z) {
        const float *col = in + (long long)z * H * W + x;
        float *ocol = out + (long long)z * H * W + x;
        float ring[N];
        // slot of row y' is (y' - y0 + R) mod N; preload rows y0 - R .. y0 + R - 1
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) {
            const int yy = y0 - R + j;
            ring[j] = (yy >= 0 && yy < H) ? col[(long long)yy * W] : 0.f;
        }
        for (int yb = y0; yb < y1; yb += N) {
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const int y = yb + k;
                if (y < y1) {   // uniform
                    const int yl = y + R;   // row entering the ring
                    ring[(k + 2 * R) % N] = yl < H ? col[(long long)yl * W] : 0.f;
                    float acc = t.w[0] * ring[(k + R) % N];
#pragma unroll
                    for (int d = 1; d <= R; ++d) acc = fmaf(t.w[d], ring[(k + R - d) % N] + ring[(k + R + d) % N], acc);
                    ocol[(long long)y * W] = acc;
                }
            }
        }
    }
}

hipError_t launch_y_ring(const float *in, float *out, int S, int H, int W, int rxy, const float *wxy, hipStream_t s)
{
    Taps t{};
    for (int d = 0; d < 8; ++d) t.w[d] = wxy[d];
    if ((H + kYSeg - 1) / kYSeg > 65535) return hipErrorInvalidValue;   // (H <= 4 M rows)
    const dim3 grid((unsigned)((W + 255) / 256), (unsigned)((H + kYSeg - 1) / kYSeg), (unsigned)std::min(S, 65535));
    switch (rxy) {
#define GDF_YR(R) \
    case R: hipLaunchKernelGGL(transpose_y_ring<R>, grid, dim3(256), 0, s, in, out, S, H, W, t); break;
        GDF_YR(0) GDF_YR(1) GDF_YR(2) GDF_YR(3) GDF_YR(4) GDF_YR(5) GDF_YR(6) GDF_YR(7)
#undef GDF_YR
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_z_ring(const float *in, float *out, int S, int H, int W, int rz, const float *wz, hipStream_t s)
{
    Taps t{};
    for (int d = 0; d < 16; ++d) t.w[d] = wz[d];
    const long long plane = (long long)H * W;
    const dim3 grid((unsigned)((plane + 255) / 256));
    switch (rz) {
#define GDF_ZR(R) \
    case R: hipLaunchKernelGGL(transpose_z_ring<R>, grid, dim3(256), 0, s, in, out, S, plane, t); break;
        GDF_ZR(0) GDF_ZR(1) GDF_ZR(2) GDF_ZR(3) GDF_ZR(4) GDF_ZR(5) GDF_ZR(6) GDF_ZR(7) GDF_ZR(8) GDF_ZR(9)
        GDF_ZR(10) GDF_ZR(11) GDF_ZR(12)
#undef GDF_ZR
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_smooth_transpose(const float *g, float *out, float *tmp, const float *inv_d, int S, int H, int W,
                                   int rxy, int rz, const float *wxy, const float *wz, hipStream_t s)
{
    const long long n = (long long)S * H * W;
    if (n == 0) return hipSuccess;
    // x (with the 1 / D scaling at the source): g -> out; y: out -> tmp; z: tmp -> out
    XArgs a{};
    a.in = g;
    a.out = out;
    a.inv_d = inv_d;
    a.S = S;
    a.H = H;
    a.W = W;
    a.r = rxy;
    for (int d = 0; d < 8; ++d) a.w[d] = wxy[d];
    const dim3 grid((unsigned)((W + 255) / 256), (unsigned)std::min(H, 65535), (unsigned)std::min(S, 65535));
    hipLaunchKernelGGL(transpose_x_kernel, grid, dim3(256), 0, s, a);
    hipError_t e0 = hipGetLastError();
    if (e0 != hipSuccess) return e0;
    const hipError_t e = launch_y_ring(out, tmp, S, H, W, rxy, wxy, s);
    if (e != hipSuccess) return e;
    return launch_z_ring(tmp, out, S, H, W, rz, wz, s);
}

}  // namespace gdf
