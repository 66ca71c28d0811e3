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

constexpr int kSeg = 16;   // outputs per thread along y or z

struct AxisArgs {
    const float *in;
    float *out;
    const float *inv_d;   // first pass: 1 / Dz, 1 / Dy, 1 / Dx tables (S, H, W), else null
    int S, H, W;
    int axis;             // 0: x, 1: y, 2: z
    int r;                // tap radius along the axis
    float w[16];          // taps w[0..r]
};

// One thread per column x of a row, with the grid's y and z dimensions over
// the other two coordinates (no index division).  x pass: one output per
// thread (its taps are neighbours in the same cache lines).  y and z passes:
// each thread marches a segment of kSeg outputs down its line, so the taps of
// consecutive outputs are the same few rows or planes, still in the caches.
__global__ __launch_bounds__(256) void transpose_axis_kernel(AxisArgs a)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= a.W) return;
    const long long plane = (long long)a.H * a.W;
    const int len = a.axis == 0 ? a.W : (a.axis == 1 ? a.H : a.S);
    const long long stride = a.axis == 0 ? 1 : (a.axis == 1 ? (long long)a.W : plane);
    // grid y / z: (y, z) for the x pass, (segment, z) for y, (y, segment) for z
    const int gy_n = a.axis == 1 ? (a.H + kSeg - 1) / kSeg : a.H;
    const int gz_n = a.axis == 2 ? (a.S + kSeg - 1) / kSeg : a.S;
    const float *iz = a.inv_d, *iy = a.inv_d + a.S, *ix = a.inv_d + a.S + a.H;
    for (int gz = blockIdx.z; gz < gz_n; gz += gridDim.z)
        for (int gy = blockIdx.y; gy < gy_n; gy += gridDim.y) {
            int y = gy, z = gz, t0 = 0, t1 = 1;
            if (a.axis == 1) {
                t0 = gy * kSeg;
                t1 = min(t0 + kSeg, a.H);
            } else if (a.axis == 2) {
                t0 = gz * kSeg;
                t1 = min(t0 + kSeg, a.S);
            }
            for (int t = t0; t < t1; ++t) {
                if (a.axis == 1) y = t;
                else if (a.axis == 2) z = t;
                const long long i = ((long long)z * a.H + y) * a.W + x;
                const int c = a.axis == 0 ? x : (a.axis == 1 ? y : z);
                const int lo = max(-a.r, -c), hi = min(a.r, len - 1 - c);
                float acc = 0.f;
                if (a.inv_d) {
                    // the source voxel's 1 / D; along the pass axis it changes per tap
                    for (int d = lo; d <= hi; ++d) {
                        const int zz = a.axis == 2 ? z + d : z, yy = a.axis == 1 ? y + d : y;
                        const int xx = a.axis == 0 ? x + d : x;
                        acc = fmaf(a.w[d < 0 ? -d : d] * (iz[zz] * iy[yy] * ix[xx]), a.in[i + d * stride], acc);
                    }
                } else {
                    for (int d = lo; d <= hi; ++d) acc = fmaf(a.w[d < 0 ? -d : d], a.in[i + d * stride], acc);
                }
                a.out[i] = acc;
            }
        }
}

}  // namespace

hipError_t launch_smooth_transpose(const float *g, float *out, float *tmp, const float *inv_d, int S, int H, int W,
                                   int rxy, int rz, const float *wxy, const float *wz, hipStream_t s)
{
    const long long n = (long long)S * H * W;
    if (n == 0) return hipSuccess;
    AxisArgs a{};
    a.S = S;
    a.H = H;
    a.W = W;
    // x (with the 1 / D scaling at the source): g -> out; y: out -> tmp; z: tmp -> out
    const float *src[3] = {g, out, tmp};
    float *dst[3] = {out, tmp, out};
    for (int p = 0; p < 3; ++p) {
        a.axis = p;
        a.r = p == 2 ? rz : rxy;
        for (int d = 0; d < 16; ++d) a.w[d] = (p == 2 ? (d < 16 ? wz[d] : 0.f) : (d < 8 ? wxy[d] : 0.f));
        a.in = src[p];
        a.out = dst[p];
        a.inv_d = p == 0 ? inv_d : nullptr;
        const int gy = p == 1 ? (H + kSeg - 1) / kSeg : H;
        const int gz = p == 2 ? (S + kSeg - 1) / kSeg : S;
        const dim3 grid((unsigned)((W + 255) / 256), (unsigned)std::min(gy, 65535), (unsigned)std::min(gz, 65535));
        hipLaunchKernelGGL(transpose_axis_kernel, grid, dim3(256), 0, s, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace gdf
