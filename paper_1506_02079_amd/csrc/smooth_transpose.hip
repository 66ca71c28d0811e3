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

// x: one thread per voxel (the taps are neighbours in the same cache lines).
// y and z: one thread per segment of kSeg voxels along the axis, marching down
// it, so the taps of consecutive outputs are the same few rows or planes,
// still in the caches (and enough segments to fill the GPU).
__global__ __launch_bounds__(256) void transpose_axis_kernel(AxisArgs a)
{
    const long long plane = (long long)a.H * a.W;
    const long long stride = a.axis == 0 ? 1 : (a.axis == 1 ? (long long)a.W : plane);
    const int len = a.axis == 0 ? a.W : (a.axis == 1 ? a.H : a.S);
    // lines along the axis: x lines are single voxels here (len 1 marched)
    const long long nlines = a.axis == 0 ? (long long)a.S * plane : (a.axis == 1 ? (long long)a.S * a.W : plane);
    const int seg = a.axis == 0 ? 1 : kSeg;
    const int nseg = (len + seg - 1) / seg;
    const long long nwork = a.axis == 0 ? nlines : nlines * nseg;
    for (long long wi = (long long)blockIdx.x * blockDim.x + threadIdx.x; wi < nwork;
         wi += (long long)gridDim.x * blockDim.x) {
        // segments outermost, so neighbouring threads take neighbouring lines
        const long long l = a.axis == 0 ? wi : wi % nlines;
        const int t0 = a.axis == 0 ? 0 : (int)(wi / nlines) * seg;
        const int t1 = a.axis == 0 ? 1 : min(t0 + seg, len);
        long long base;   // index of the line's first voxel
        if (a.axis == 0) base = l;
        else if (a.axis == 1) base = (l / a.W) * plane + (l % a.W);   // (z, x)
        else base = l;                                               // (y, x) in plane 0
        for (int t = t0; t < t1; ++t) {
            const long long i = base + (long long)t * (a.axis == 0 ? 0 : stride);
            const int x = (int)(i % a.W);
            const int y = (int)((i / a.W) % a.H);
            const int z = (int)(i / plane);
            const int c = a.axis == 0 ? x : (a.axis == 1 ? y : z);
            const int lo = max(-a.r, -c), hi = min(a.r, len - 1 - c);
            float acc = 0.f;
            if (a.inv_d) {
                // the source voxel's 1 / D; along the pass axis it changes per tap
                const float *iz = a.inv_d;
                const float *iy = a.inv_d + a.S;
                const float *ix = a.inv_d + a.S + a.H;
                for (int d = lo; d <= hi; ++d) {
                    const int zz = a.axis == 2 ? z + d : z, yy = a.axis == 1 ? y + d : y, xx = a.axis == 0 ? x + d : x;
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
        const long long lines = p == 0 ? n : (p == 1 ? (long long)S * W * ((H + kSeg - 1) / kSeg)
                                                     : (long long)H * W * ((S + kSeg - 1) / kSeg));
        const int blocks = (int)std::min<long long>((lines + 255) / 256, 65536);
        hipLaunchKernelGGL(transpose_axis_kernel, dim3(blocks), dim3(256), 0, s, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace gdf
