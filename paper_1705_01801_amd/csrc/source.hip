// Driven sources and response intensity (Sec. IV.A and IV.C: a pressure,
// or the flux of an oscillating plate, imposed at chosen nodes as a harmonic
// function of time, and the largest pressure seen at a probe once the driven
// field is steady, which the paper's frequency sweeps plot against the drive
// frequency).
#include "lbw_internal.h"

namespace lbw {
namespace {

// One thread per source node, v = sin(omega t) with t read from the node's
// step counter.  Pressure (kind 0): the populations are put at rest at the
// pressure amplitude v (a0, a1 hold amplitude w_0 sqrt(g) and amplitude
// w sqrt(g)).  Flux along axis a (kind 1 + a): the node keeps its zeroth
// moment S and takes the equilibrium whose first moment is sqrt(g) times
// amplitude v along a, f_l = w_l S plus or minus a0 v on the two links of
// axis a (a0 = amplitude sqrt(g) / 2, a1 = w, w_0 = 1 - (q - 1) w).
__global__ void source_kernel(const SourceEntry* __restrict__ src, int n, const int64_t* __restrict__ counters,
                              float* __restrict__ f) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const SourceEntry s = src[i];
    const int64_t t = counters[s.counter];
    const double v = sin(s.omega * (double)t);
    float* p = f + s.f_off;
    if (s.kind == 0) {
        p[0] = (float)(s.a0 * v);
        const float u = (float)(s.a1 * v);
        for (int l = 1; l < s.q; ++l) p[(uint64_t)l * s.N] = u;
        return;
    }
    double S = 0.0;
    for (int l = 0; l < s.q; ++l) S += (double)p[(uint64_t)l * s.N];
    const double h = s.a0 * v;
    p[0] = (float)((1.0 - (s.q - 1) * s.a1) * S);
    for (int l = 1; l < s.q; ++l) {
        double val = s.a1 * S;
        if ((l - 1) / 2 == s.kind - 1) val += (l & 1) ? h : -h;
        p[(uint64_t)l * s.N] = (float)val;
    }
}

// NaN-propagating maximum of |x|
__device__ inline double absmax(double a, double x) {
    const double b = fabs(x);
    return (b > a || b != b) ? b : a;
}

// One workgroup per trace column: the largest |trace[t][col]| over rows
// [t0, t1) (a NaN anywhere in the window gives NaN).
__global__ void amplitude_kernel(const double* __restrict__ trace, int64_t stride, int64_t t0, int64_t t1,
                                 double* __restrict__ out) {
    __shared__ double red[256];
    const int64_t col = blockIdx.x;
    double m = 0.0;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += 256) m = absmax(m, trace[t * stride + col]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = absmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[col] = red[0];
}

}  // namespace

hipError_t launch_sources(const SourceEntry* src, int n, const int64_t* counters, float* f, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(source_kernel, dim3((n + 255) / 256), dim3(256), 0, st, src, n, counters, f);
    return hipGetLastError();
}

hipError_t launch_amplitude(const double* trace, int64_t stride, int64_t cols, int64_t t0, int64_t t1, double* out,
                            hipStream_t st) {
    if (cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(amplitude_kernel, dim3((unsigned)cols), dim3(256), 0, st, trace, stride, t0, t1, out);
    return hipGetLastError();
}

}  // namespace lbw
