// Driven sources and response intensity (Sec. IV.A and IV.C: a pressure,
// or the flux of an oscillating plate, imposed at chosen nodes as a harmonic
// function of time, and the largest pressure seen at a probe once the driven
// field is steady, which the paper's frequency sweeps plot against the drive
// frequency).
#include "march_common.h"

namespace lbw {
namespace {

// One thread per source node, imposed at the time read from the node's step
// counter by drive_node (pressure kind 0, flux along axis a kind 1 + a; a0,
// a1 as in SourceEntry).
template <int Q>
__device__ void drive_entry(const SourceEntry& s, int64_t t, float* __restrict__ p) {
    float v[Q];
#pragma unroll
    for (int l = 0; l < Q; ++l) v[l] = p[(uint64_t)l * s.N];
    march::drive_node<Q>(s.kind, s.a0, s.a1, s.omega, t, v);
#pragma unroll
    for (int l = 0; l < Q; ++l) p[(uint64_t)l * s.N] = v[l];
}

__global__ void source_kernel(const SourceEntry* __restrict__ src, int n, const int64_t* __restrict__ counters,
                              float* __restrict__ f) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const SourceEntry s = src[i];
    const int64_t t = counters[s.counter];
    if (s.q == 5) drive_entry<5>(s, t, f + s.f_off);
    else drive_entry<7>(s, t, f + s.f_off);
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
