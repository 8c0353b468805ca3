// Step for geometries given by their metric (Sec. III: the geometry enters
// the scheme only through sqrt(g), the inverse metric and the contracted
// Christoffel symbols, so any coordinate system runs by supplying them per
// node).  Same arithmetic as the per-node description in step.hip (BGK
// tau = 1/2, corrected equilibrium, Christoffel and metric-gradient forcing,
// push streaming with the wall rules), here with all six metric components,
// each varying along every axis, in two passes:
//  - general_s_kernel: S = sum_l f_l into a buffer of N floats; workgroup 0
//    first records the probes of time t and advances the step counter;
//  - general_step_kernel: one thread per node (axis 0 fastest), momentum
//    with the metric-gradient term from S and the coefficients of the six
//    axis neighbours, collision, push.
// Coefficients are FP32 planes of N values: c^2 Mhat 00, 11, 22, 01, 02, 12
// and c^2 Gamh / 2 per axis.  For axis d the metric-gradient term needs
// A^{de} = c^2 Mhat^{de} S at the neighbours along e, i.e. at x +- e_0 the
// components (d0), at x +- e_1 (d1), at x +- e_2 (d2); beyond a wall the
// node's own A is mirrored, odd for fixed walls.
#include "lbw_internal.h"

namespace lbw {
namespace {

constexpr int kBS = 256;

// component plane of Mhat^{de}
__device__ constexpr int mplane(int d, int e) {
    return d == e ? d : ((d + e == 1) ? 3 : ((d + e == 2) ? 4 : 5));
}

__device__ inline float bounce_rule(int wall, float damp, float out_l, float own_opposite) {
    return wall == LBW_BC_BOUNCEBACK ? damp * out_l : (wall == LBW_BC_FREE ? own_opposite : -out_l);
}

__global__ void general_s_kernel(GeomDev g, ProbeArgs pr, const float* __restrict__ fin, float* __restrict__ S) {
    if (blockIdx.x == 0) {
        const int64_t t = *(volatile const int64_t*)pr.tcount;
        __syncthreads();
        if (t >= 0 && t < pr.t_max) {
            for (int p = threadIdx.x; p < pr.n; p += blockDim.x) {
                const int64_t node = pr.nodes[p];
                double s = 0.0;
                for (int l = 0; l < 7; ++l) s += (double)fin[l * g.N + node];
                pr.trace[t * pr.n + p] = s / g.sqrtg[sg_index(g, node)];
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) *(volatile int64_t*)pr.tcount = t + 1;
    }
    const int64_t n = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (n >= g.N) return;
    float s = 0.f;
    for (int l = 0; l < 7; ++l) s += fin[l * g.N + n];
    S[n] = s;
}

__global__ void general_step_kernel(GeomDev g, const float* __restrict__ fin, const float* __restrict__ S,
                                    float* __restrict__ fout) {
    const int64_t n = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (n >= g.N) return;
    const int64_t N = g.N;
    const int n0 = g.n0, n1 = g.n1, n2 = g.n2;
    const int64_t plane = (int64_t)n0 * n1;
    const int x = (int)(n % n0), y = (int)((n / n0) % n1), z = (int)(n / plane);
    const float* __restrict__ T = g.tab;
    // axis neighbours: node index, or the node itself beyond a wall (then
    // the wall code is in w[a][side] and the neighbour is not read)
    int w[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    int j[3][2];
    j[0][0] = link_coord(x, +1, n0, g.bc_lo[0], g.bc_hi[0], &w[0][0]);
    j[0][1] = link_coord(x, -1, n0, g.bc_lo[0], g.bc_hi[0], &w[0][1]);
    j[1][0] = link_coord(y, +1, n1, g.bc_lo[1], g.bc_hi[1], &w[1][0]);
    j[1][1] = link_coord(y, -1, n1, g.bc_lo[1], g.bc_hi[1], &w[1][1]);
    j[2][0] = link_coord(z, +1, n2, g.bc_lo[2], g.bc_hi[2], &w[2][0]);
    j[2][1] = link_coord(z, -1, n2, g.bc_lo[2], g.bc_hi[2], &w[2][1]);
    const int own[3] = {x, y, z};
    const int64_t stride[3] = {1, n0, plane};
    int64_t nb[3][2];
    for (int a = 0; a < 3; ++a)
        for (int s = 0; s < 2; ++s) nb[a][s] = j[a][s] >= 0 ? n + (int64_t)(j[a][s] - own[a]) * stride[a] : n;
    float f[7];
    for (int l = 0; l < 7; ++l) f[l] = fin[l * N + n];
    const float Sc = S[n];
    float K[3];
    for (int d = 0; d < 3; ++d) {
        float div = 0.f;
        for (int e = 0; e < 3; ++e) {
            const int m = mplane(d, e);
            const float ahere = T[m * N + n] * Sc;
            float side[2];
            for (int s = 0; s < 2; ++s)
                side[s] = j[e][s] >= 0 ? T[m * N + nb[e][s]] * S[nb[e][s]]
                                       : (w[e][s] == LBW_BC_FIXED ? -ahere : ahere);
            div += side[0] - side[1];
        }
        K[d] = (f[1 + 2 * d] - f[2 + 2 * d]) - T[(6 + d) * N + n] * Sc - 0.25f * div;
    }
    const float cs = g.c2 * Sc;
    float fs[7];
    fs[0] = g.two_w0 * Sc - f[0];
    for (int d = 0; d < 3; ++d) {
        fs[1 + 2 * d] = cs + K[d] - f[1 + 2 * d];
        fs[2 + 2 * d] = cs - K[d] - f[2 + 2 * d];
    }
    fout[n] = fs[0];
    for (int d = 0; d < 3; ++d) {
        const int lp = 1 + 2 * d, lm = 2 + 2 * d;
        // +e_d population: to the neighbour, or reflected into -e_d here
        if (j[d][0] >= 0) fout[lp * N + nb[d][0]] = fs[lp];
        else fout[lm * N + n] = bounce_rule(w[d][0], g.damp, fs[lp], fs[lm]);
        if (j[d][1] >= 0) fout[lm * N + nb[d][1]] = fs[lm];
        else fout[lp * N + n] = bounce_rule(w[d][1], g.damp, fs[lm], fs[lp]);
    }
}

}  // namespace

hipError_t launch_step_general(const GeomDev& g, const ProbeArgs& pr, const float* fin, float* S, float* fout,
                               hipStream_t st) {
    const unsigned blocks = (unsigned)((g.N + kBS - 1) / kBS);
    hipLaunchKernelGGL(general_s_kernel, dim3(blocks), dim3(kBS), 0, st, g, pr, fin, S);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(general_step_kernel, dim3(blocks), dim3(kBS), 0, st, g, fin, S, fout);
    return hipGetLastError();
}

}  // namespace lbw
