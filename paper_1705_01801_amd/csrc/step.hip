// One time step of the curvilinear wave LBM (BGK, tau = 1/2), fused
// collide-and-push-stream with walls, plus probe recording.
//
// Per node x (Sec. III; c_s = c, w_0 = 1 - D c^2, w_l = c^2/2):
//   S   = sqrt(g) P = sum_l f_l
//   A^{de} = c^2 S Mhat^{de}            (metric part of the stress)
//   K_d = sqrt(g) J'^d = f_{+d} - f_{-d} - (c^2/2) S Gamh^d
//         - (1/4) sum_e [A^{de}(x + e_e) - A^{de}(x - e_e)]
//   f*_0 = 2 w_0 S - f_0,  f*_{+-d} = c^2 S +- K_d - f_{+-d}   (2 f^eq - f)
//   push: f_l(x + xi_l, t + 1) = f*_l(x); a link that crosses a wall feeds
//   the opposite population at x: bounce-back D f*_l, free f*_{lbar},
//   fixed -f*_l.
// Beyond a wall A is mirrored: even for bounce-back and free walls, odd for
// fixed walls.  The gradient uses S of the same (pre-collision) time level.
#include "lbw_internal.h"

namespace lbw {
namespace {

constexpr int kBlock = 256;

// Probe block: trace[t][p] = sum_l f_l(node_p) / sqrt(g), t read from the
// device step counter, which is then advanced.
__device__ void record_probes(const GeomDev& g, const ProbeArgs& pr, const float* __restrict__ fin) {
    const int64_t t = *(volatile const int64_t*)pr.tcount;
    __syncthreads();
    if (t >= 0 && t < pr.t_max) {
        const int Q = 2 * g.dim + 1;
        for (int p = threadIdx.x; p < pr.n; p += blockDim.x) {
            const int64_t node = pr.nodes[p];
            double s = 0.0;
            for (int l = 0; l < Q; ++l) s += (double)fin[l * g.N + node];
            pr.trace[t * pr.n + p] = s / g.sqrtg[sg_index(g, node)];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) *(volatile int64_t*)pr.tcount = t + 1;
}

template <int Q>
__device__ inline float node_sum(const float* __restrict__ f, int64_t N, int64_t m) {
    float s = f[m];
#pragma unroll
    for (int l = 1; l < Q; ++l) s += f[l * N + m];
    return s;
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void step_simple_kernel(GeomDev g, ProbeArgs pr, const float* __restrict__ fin,
                                                            float* __restrict__ fout) {
    constexpr int Q = 2 * DIM + 1;
    if (blockIdx.x == gridDim.x - 1) {
        record_probes(g, pr, fin);
        return;
    }
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    const int64_t N = g.N;
    const int n0 = g.n0, n1 = g.n1, n2 = g.n2;
    const int i0 = (int)(n % n0);
    const int64_t rest = n / n0;
    const int i1 = (int)(rest % n1);
    const int i2 = (int)(rest / n1);
    const int64_t plane = (int64_t)n0 * n1;

    float f[Q];
#pragma unroll
    for (int l = 0; l < Q; ++l) f[l] = fin[l * N + n];
    float S = f[0];
#pragma unroll
    for (int l = 1; l < Q; ++l) S += f[l];

    const float* te = g.tab + (size_t)(i0 + n0 * i2) * kTabF32;
    const float cM00 = te[0], cM02 = te[1], cM22 = te[2], cM11 = te[3], hG0 = te[4], hG2 = te[5];

    // axis 0 neighbours: A^{00} and A^{20}
    float A00[2], A20[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const int s = side == 0 ? 1 : -1;
        int wall = 0;
        const int j = link_coord(i0, s, n0, g.bc_lo[0], g.bc_hi[0], &wall);
        if (j >= 0) {
            const float Sn = node_sum<Q>(fin, N, n + (j - i0));
            const float* tn = g.tab + (size_t)(j + n0 * i2) * kTabF32;
            A00[side] = tn[0] * Sn;
            A20[side] = tn[1] * Sn;
        } else {
            const float sg = wall == LBW_BC_FIXED ? -1.0f : 1.0f;
            A00[side] = sg * cM00 * S;
            A20[side] = sg * cM02 * S;
        }
    }
    // axis 1 neighbours: A^{11} (coefficients do not depend on i1)
    float A11[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const int s = side == 0 ? 1 : -1;
        int wall = 0;
        const int j = link_coord(i1, s, n1, g.bc_lo[1], g.bc_hi[1], &wall);
        if (j >= 0) {
            A11[side] = cM11 * node_sum<Q>(fin, N, n + (int64_t)(j - i1) * n0);
        } else {
            A11[side] = (wall == LBW_BC_FIXED ? -cM11 : cM11) * S;
        }
    }
    float K0 = (f[1] - f[2]) - hG0 * S - 0.25f * (A00[0] - A00[1]);
    float K1 = (f[3] - f[4]) - 0.25f * (A11[0] - A11[1]);
    float K2 = 0.0f;
    if constexpr (DIM == 3) {
        float A22[2], A02[2];
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int s = side == 0 ? 1 : -1;
            int wall = 0;
            const int j = link_coord(i2, s, n2, g.bc_lo[2], g.bc_hi[2], &wall);
            if (j >= 0) {
                const float Sn = node_sum<Q>(fin, N, n + (int64_t)(j - i2) * plane);
                const float* tn = g.tab + (size_t)(i0 + n0 * j) * kTabF32;
                A22[side] = tn[2] * Sn;
                A02[side] = tn[1] * Sn;
            } else {
                const float sg = wall == LBW_BC_FIXED ? -1.0f : 1.0f;
                A22[side] = sg * cM22 * S;
                A02[side] = sg * cM02 * S;
            }
        }
        K0 -= 0.25f * (A02[0] - A02[1]);
        K2 = (f[5] - f[6]) - hG2 * S - 0.25f * ((A22[0] - A22[1]) + (A20[0] - A20[1]));
    }

    const float cs = g.c2 * S;
    float fs[Q];
    fs[0] = g.two_w0 * S - f[0];
    fs[1] = cs + K0 - f[1];
    fs[2] = cs - K0 - f[2];
    fs[3] = cs + K1 - f[3];
    fs[4] = cs - K1 - f[4];
    if constexpr (DIM == 3) {
        fs[5] = cs + K2 - f[5];
        fs[6] = cs - K2 - f[6];
    }

    fout[n] = fs[0];
    const int idx[3] = {i0, i1, i2};
    const int nn[3] = {n0, n1, n2};
    const int64_t stride[3] = {1, n0, plane};
#pragma unroll
    for (int l = 1; l < Q; ++l) {
        const int a = (l - 1) >> 1;
        const int s = (l & 1) ? 1 : -1;
        const int lb = (l & 1) ? l + 1 : l - 1;
        int wall = 0;
        const int j = link_coord(idx[a], s, nn[a], g.bc_lo[a], g.bc_hi[a], &wall);
        if (j >= 0) {
            fout[l * N + n + (int64_t)(j - idx[a]) * stride[a]] = fs[l];
        } else if (wall == LBW_BC_BOUNCEBACK) {
            fout[lb * N + n] = g.damp * fs[l];
        } else if (wall == LBW_BC_FREE) {
            fout[lb * N + n] = fs[lb];
        } else {
            fout[lb * N + n] = -fs[l];
        }
    }
}

}  // namespace

hipError_t launch_step(const GeomDev& g, const ProbeArgs& pr, const float* fin, float* fout, hipStream_t st) {
    const unsigned blocks = (unsigned)((g.N + kBlock - 1) / kBlock) + 1;  // + probe block
    if (g.dim == 3)
        hipLaunchKernelGGL(step_simple_kernel<3>, dim3(blocks), dim3(kBlock), 0, st, g, pr, fin, fout);
    else
        hipLaunchKernelGGL(step_simple_kernel<2>, dim3(blocks), dim3(kBlock), 0, st, g, pr, fin, fout);
    return hipGetLastError();
}

}  // namespace lbw
