// D3Q7 step kernel for MI355X: z-marching column tiles with an LDS halo.
//
// Same arithmetic as the per-node description in step.hip (BGK tau = 1/2,
// corrected equilibrium, Christoffel and metric-gradient forcing, push
// streaming with wall rules); only the data movement differs:
//  - a workgroup of 256 threads owns a TX x TY tile of (axis 0, axis 1)
//    columns and walks a chunk of LZ planes along axis 2;
//  - each thread keeps its own column's populations and S = sum_l f_l of
//    planes z-1, z, z+1 in registers, so axis-2 neighbours cost nothing;
//  - S of the tile plus a one-node ring is staged in LDS (double-buffered
//    by plane parity) for the axis-0 and axis-1 neighbours; ring nodes are
//    loaded by the first 2 TX + 2 TY threads;
//  - the next plane's populations and coefficient entry are loaded before
//    the current plane is computed, so their latency hides behind it;
//  - a persistent grid walks the tiles; each XCD (blocks b with the same
//    b mod 8) gets one contiguous range of tiles, so ring and chunk-boundary
//    planes shared by neighbouring tiles are re-read from the same L2.
#include "lbw_internal.h"

namespace lbw {
namespace {

constexpr int kThreads = 256;
constexpr int kXcds = 8;

__device__ inline void load7(const float* __restrict__ f, int64_t N, int64_t n, float v[7]) {
#pragma unroll
    for (int l = 0; l < 7; ++l) v[l] = f[l * N + n];
}

__device__ inline float sum7(const float v[7]) {
    return v[0] + v[1] + v[2] + v[3] + v[4] + v[5] + v[6];
}

__device__ void probe_block(const GeomDev& g, const ProbeArgs& pr, const float* __restrict__ fin) {
    const int64_t t = *(volatile const int64_t*)pr.tcount;
    __syncthreads();
    if (t < pr.t_max) {
        for (int p = threadIdx.x; p < pr.n; p += blockDim.x) {
            const int64_t node = pr.nodes[p];
            double s = 0.0;
            for (int l = 0; l < 7; ++l) s += (double)fin[l * g.N + node];
            const int i0 = (int)(node % g.n0);
            const int i2 = (int)(node / ((int64_t)g.n0 * g.n1));
            pr.trace[t * pr.n + p] = s / g.sqrtg[i0 + g.n0 * i2];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) *(volatile int64_t*)pr.tcount = t + 1;
}

template <int TX>
__global__ __launch_bounds__(kThreads) void step_march_kernel(GeomDev g, ProbeArgs pr, MarchPlan plan,
                                                              const float* __restrict__ fin,
                                                              float* __restrict__ fout) {
    constexpr int TY = kThreads / TX;
    constexpr int W = TX + 2;
    __shared__ float lds[2][(TY + 2) * W];

    if (blockIdx.x == 0) probe_block(g, pr, fin);

    const int n0 = g.n0, n1 = g.n1, n2 = g.n2;
    const int64_t N = g.N;
    const int64_t plane = (int64_t)n0 * n1;
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const float c2 = g.c2, two_w0 = g.two_w0, damp = g.damp;

    // tiles of this block: XCD-contiguous ranges
    const int xcd = blockIdx.x % kXcds;
    const int slot = blockIdx.x / kXcds;
    const int per_xcd_blocks = gridDim.x / kXcds;
    const int64_t t_begin = (int64_t)plan.tiles * xcd / kXcds;
    const int64_t t_end = (int64_t)plan.tiles * (xcd + 1) / kXcds;

    for (int64_t tile = t_begin + slot; tile < t_end; tile += per_xcd_blocks) {
        const int tx = (int)(tile % plan.ntx);
        const int64_t r1 = tile / plan.ntx;
        const int ty = (int)(r1 % plan.nty);
        const int chunk = (int)(r1 / plan.nty);
        const int x0 = tx * TX, y0 = ty * TY;
        const int z0 = chunk * plan.lz;
        const int z1 = min(z0 + plan.lz, n2);
        const int wdt = min(TX, n0 - x0);
        const int hgt = min(TY, n1 - y0);
        const int x = x0 + lx, y = y0 + ly;
        const bool active = lx < wdt && ly < hgt;
        const int64_t col = (int64_t)x + (int64_t)n0 * y;  // node index at plane 0

        // wall / wrap information of this thread's links in x and y
        int wx_p = 0, wx_m = 0, wy_p = 0, wy_m = 0;
        const int jx_p = link_coord(x, +1, n0, g.bc_lo[0], g.bc_hi[0], &wx_p);
        const int jx_m = link_coord(x, -1, n0, g.bc_lo[0], g.bc_hi[0], &wx_m);
        const int jy_p = link_coord(y, +1, n1, g.bc_lo[1], g.bc_hi[1], &wy_p);
        const int jy_m = link_coord(y, -1, n1, g.bc_lo[1], g.bc_hi[1], &wy_m);

        // ring node handled by this thread (if any): position in the LDS
        // window and its (wrapped) global coordinates
        int ring_lds = -1;
        int64_t ring_col = 0;
        {
            const int r = threadIdx.x;
            int rx = 0, ry = 0, sx = 0, sy = 0;  // sx, sy: LDS window coords (1-based interior)
            bool have = false;
            if (r < wdt) {  // below
                rx = x0 + r; ry = y0 - 1; sx = r + 1; sy = 0; have = true;
            } else if (r >= TX && r < TX + wdt) {  // above
                rx = x0 + (r - TX); ry = y0 + hgt; sx = r - TX + 1; sy = hgt + 1; have = true;
            } else if (r >= 2 * TX && r < 2 * TX + hgt) {  // left
                rx = x0 - 1; ry = y0 + (r - 2 * TX); sx = 0; sy = r - 2 * TX + 1; have = true;
            } else if (r >= 2 * TX + TY && r < 2 * TX + TY + hgt) {  // right
                rx = x0 + wdt; ry = y0 + (r - 2 * TX - TY); sx = wdt + 1; sy = r - 2 * TX - TY + 1; have = true;
            }
            if (have) {
                int w = 0;
                const int gx = rx < 0 || rx >= n0 ? link_coord(rx < 0 ? 0 : n0 - 1, rx < 0 ? -1 : 1, n0, g.bc_lo[0],
                                                               g.bc_hi[0], &w)
                                                  : rx;
                const int gy = ry < 0 || ry >= n1 ? link_coord(ry < 0 ? 0 : n1 - 1, ry < 0 ? -1 : 1, n1, g.bc_lo[1],
                                                               g.bc_hi[1], &w)
                                                  : ry;
                if (gx >= 0 && gy >= 0) {
                    ring_lds = sy * W + sx;
                    ring_col = (int64_t)gx + (int64_t)n0 * gy;
                }
            }
        }
        const int my_lds = (ly + 1) * W + (lx + 1);

        // wrapped plane index (or -1 beyond a wall)
        auto zlink = [&](int z, int s, int* wall) { return link_coord(z, s, n2, g.bc_lo[2], g.bc_hi[2], wall); };
        auto entry = [&](int xx, int zz) { return g.tab + (size_t)(xx + n0 * zz) * kTabF32; };

        // ---- prologue ----
        int wz_dummy = 0;
        const int zm0 = zlink(z0, -1, &wz_dummy);
        float fc[7], fnx[7], tmp[7];
        float Sm = 0.f, Sc = 0.f, Sp = 0.f;
        float em22 = 0.f, em02 = 0.f;
        float ec[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, ep[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (active) {
            if (zm0 >= 0) {
                load7(fin, N, col + zm0 * plane, tmp);
                Sm = sum7(tmp);
                const float* e = entry(x, zm0);
                em22 = e[2];
                em02 = e[3];
            }
            load7(fin, N, col + z0 * plane, fc);
            Sc = sum7(fc);
            const float* e = entry(x, z0);
#pragma unroll
            for (int i = 0; i < 6; ++i) ec[i] = e[i];
        }
        int wdum = 0;
        const int zp0 = zlink(z0, +1, &wdum);
        if (active && zp0 >= 0) {
            load7(fin, N, col + zp0 * plane, fnx);
            Sp = sum7(fnx);
            const float* e = entry(x, zp0);
#pragma unroll
            for (int i = 0; i < 6; ++i) ep[i] = e[i];
        }
        if (ring_lds >= 0) {
            load7(fin, N, ring_col + z0 * plane, tmp);
            lds[z0 & 1][ring_lds] = sum7(tmp);
        }
        if (active) lds[z0 & 1][my_lds] = Sc;

        for (int z = z0; z < z1; ++z) {
            const int b = z & 1;
            int wz_p = 0, wz_m = 0;
            const int jz_p = zlink(z, +1, &wz_p);
            const int jz_m = zlink(z, -1, &wz_m);
            // prefetch: own column at z+2 (needed while z+1 < z1), ring at z+1
            float fnn[7], hr[7];
            float en[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            int wq = 0;
            const int zq = jz_p >= 0 && z + 1 < z1 ? zlink(jz_p, +1, &wq) : -1;
            if (active && zq >= 0) {
                load7(fin, N, col + zq * plane, fnn);
                const float* e = entry(x, zq);
#pragma unroll
                for (int i = 0; i < 6; ++i) en[i] = e[i];
            }
            const bool ring_next = ring_lds >= 0 && z + 1 < z1;
            if (ring_next) load7(fin, N, ring_col + jz_p * plane, hr);
            float nx00p = 0.f, nx02p = 0.f, nx00m = 0.f, nx02m = 0.f;
            if (active) {
                if (jx_p >= 0) {
                    const float* e = entry(jx_p, z);
                    nx00p = e[0];
                    nx02p = e[3];
                }
                if (jx_m >= 0) {
                    const float* e = entry(jx_m, z);
                    nx00m = e[0];
                    nx02m = e[3];
                }
            }
            __syncthreads();

            if (active) {
                const float* L = lds[b];
                const float S = Sc;
                const float cM00 = ec[0], cM11 = ec[1], cM22 = ec[2], cM02 = ec[3], hG0 = ec[4], hG2 = ec[5];
                float A00p, A00m, A20p, A20m, A11p, A11m, A22p, A22m, A02p, A02m;
                if (jx_p >= 0) {
                    const float Sn = L[my_lds + 1];
                    A00p = nx00p * Sn;
                    A20p = nx02p * Sn;
                } else {
                    const float sg = wx_p == LBW_BC_FIXED ? -S : S;
                    A00p = cM00 * sg;
                    A20p = cM02 * sg;
                }
                if (jx_m >= 0) {
                    const float Sn = L[my_lds - 1];
                    A00m = nx00m * Sn;
                    A20m = nx02m * Sn;
                } else {
                    const float sg = wx_m == LBW_BC_FIXED ? -S : S;
                    A00m = cM00 * sg;
                    A20m = cM02 * sg;
                }
                A11p = cM11 * (jy_p >= 0 ? L[my_lds + W] : (wy_p == LBW_BC_FIXED ? -S : S));
                A11m = cM11 * (jy_m >= 0 ? L[my_lds - W] : (wy_m == LBW_BC_FIXED ? -S : S));
                if (jz_p >= 0) {
                    A22p = ep[2] * Sp;
                    A02p = ep[3] * Sp;
                } else {
                    const float sg = wz_p == LBW_BC_FIXED ? -S : S;
                    A22p = cM22 * sg;
                    A02p = cM02 * sg;
                }
                if (jz_m >= 0) {
                    A22m = em22 * Sm;
                    A02m = em02 * Sm;
                } else {
                    const float sg = wz_m == LBW_BC_FIXED ? -S : S;
                    A22m = cM22 * sg;
                    A02m = cM02 * sg;
                }
                const float K0 = (fc[1] - fc[2]) - hG0 * S - 0.25f * (A00p - A00m) - 0.25f * (A02p - A02m);
                const float K1 = (fc[3] - fc[4]) - 0.25f * (A11p - A11m);
                const float K2 = (fc[5] - fc[6]) - hG2 * S - 0.25f * ((A22p - A22m) + (A20p - A20m));
                const float cs = c2 * S;
                float fs[7];
                fs[0] = two_w0 * S - fc[0];
                fs[1] = cs + K0 - fc[1];
                fs[2] = cs - K0 - fc[2];
                fs[3] = cs + K1 - fc[3];
                fs[4] = cs - K1 - fc[4];
                fs[5] = cs + K2 - fc[5];
                fs[6] = cs - K2 - fc[6];

                const int64_t n = col + (int64_t)z * plane;
                fout[n] = fs[0];
                // +-e0
                if (jx_p >= 0) fout[1 * N + n + (jx_p - x)] = fs[1];
                else fout[2 * N + n] = wx_p == LBW_BC_BOUNCEBACK ? damp * fs[1] : (wx_p == LBW_BC_FREE ? fs[2] : -fs[1]);
                if (jx_m >= 0) fout[2 * N + n + (jx_m - x)] = fs[2];
                else fout[1 * N + n] = wx_m == LBW_BC_BOUNCEBACK ? damp * fs[2] : (wx_m == LBW_BC_FREE ? fs[1] : -fs[2]);
                // +-e1
                if (jy_p >= 0) fout[3 * N + n + (int64_t)(jy_p - y) * n0] = fs[3];
                else fout[4 * N + n] = wy_p == LBW_BC_BOUNCEBACK ? damp * fs[3] : (wy_p == LBW_BC_FREE ? fs[4] : -fs[3]);
                if (jy_m >= 0) fout[4 * N + n + (int64_t)(jy_m - y) * n0] = fs[4];
                else fout[3 * N + n] = wy_m == LBW_BC_BOUNCEBACK ? damp * fs[4] : (wy_m == LBW_BC_FREE ? fs[3] : -fs[4]);
                // +-e2
                if (jz_p >= 0) fout[5 * N + col + (int64_t)jz_p * plane] = fs[5];
                else fout[6 * N + n] = wz_p == LBW_BC_BOUNCEBACK ? damp * fs[5] : (wz_p == LBW_BC_FREE ? fs[6] : -fs[5]);
                if (jz_m >= 0) fout[6 * N + col + (int64_t)jz_m * plane] = fs[6];
                else fout[5 * N + n] = wz_m == LBW_BC_BOUNCEBACK ? damp * fs[6] : (wz_m == LBW_BC_FREE ? fs[5] : -fs[6]);
            }

            // stage plane z+1 and rotate the register window
            if (z + 1 < z1) {
                if (ring_next) lds[b ^ 1][ring_lds] = sum7(hr);
                if (active) {
                    lds[b ^ 1][my_lds] = Sp;
                    Sm = Sc;
                    Sc = Sp;
                    em22 = ec[2];
                    em02 = ec[3];
#pragma unroll
                    for (int i = 0; i < 6; ++i) ec[i] = ep[i];
#pragma unroll
                    for (int l = 0; l < 7; ++l) fc[l] = fnx[l];
                    if (zq >= 0) {
#pragma unroll
                        for (int l = 0; l < 7; ++l) fnx[l] = fnn[l];
                        Sp = sum7(fnn);
#pragma unroll
                        for (int i = 0; i < 6; ++i) ep[i] = en[i];
                    }
                }
            }
        }
        __syncthreads();  // LDS reuse by the next tile
    }
}

}  // namespace

int march_tx_for(int n0) { return n0 <= 32 ? 32 : 64; }

int march_blocks_per_cu(int tx) {
    int nb = 0;
    hipError_t e = tx == 32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_march_kernel<32>, kThreads, 0)
                            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_march_kernel<64>, kThreads, 0);
    return e == hipSuccess && nb > 0 ? nb : 1;
}

hipError_t launch_step_march(const GeomDev& g, const ProbeArgs& pr, const MarchPlan& plan, const float* fin,
                             float* fout, hipStream_t st) {
    if (plan.tx == 32)
        hipLaunchKernelGGL(step_march_kernel<32>, dim3(plan.blocks), dim3(kThreads), 0, st, g, pr, plan, fin, fout);
    else
        hipLaunchKernelGGL(step_march_kernel<64>, dim3(plan.blocks), dim3(kThreads), 0, st, g, pr, plan, fin, fout);
    return hipGetLastError();
}

MarchPlan make_march_plan(const GeomDev& g, int tx, int lz, int blocks) {
    MarchPlan p{};
    p.tx = tx;
    p.ty = kThreads / tx;
    p.lz = lz < 1 ? 1 : lz;
    p.ntx = (g.n0 + p.tx - 1) / p.tx;
    p.nty = (g.n1 + p.ty - 1) / p.ty;
    p.nchunks = (g.n2 + p.lz - 1) / p.lz;
    p.tiles = (int64_t)p.ntx * p.nty * p.nchunks;
    int b = blocks < kXcds ? kXcds : blocks;
    b = (b / kXcds) * kXcds;
    const int64_t cap = ((p.tiles + kXcds - 1) / kXcds) * kXcds;
    if (b > cap) b = (int)cap;
    if (b < kXcds) b = kXcds;
    p.blocks = b;
    return p;
}

}  // namespace lbw
