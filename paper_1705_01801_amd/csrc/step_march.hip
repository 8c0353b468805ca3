// D3Q7 step kernel for MI355X: z-marching column tiles with LDS staging.
//
// Same arithmetic as the per-node description in step.hip (BGK tau = 1/2,
// corrected equilibrium, Christoffel and metric-gradient forcing, push
// streaming with wall rules); only the data movement differs:
//  - a workgroup of 256 threads owns a TX x TY tile of (axis 0, axis 1)
//    columns (TX = 16, 32 or 64, TY = 256 / TX) and walks a chunk of LZ
//    planes along axis 2;
//  - each thread keeps its own column's populations and S = sum_l f_l of
//    planes z-1, z, z+1 in registers, so axis-2 neighbours cost no loads;
//  - S of the tile plus a one-node ring is staged in LDS (two plane slots)
//    for the axis-0 and axis-1 neighbours; the ring's populations are
//    loaded by the first 2 TX + 2 TY threads;
//  - the coefficient row of a plane (entries x0-1 .. x0+TX, 32 bytes each)
//    is staged in LDS (three plane slots: z, z+1 and the one being filled),
//    so a node reads its own and its axis-0 neighbours' coefficients there;
//  - populations, ring and coefficient row of plane z+2 (z+1 for the ring)
//    are loaded before plane z is computed and stored after it, so their
//    latency hides behind the computation;
//  - a persistent grid walks the tiles; each XCD (blocks b with the same
//    b mod 8) gets one contiguous range of tiles, so ring and chunk-boundary
//    planes shared by neighbouring tiles are re-read from the same L2.
// Node offsets are 32-bit (the library keeps Q * N below 2^31).
#include "lbw_internal.h"

namespace lbw {
namespace {

constexpr int kThreads = 256;
constexpr int kXcds = 8;

__device__ inline void load7(const float* __restrict__ f, uint32_t N, uint32_t n, float v[7]) {
#pragma unroll
    for (int l = 0; l < 7; ++l) v[l] = f[l * N + n];
}

__device__ inline float sum7(const float v[7]) {
    return v[0] + v[1] + v[2] + v[3] + v[4] + v[5] + v[6];
}

struct TileGeom {
    int n0, n1, n2;
    uint32_t N;
    int bc_lo[3], bc_hi[3];
    float c2, two_w0, damp;
    const float4* tab4;
    int ntx, nty, lz;
};

__device__ void probe_block(const GeomDev& g, const ProbeArgs& pr, const float* __restrict__ fin) {
    const int64_t t = *(volatile const int64_t*)pr.tcount;
    __syncthreads();
    if (t >= 0 && t < pr.t_max) {
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

// value beyond a wall: mirrored, odd for fixed walls
__device__ inline float ghost(int wall, float v) { return wall == LBW_BC_FIXED ? -v : v; }

__device__ inline float bounce(int wall, float damp, float out_l, float own_lb) {
    return wall == LBW_BC_BOUNCEBACK ? damp * out_l : (wall == LBW_BC_FREE ? own_lb : -out_l);
}

// One tile of one geometry: columns [x0, x0 + TX) x [y0, y0 + TY), planes
// [z0, z0 + lz).  fin/fout point at the geometry's own population block.
template <int TX>
__device__ __forceinline__ void march_tile(const TileGeom& g, int tile, const float* __restrict__ fin,
                                           float* __restrict__ fout, float (&sS)[2][(kThreads / TX + 2) * (TX + 2)],
                                           float4 (&sE)[3][TX + 2][2]) {
    constexpr int TY = kThreads / TX;
    constexpr int W = TX + 2;
    const int n0 = g.n0, n1 = g.n1, n2 = g.n2;
    const uint32_t N = g.N;
    const uint32_t plane = (uint32_t)n0 * (uint32_t)n1;
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const float c2 = g.c2, two_w0 = g.two_w0, damp = g.damp;
    const float4* __restrict__ tab4 = g.tab4;
    {
        const int tx = tile % g.ntx;
        const int r1 = tile / g.ntx;
        const int ty = r1 % g.nty;
        const int chunk = r1 / g.nty;
        const int x0 = tx * TX, y0 = ty * TY;
        const int z0 = chunk * g.lz;
        if (z0 >= n2 || ty >= g.nty) return;  // tile outside the grid (uniform per block)
        const int z1 = min(z0 + g.lz, n2);
        const int wdt = min(TX, n0 - x0);
        const int hgt = min(TY, n1 - y0);
        const int x = x0 + lx, y = y0 + ly;
        const bool active = lx < wdt && ly < hgt;
        const uint32_t col = (uint32_t)x + (uint32_t)n0 * (uint32_t)y;

        int wx_p = 0, wx_m = 0, wy_p = 0, wy_m = 0;
        const int jx_p = link_coord(x, +1, n0, g.bc_lo[0], g.bc_hi[0], &wx_p);
        const int jx_m = link_coord(x, -1, n0, g.bc_lo[0], g.bc_hi[0], &wx_m);
        const int jy_p = link_coord(y, +1, n1, g.bc_lo[1], g.bc_hi[1], &wy_p);
        const int jy_m = link_coord(y, -1, n1, g.bc_lo[1], g.bc_hi[1], &wy_m);

        // ring node of this thread: LDS position and wrapped column, or -1
        int ring_lds = -1;
        uint32_t ring_col = 0;
        {
            const int r = threadIdx.x;
            int rx = 0, ry = 0, sx = 0, sy = 0;
            bool have = false;
            if (r < wdt) {
                rx = x0 + r; ry = y0 - 1; sx = r + 1; sy = 0; have = true;
            } else if (r >= TX && r < TX + wdt) {
                rx = x0 + (r - TX); ry = y0 + hgt; sx = r - TX + 1; sy = hgt + 1; have = true;
            } else if (r >= 2 * TX && r < 2 * TX + hgt) {
                rx = x0 - 1; ry = y0 + (r - 2 * TX); sx = 0; sy = r - 2 * TX + 1; have = true;
            } else if (r >= 2 * TX + TY && r < 2 * TX + TY + hgt) {
                rx = x0 + wdt; ry = y0 + (r - 2 * TX - TY); sx = wdt + 1; sy = r - 2 * TX - TY + 1; have = true;
            }
            if (have) {
                int w = 0;
                const int gx = rx < 0 || rx >= n0
                                   ? link_coord(rx < 0 ? 0 : n0 - 1, rx < 0 ? -1 : 1, n0, g.bc_lo[0], g.bc_hi[0], &w)
                                   : rx;
                const int gy = ry < 0 || ry >= n1
                                   ? link_coord(ry < 0 ? 0 : n1 - 1, ry < 0 ? -1 : 1, n1, g.bc_lo[1], g.bc_hi[1], &w)
                                   : ry;
                if (gx >= 0 && gy >= 0) {
                    ring_lds = sy * W + sx;
                    ring_col = (uint32_t)gx + (uint32_t)n0 * (uint32_t)gy;
                }
            }
        }
        const int my_lds = (ly + 1) * W + (lx + 1);

        // coefficient-row loader: thread t < wdt + 2 stages entry x0 - 1 + t
        int erow_x = -1;
        if ((int)threadIdx.x < wdt + 2) {
            const int ex = x0 - 1 + (int)threadIdx.x;
            int w = 0;
            erow_x = ex < 0 || ex >= n0
                         ? link_coord(ex < 0 ? 0 : n0 - 1, ex < 0 ? -1 : 1, n0, g.bc_lo[0], g.bc_hi[0], &w)
                         : ex;
        }

        int wz = 0;
        const int zm0 = link_coord(z0, -1, n2, g.bc_lo[2], g.bc_hi[2], &wz);
        const int zp0 = link_coord(z0, +1, n2, g.bc_lo[2], g.bc_hi[2], &wz);

        // ---- prologue: planes z0-1 (S only), z0, z0+1 ----
        float fc[7], fnx[7], tmp[7];
        float Sm = 0.f, Sc = 0.f, Sp = 0.f;
        float2 em = make_float2(0.f, 0.f);  // (c^2 Mhat02, c^2 Mhat22) at z-1
        if (active) {
            if (zm0 >= 0) {
                load7(fin, N, col + (uint32_t)zm0 * plane, tmp);
                Sm = sum7(tmp);
                const float4 e = tab4[2 * (x + n0 * zm0)];
                em = make_float2(e.y, e.z);
            }
            load7(fin, N, col + (uint32_t)z0 * plane, fc);
            Sc = sum7(fc);
            if (zp0 >= 0) {
                load7(fin, N, col + (uint32_t)zp0 * plane, fnx);
                Sp = sum7(fnx);
            }
        }
        if (erow_x >= 0) {
            const int e0 = 2 * (erow_x + n0 * z0);
            sE[0][threadIdx.x][0] = tab4[e0];
            sE[0][threadIdx.x][1] = tab4[e0 + 1];
            if (zp0 >= 0) {
                const int e1 = 2 * (erow_x + n0 * zp0);
                sE[1][threadIdx.x][0] = tab4[e1];
                sE[1][threadIdx.x][1] = tab4[e1 + 1];
            }
        }
        if (ring_lds >= 0) {
            load7(fin, N, ring_col + (uint32_t)z0 * plane, tmp);
            sS[0][ring_lds] = sum7(tmp);
        }
        if (active) sS[0][my_lds] = Sc;

        int es = 0;  // coefficient-row slot of plane z (z+1 in es+1 mod 3)
        for (int z = z0; z < z1; ++z) {
            const int sb = (z - z0) & 1;
            const int es1 = es == 2 ? 0 : es + 1;
            const int es2 = es1 == 2 ? 0 : es1 + 1;
            int wz_p = 0, wz_m = 0;
            const int jz_p = link_coord(z, +1, n2, g.bc_lo[2], g.bc_hi[2], &wz_p);
            const int jz_m = link_coord(z, -1, n2, g.bc_lo[2], g.bc_hi[2], &wz_m);
            const bool more = z + 1 < z1;
            int wq = 0;
            const int zq = more ? link_coord(jz_p, +1, n2, g.bc_lo[2], g.bc_hi[2], &wq) : -1;

            // prefetch plane zq (own column, coefficient row) and plane z+1 (ring)
            float fnn[7], hr[7];
            float4 ea = make_float4(0.f, 0.f, 0.f, 0.f), eb = ea;
            if (active && zq >= 0) load7(fin, N, col + (uint32_t)zq * plane, fnn);
            if (erow_x >= 0 && zq >= 0) {
                const int e2 = 2 * (erow_x + n0 * zq);
                ea = tab4[e2];
                eb = tab4[e2 + 1];
            }
            const bool ring_next = ring_lds >= 0 && more;
            if (ring_next) load7(fin, N, ring_col + (uint32_t)jz_p * plane, hr);
            __syncthreads();

            if (active) {
                const float* L = sS[sb];
                const float S = Sc;
                const float4 e_lo = sE[es][lx + 1][0];  // 00, 02, 22, 11
                const float4 e_hi = sE[es][lx + 1][1];  // g0/2, g2/2, 0, 0
                const float cM00 = e_lo.x, cM02 = e_lo.y, cM22 = e_lo.z, cM11 = e_lo.w;
                const float hG0 = e_hi.x, hG2 = e_hi.y;
                float A00p, A00m, A20p, A20m, A22p, A22m, A02p, A02m;
                if (jx_p >= 0) {
                    const float4 en = sE[es][lx + 2][0];
                    const float Sn = L[my_lds + 1];
                    A00p = en.x * Sn;
                    A20p = en.y * Sn;
                } else {
                    const float sg = ghost(wx_p, S);
                    A00p = cM00 * sg;
                    A20p = cM02 * sg;
                }
                if (jx_m >= 0) {
                    const float4 en = sE[es][lx][0];
                    const float Sn = L[my_lds - 1];
                    A00m = en.x * Sn;
                    A20m = en.y * Sn;
                } else {
                    const float sg = ghost(wx_m, S);
                    A00m = cM00 * sg;
                    A20m = cM02 * sg;
                }
                const float A11p = cM11 * (jy_p >= 0 ? L[my_lds + W] : ghost(wy_p, S));
                const float A11m = cM11 * (jy_m >= 0 ? L[my_lds - W] : ghost(wy_m, S));
                if (jz_p >= 0) {
                    const float4 en = sE[es1][lx + 1][0];
                    A02p = en.y * Sp;
                    A22p = en.z * Sp;
                } else {
                    const float sg = ghost(wz_p, S);
                    A22p = cM22 * sg;
                    A02p = cM02 * sg;
                }
                if (jz_m >= 0) {
                    A02m = em.x * Sm;
                    A22m = em.y * Sm;
                } else {
                    const float sg = ghost(wz_m, S);
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

                const uint32_t n = col + (uint32_t)z * plane;
                fout[n] = fs[0];
                if (jx_p >= 0) fout[1 * N + n + (uint32_t)(jx_p - x)] = fs[1];
                else fout[2 * N + n] = bounce(wx_p, damp, fs[1], fs[2]);
                if (jx_m >= 0) fout[2 * N + n + (uint32_t)(jx_m - x)] = fs[2];
                else fout[1 * N + n] = bounce(wx_m, damp, fs[2], fs[1]);
                if (jy_p >= 0) fout[3 * N + n + (uint32_t)((jy_p - y) * n0)] = fs[3];
                else fout[4 * N + n] = bounce(wy_p, damp, fs[3], fs[4]);
                if (jy_m >= 0) fout[4 * N + n + (uint32_t)((jy_m - y) * n0)] = fs[4];
                else fout[3 * N + n] = bounce(wy_m, damp, fs[4], fs[3]);
                if (jz_p >= 0) fout[5 * N + col + (uint32_t)jz_p * plane] = fs[5];
                else fout[6 * N + n] = bounce(wz_p, damp, fs[5], fs[6]);
                if (jz_m >= 0) fout[6 * N + col + (uint32_t)jz_m * plane] = fs[6];
                else fout[5 * N + n] = bounce(wz_m, damp, fs[6], fs[5]);
                em = make_float2(cM02, cM22);
            }

            if (more) {
                if (ring_next) sS[sb ^ 1][ring_lds] = sum7(hr);
                if (erow_x >= 0 && zq >= 0) {
                    sE[es2][threadIdx.x][0] = ea;
                    sE[es2][threadIdx.x][1] = eb;
                }
                if (active) {
                    sS[sb ^ 1][my_lds] = Sp;
                    Sm = Sc;
                    Sc = Sp;
#pragma unroll
                    for (int l = 0; l < 7; ++l) fc[l] = fnx[l];
                    if (zq >= 0) {
#pragma unroll
                        for (int l = 0; l < 7; ++l) fnx[l] = fnn[l];
                        Sp = sum7(fnn);
                    }
                }
            }
            es = es1;
        }
        __syncthreads();  // LDS reuse by the next tile
    }
}

template <int TX>
__global__ __launch_bounds__(kThreads) void step_march_kernel(GeomDev g, ProbeArgs pr, MarchPlan plan,
                                                              const float* __restrict__ fin,
                                                              float* __restrict__ fout) {
    __shared__ float sS[2][(kThreads / TX + 2) * (TX + 2)];
    __shared__ float4 sE[3][TX + 2][2];
    if (blockIdx.x == 0) probe_block(g, pr, fin);
    TileGeom tg;
    tg.n0 = g.n0;
    tg.n1 = g.n1;
    tg.n2 = g.n2;
    tg.N = (uint32_t)g.N;
    for (int a = 0; a < 3; ++a) {
        tg.bc_lo[a] = g.bc_lo[a];
        tg.bc_hi[a] = g.bc_hi[a];
    }
    tg.c2 = g.c2;
    tg.two_w0 = g.two_w0;
    tg.damp = g.damp;
    tg.tab4 = reinterpret_cast<const float4*>(g.tab);
    tg.ntx = plan.ntx;
    tg.nty = plan.nty;
    tg.lz = plan.lz;
    const int xcd = blockIdx.x % kXcds;
    const int per_xcd_blocks = gridDim.x / kXcds;
    const int t_begin = (int)(plan.tiles * xcd / kXcds);
    const int t_end = (int)(plan.tiles * (xcd + 1) / kXcds);
    for (int tile = t_begin + (int)blockIdx.x / kXcds; tile < t_end; tile += per_xcd_blocks)
        march_tile<TX>(tg, tile, fin, fout, sS, sE);
}

// Batch of geometries advanced by one launch: tiles of all geometries form
// one list (geometry h owns tiles [tile_begin, tile_begin + tiles)), split
// into one contiguous range per XCD.  Block b first records the probes of
// geometries b, b + gridDim.x, ... (one step counter per geometry).
template <int TX>
__global__ __launch_bounds__(kThreads) void step_batch_kernel(const BatchItem* __restrict__ items, int n_items,
                                                              int64_t tiles_total, BatchProbeArgs bp,
                                                              const float* __restrict__ fin,
                                                              float* __restrict__ fout) {
    __shared__ float sS[2][(kThreads / TX + 2) * (TX + 2)];
    __shared__ float4 sE[3][TX + 2][2];
    for (int h = blockIdx.x; h < n_items; h += gridDim.x) {
        const BatchItem& it = items[h];
        const int64_t t = *(volatile const int64_t*)(bp.tcount + h);
        __syncthreads();
        if (t >= 0 && t < bp.t_max) {
            const float* f = fin + it.f_off;
            for (int p = threadIdx.x; p < it.n_probes; p += blockDim.x) {
                const uint32_t node = (uint32_t)bp.nodes[it.probe_off + p];
                double s = 0.0;
                for (int l = 0; l < 7; ++l) s += (double)f[l * it.N + node];
                const uint32_t i0 = node % (uint32_t)it.n0;
                const uint32_t i2 = node / ((uint32_t)it.n0 * (uint32_t)it.n1);
                bp.trace[t * bp.stride + it.probe_off + p] = s / bp.sqrtg[it.sg_off + i0 + (uint32_t)it.n0 * i2];
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) *(volatile int64_t*)(bp.tcount + h) = t + 1;
    }
    const int xcd = blockIdx.x % kXcds;
    const int per_xcd_blocks = gridDim.x / kXcds;
    const int64_t t_begin = tiles_total * xcd / kXcds;
    const int64_t t_end = tiles_total * (xcd + 1) / kXcds;
    int h = 0;
    for (int64_t tile = t_begin + (int)blockIdx.x / kXcds; tile < t_end; tile += per_xcd_blocks) {
        // geometry owning this tile (tiles ascend, so search upward from the last one)
        if (!(tile >= items[h].tile_begin && tile < items[h].tile_begin + items[h].tiles)) {
            int lo = 0, hi = n_items - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) / 2;
                if (items[mid].tile_begin <= tile) lo = mid;
                else hi = mid - 1;
            }
            h = lo;
        }
        const BatchItem& it = items[h];
        if (tile < it.tile_begin || tile >= it.tile_begin + it.tiles) continue;  // inconsistent table: skip
        TileGeom tg;
        tg.n0 = it.n0;
        tg.n1 = it.n1;
        tg.n2 = it.n2;
        tg.N = it.N;
        for (int a = 0; a < 3; ++a) {
            tg.bc_lo[a] = it.bc_lo[a];
            tg.bc_hi[a] = it.bc_hi[a];
        }
        tg.c2 = it.c2;
        tg.two_w0 = it.two_w0;
        tg.damp = it.damp;
        tg.tab4 = bp.tab4 + 2 * (size_t)it.tab_off;
        tg.ntx = it.ntx;
        tg.nty = it.nty;
        tg.lz = it.lz;
        march_tile<TX>(tg, (int)(tile - it.tile_begin), fin + it.f_off, fout + it.f_off, sS, sE);
    }
}

}  // namespace

int march_tx_for(int n0) { return n0 <= 16 ? 16 : (n0 <= 32 ? 32 : 64); }

int march_blocks_per_cu(int tx) {
    int nb = 0;
    hipError_t e = tx == 16   ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_march_kernel<16>, kThreads, 0)
                   : tx == 32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_march_kernel<32>, kThreads, 0)
                              : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_march_kernel<64>, kThreads, 0);
    return e == hipSuccess && nb > 0 ? nb : 1;
}

hipError_t launch_step_march(const GeomDev& g, const ProbeArgs& pr, const MarchPlan& plan, const float* fin,
                             float* fout, hipStream_t st) {
    if (plan.tx == 16)
        hipLaunchKernelGGL(step_march_kernel<16>, dim3(plan.blocks), dim3(kThreads), 0, st, g, pr, plan, fin, fout);
    else if (plan.tx == 32)
        hipLaunchKernelGGL(step_march_kernel<32>, dim3(plan.blocks), dim3(kThreads), 0, st, g, pr, plan, fin, fout);
    else
        hipLaunchKernelGGL(step_march_kernel<64>, dim3(plan.blocks), dim3(kThreads), 0, st, g, pr, plan, fin, fout);
    return hipGetLastError();
}

int batch_blocks_per_cu(int tx) {
    int nb = 0;
    hipError_t e = tx == 16   ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_batch_kernel<16>, kThreads, 0)
                   : tx == 32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_batch_kernel<32>, kThreads, 0)
                              : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_batch_kernel<64>, kThreads, 0);
    return e == hipSuccess && nb > 0 ? nb : 1;
}

hipError_t launch_step_batch(const BatchItem* items, int n_items, int64_t tiles_total, int tx, int blocks,
                             const BatchProbeArgs& bp, const float* fin, float* fout, hipStream_t st) {
    if (tx == 16)
        hipLaunchKernelGGL(step_batch_kernel<16>, dim3(blocks), dim3(kThreads), 0, st, items, n_items, tiles_total,
                           bp, fin, fout);
    else if (tx == 32)
        hipLaunchKernelGGL(step_batch_kernel<32>, dim3(blocks), dim3(kThreads), 0, st, items, n_items, tiles_total,
                           bp, fin, fout);
    else
        hipLaunchKernelGGL(step_batch_kernel<64>, dim3(blocks), dim3(kThreads), 0, st, items, n_items, tiles_total,
                           bp, fin, fout);
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
