// D3Q7 step kernel for MI355X: z-marching column tiles with LDS staging.
//
// Same arithmetic as the per-node description in step.hip (BGK tau = 1/2,
// corrected equilibrium, Christoffel and metric-gradient forcing, push
// streaming with wall rules); only the data movement differs:
//  - a workgroup of NT = 256 or 512 threads owns a TX x TY tile of (axis 0,
//    axis 1) columns (TX = 16, 32 or 64, TY = NT / TX) and walks a chunk of
//    LZ planes along axis 2 (the batch kernel uses NT = 256);
//  - each thread keeps its own column's populations and S = sum_l f_l of
//    planes z-1, z, z+1 in registers, so axis-2 neighbours cost no loads;
//  - S of the tile plus a one-node ring is staged in LDS (two plane slots)
//    for the axis-0 and axis-1 neighbours; the ring's populations are
//    loaded by the first 2 TX + 2 TY threads;
//  - the coefficient row of a plane (entries x0-1 .. x0+TX, 32 bytes each)
//    is staged in LDS (three plane slots: z, z+1 and the one being filled),
//    so a node reads its own and its axis-0 neighbours' coefficients there;
//  - loads run one plane step ahead of their use: while plane z is
//    computed, the own column of plane z+2, the ring of plane z+2 and the
//    coefficient row of plane z+3 are in flight, and what plane z+1 needs
//    (loaded during plane z-1) is consumed; the loop is unrolled by three so
//    the register sets rotate by name, not by copies;
//  - every load and store of the plane loop is a buffer instruction issued by
//    every lane with a 32-bit byte offset from the geometry's own base;
//    disabled ones carry an offset outside the buffer, which the hardware
//    range check turns into a zero load or a dropped store.  With no branch
//    around a memory operation the compiler's wait counts stay exact (a
//    branch makes it drain every outstanding access at the join), and no
//    access can leave the geometry's buffers;
//  - a persistent grid walks the tiles; each XCD (blocks b with the same
//    b mod 8) gets one contiguous range of tiles, so ring and chunk-boundary
//    planes shared by neighbouring tiles are re-read from the same L2.
// Byte offsets are 32-bit: the library keeps 4 Q N below 2^31.
#include <type_traits>

#include "march_common.h"

namespace lbw {
namespace {

constexpr int kBatchThreads = 256;

using namespace march;

struct TileGeom {
    int n0, n1, n2;
    uint32_t N;
    int bc_lo[3], bc_hi[3];
    float c2, two_w0, damp;
    const float4* tab4;
    int ntx, nty, lz;
    int rtx, rty;  // tile width and height when they are run-time values
    // driven nodes of the geometry (batch tiles): src_count of them on planes
    // src_zlo .. src_zhi, imposed at time src_t; src_map holds, for each node
    // of those planes (plane-major), its entry in src or -1
    const BatchSource* src;
    const int32_t* src_map;
    int src_count, src_zlo, src_zhi;
    int64_t src_t;
};

// Imposes the driven value on populations v of the node in column `col` of
// plane z, loaded by this lane (on), when that node is driven.  The plane
// test is uniform, so tiles and planes without driven nodes skip it; a
// driven plane costs one map load per lane.
template <bool SRC>
__device__ __forceinline__ void drive_loaded(const TileGeom& g, int z, bool on, uint32_t col, float (&v)[7]) {
    if constexpr (SRC) {
        if (g.src_count > 0 && z >= g.src_zlo && z <= g.src_zhi) {
            const uint32_t plane = (uint32_t)g.n0 * (uint32_t)g.n1;
            const int hit = on ? g.src_map[(uint32_t)(z - g.src_zlo) * plane + col] : -1;
            if (hit >= 0) {
                const BatchSource e = g.src[hit];
                drive_node<7>(e.kind, e.a0, e.a1, e.omega, g.src_t, v);
            }
        }
    }
}

// LDS floats per S slot: the tile plus its one-node ring (and a sink slot).
// With a run-time tile of at most NT columns the ring-padded tile and every
// neighbour read of an idle lane (lane index up to NT - 1) stay below
// 4 NT + 8.
template <int TX, int NT, bool RT>
constexpr int lds_s() {
    return RT ? 4 * NT + 8 : (NT / TX + 2) * (TX + 2) + 1;
}

__device__ void probe_block(const GeomDev& g, const ProbeArgs& pr, const float* __restrict__ fin) {
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

// One tile of one geometry: columns [x0, x0 + TX) x [y0, y0 + TY), planes
// [z0, z0 + lz).  fin/fout point at the geometry's own population block.
// RT: the tile is g.rtx x g.rty columns instead (at most NT of them, with
// 2 (rtx + rty) <= NT ring loaders and rtx + 2 <= NT row loaders, checked by
// the host); TX = NT then only sizes the LDS arrays.  SRC: driven nodes
// (g.src) are imposed on every population set as it is loaded (own column,
// ring), before any use, as if imposed in memory before the step.  NTS:
// population stores non-temporal; NTL: the own column's loads too (its
// planes are read once per pass; the ring's are read again by neighbours).
// PERY: axis 1 is periodic (its wall rules compiled out).
template <int TX, int NT, bool ROW, bool RT = false, bool NTS = false, bool SRC = false, bool NTL = false,
          bool PERY = false>
__device__ __forceinline__ void march_tile(const TileGeom& g, int tile, const float* __restrict__ fin,
                                           float* __restrict__ fout, float (&sS)[2][lds_s<TX, NT, RT>()],
                                           float4 (&sElo)[3][TX + 3], float4 (&sEhi)[3][TX + 3]) {
    const int TXr = RT ? g.rtx : TX;
    const int TY = RT ? g.rty : NT / TX;
    const int W = TXr + 2;
    const int kSinkS = (TY + 2) * W;  // LDS slot written by disabled lanes
    const int n0 = g.n0, n1 = g.n1, n2 = g.n2;
    const uint32_t N = g.N;
    const uint32_t plane = (uint32_t)n0 * (uint32_t)n1;
    const int lx = (int)(threadIdx.x % (unsigned)TXr), ly = (int)(threadIdx.x / (unsigned)TXr);
    const float c2 = g.c2, two_w0 = g.two_w0, damp = g.damp;
    const float4* __restrict__ tab4 = g.tab4;
    {
        const int tx = tile % g.ntx;
        const int r1 = tile / g.ntx;
        const int ty = r1 % g.nty;
        const int chunk = r1 / g.nty;
        const int x0 = tx * TXr, y0 = ty * TY;
        const int z0 = chunk * g.lz;
        if (z0 >= n2 || ty >= g.nty) return;  // tile outside the grid (uniform per block)
        const int z1 = min(z0 + g.lz, n2);
        const int wdt = min(TXr, n0 - x0);
        const int hgt = min(TY, n1 - y0);
        const int x = x0 + lx, y = y0 + ly;
        const bool active = lx < wdt && ly < hgt;
        const uint32_t col = (uint32_t)x + (uint32_t)n0 * (uint32_t)y;
        // the tile holds whole walled axis-0 rows: the axis-0 populations
        // reach their destinations by a lane shift, so each lane stores its
        // own node's (aligned stores instead of stores shifted by one float);
        // ROW = false compiles the shift out (grids wider than a tile)
        const bool row_tile = ROW && x0 == 0 && wdt == n0 && g.bc_lo[0] != LBW_BC_PERIODIC;

        // a wall code matters only where the link is missing, and there it
        // is that end's code: the wall rules take the ends' codes (uniform,
        // tested on the scalar unit), so link_coord's code is not kept
        int wall_unused = 0;
        const int jx_p = link_coord(x, +1, n0, g.bc_lo[0], g.bc_hi[0], &wall_unused);
        const int jx_m = link_coord(x, -1, n0, g.bc_lo[0], g.bc_hi[0], &wall_unused);
        const int jy_p = link_coord(y, +1, n1, g.bc_lo[1], g.bc_hi[1], &wall_unused);
        const int jy_m = link_coord(y, -1, n1, g.bc_lo[1], g.bc_hi[1], &wall_unused);
        const int bcx_lo = g.bc_lo[0], bcx_hi = g.bc_hi[0], bcy_lo = g.bc_lo[1], bcy_hi = g.bc_hi[1];
        // byte offsets to the axis-1 neighbours' columns (used where the link exists)
        const uint32_t dyp4 = (uint32_t)((jy_p - y) * n0) * 4u, dym4 = (uint32_t)((jy_m - y) * n0) * 4u;

        // ring node of this thread: LDS position and wrapped column, or -1
        int ring_lds = -1;
        uint32_t ring_col = 0;
        {
            const int r = threadIdx.x;
            int rx = 0, ry = 0, sx = 0, sy = 0;
            bool have = false;
            if (r < wdt) {
                rx = x0 + r; ry = y0 - 1; sx = r + 1; sy = 0; have = true;
            } else if (r >= TXr && r < TXr + wdt) {
                rx = x0 + (r - TXr); ry = y0 + hgt; sx = r - TXr + 1; sy = hgt + 1; have = true;
            } else if (r >= 2 * TXr && r < 2 * TXr + hgt) {
                rx = x0 - 1; ry = y0 + (r - 2 * TXr); sx = 0; sy = r - 2 * TXr + 1; have = true;
            } else if (r >= 2 * TXr + TY && r < 2 * TXr + TY + hgt) {
                rx = x0 + wdt; ry = y0 + (r - 2 * TXr - TY); sx = wdt + 1; sy = r - 2 * TXr - TY + 1; have = true;
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

        const uint32_t N4 = N * 4u, plane4 = plane * 4u, col4 = col * 4u, ring4 = ring_col * 4u;
        const __amdgpu_buffer_rsrc_t rin = make_rsrc(fin, 7u * N4);
        const __amdgpu_buffer_rsrc_t rout = make_rsrc(fout, 7u * N4);
        const __amdgpu_buffer_rsrc_t rtab = make_rsrc(tab4, (uint32_t)n0 * (uint32_t)n2 * 32u);
        const bool ring_on = ring_lds >= 0, erow_on = erow_x >= 0;

        // ---- prologue: planes z0-1 (S only), z0 (populations, S, ring S,
        // coefficient rows z0 and z0+1); pending into the loop: own column
        // and ring of plane z0+1 ----
        float fc[7], fnx[7], tmp[7];
        float Sm = 0.f, Sc = 0.f, Sp = 0.f;
        float2 em = make_float2(0.f, 0.f);  // (c^2 Mhat02, c^2 Mhat22) at z-1
        {
            const bool m_on = active && zm0 >= 0;
            bload7(rin, N4, m_on, col4 + (uint32_t)zm0 * plane4, tmp);
            const float4 e = bld4(rtab, m_on ? (uint32_t)(x + n0 * zm0) * 32u : kOff);
            bload7p<NTL>(rin, N4, active, col4 + (uint32_t)z0 * plane4, fc);
            const bool e0_on = erow_on, e1_on = erow_on && zp0 >= 0;
            const float4 a0 = bld4(rtab, e0_on ? (uint32_t)(erow_x + n0 * z0) * 32u : kOff);
            const float4 b0 = bld4(rtab, e0_on ? (uint32_t)(erow_x + n0 * z0) * 32u + 16u : kOff);
            const float4 a1 = bld4(rtab, e1_on ? (uint32_t)(erow_x + n0 * zp0) * 32u : kOff);
            const float4 b1 = bld4(rtab, e1_on ? (uint32_t)(erow_x + n0 * zp0) * 32u + 16u : kOff);
            float rz[7];
            bload7(rin, N4, ring_on, ring4 + (uint32_t)z0 * plane4, rz);
            drive_loaded<SRC>(g, zm0, m_on, col, tmp);
            drive_loaded<SRC>(g, z0, active, col, fc);
            drive_loaded<SRC>(g, z0, ring_on, ring_col, rz);
            Sm = sum7(tmp);
            em = make_float2(e.y, e.z);
            Sc = sum7(fc);
            if (e0_on) {
                sElo[0][threadIdx.x] = a0;
                sEhi[0][threadIdx.x] = b0;
            }
            if (e1_on) {
                sElo[1][threadIdx.x] = a1;
                sEhi[1][threadIdx.x] = b1;
            }
            if (ring_on) sS[0][ring_lds] = sum7(rz);
            if (active) sS[0][my_lds] = Sc;
        }
        float rA[7], rB[7], rC[7];  // ring populations: plane z+1 (loaded one step ago), plane z+2 (loading)
        float4 eA[2], eB[2], eC[2];  // coefficient rows: plane z+2 (loaded one step ago), plane z+3 (loading)
        bload7p<NTL>(rin, N4, active && zp0 >= 0, col4 + (uint32_t)zp0 * plane4, fnx);
        bload7(rin, N4, ring_on && z0 + 1 < z1, ring4 + (uint32_t)zp0 * plane4, rA);
        {
            int w = 0;
            const int zq0 = z0 + 1 < z1 && zp0 >= 0 ? link_coord(zp0, +1, n2, g.bc_lo[2], g.bc_hi[2], &w) : -1;
            const bool on = erow_on && zq0 >= 0;
            const uint32_t off = (uint32_t)(erow_x + n0 * zq0) * 32u;
            eA[0] = bld4(rtab, on ? off : kOff);
            eA[1] = bld4(rtab, on ? off + 16u : kOff);
        }

        // One plane.  fc: populations of plane z, fnx: of plane z+1 (loaded
        // one step ago), fnn: receives plane z+2; r1: ring of plane z+1
        // (loaded one step ago), r2: receives the ring of plane z+2.  The
        // caller rotates the arrays by argument order (no register copies);
        // the coefficient-row slot of plane z is es (z+1 in es+1, z+2 in
        // es+2, mod 3).
        auto plane_step = [&](auto es_c, float (&fc)[7], float (&fnx)[7], float (&fnn)[7], float (&r1)[7],
                              float (&r2)[7], float4 (&e1)[2], float4 (&e2)[2], int z) {
            constexpr int es = decltype(es_c)::value;
            constexpr int es1 = (es + 1) % 3;
            constexpr int es2 = (es + 2) % 3;
            const int sb = (z - z0) & 1;
            int wz_p = 0, wz_m = 0;
            const int jz_p = link_coord(z, +1, n2, g.bc_lo[2], g.bc_hi[2], &wz_p);
            const int jz_m = link_coord(z, -1, n2, g.bc_lo[2], g.bc_hi[2], &wz_m);
            const bool more = z + 1 < z1;
            const bool more2 = z + 2 < z1;
            int wq = 0;
            const int zq = more ? link_coord(jz_p, +1, n2, g.bc_lo[2], g.bc_hi[2], &wq) : -1;  // plane z+2

            // loads consumed one step later: coefficient row of plane z+3,
            // own column and ring of plane z+2
            const bool e_on = erow_on && zq >= 0;  // row of plane z+2 (in e1) is staged
            const int z3 = more2 && zq >= 0 ? link_coord(zq, +1, n2, g.bc_lo[2], g.bc_hi[2], &wq) : -1;
            const bool e3_on = erow_on && z3 >= 0;
            const uint32_t eoff = (uint32_t)(erow_x + n0 * z3) * 32u;
            e2[0] = bld4(rtab, e3_on ? eoff : kOff);
            e2[1] = bld4(rtab, e3_on ? eoff + 16u : kOff);
            bload7p<NTL>(rin, N4, active && zq >= 0, col4 + (uint32_t)zq * plane4, fnn);
            bload7(rin, N4, ring_on && more2, ring4 + (uint32_t)zq * plane4, r2);
            // plane z+1 (own column; ring below) as loaded one step ago:
            // driven nodes imposed before their first use (fnx becomes fc)
            drive_loaded<SRC>(g, jz_p, active && jz_p >= 0, col, fnx);
            Sp = sum7(fnx);  // S of plane z+1 (zeros when there is none: then unused)
            __syncthreads();

            const float* L = sS[sb];
            const float S = Sc;
            const float4 e_lo = sElo[es][lx + 1];  // 00, 02, 22, 11
            const float4 e_hi = sEhi[es][lx + 1];  // g0/2, g2/2, 0, 0
            // axis-0/1 neighbours: read unconditionally (every index is inside
            // the LDS arrays); collide() selects the wall rule
            Links k;
            k.jx_p = jx_p;
            k.jx_m = jx_m;
            k.jy_p = PERY ? 0 : jy_p;  // (collide() uses only their presence)
            k.jy_m = PERY ? 0 : jy_m;
            k.jz_p = jz_p;
            k.jz_m = jz_m;
            k.wx_p = bcx_hi;
            k.wx_m = bcx_lo;
            k.wy_p = bcy_hi;
            k.wy_m = bcy_lo;
            k.wz_p = wz_p;
            k.wz_m = wz_m;
            float fs[7];
            collide(fc, S, e_lo, e_hi, sElo[es][lx + 2], sElo[es][lx], sElo[es1][lx + 1], em, L[my_lds + 1],
                    L[my_lds - 1], L[my_lds + W], L[my_lds - W], Sp, Sm, k, c2, two_w0, fs);
            const float cM02 = e_lo.y, cM22 = e_lo.z;

            // push with the wall rules: destination offset and value by select
            const uint32_t nb = col4 + (uint32_t)z * plane4;
            const uint32_t o0 = nb;
            const uint32_t o1 = row_tile ? 1u * N4 + nb
                                : jx_p >= 0 ? 1u * N4 + nb + (uint32_t)(jx_p - x) * 4u : 2u * N4 + nb;
            const uint32_t o2 = row_tile ? 2u * N4 + nb
                                : jx_m >= 0 ? 2u * N4 + nb + (uint32_t)(jx_m - x) * 4u : 1u * N4 + nb;
            const uint32_t o3 = k.jy_p >= 0 ? 3u * N4 + nb + dyp4 : 4u * N4 + nb;
            const uint32_t o4 = k.jy_m >= 0 ? 4u * N4 + nb + dym4 : 3u * N4 + nb;
            const uint32_t o5 = jz_p >= 0 ? 5u * N4 + col4 + (uint32_t)jz_p * plane4 : 6u * N4 + nb;
            const uint32_t o6 = jz_m >= 0 ? 6u * N4 + col4 + (uint32_t)jz_m * plane4 : 5u * N4 + nb;
            float v1 = jx_p >= 0 ? fs[1] : bounce(bcx_hi, damp, fs[1], fs[2]);
            float v2 = jx_m >= 0 ? fs[2] : bounce(bcx_lo, damp, fs[2], fs[1]);
            if constexpr (ROW) {
                // whole-row tile: population 1 of this node comes from the
                // lane on the left (or the wall at x = 0), population 2 from
                // the lane on the right (or the wall at x = n0 - 1)
                float from_left, from_right;
                if constexpr (TX > 64) {
                    // a row may span several waves (always so for run-time
                    // tiles, where TX = NT): exchange through LDS (the reads
                    // of the previous plane ended before this plane's first
                    // barrier, so the slots are free)
                    __shared__ float sX[2][NT];
                    sX[0][threadIdx.x] = fs[1];
                    sX[1][threadIdx.x] = fs[2];
                    __syncthreads();
                    from_left = sX[0][lx > 0 ? threadIdx.x - 1 : threadIdx.x];
                    // (a run-time tile may end inside a row: the last lane
                    // then has no right neighbour in the workgroup; its
                    // value is unused, the index is kept in range)
                    const unsigned xr = lx < TXr - 1 ? threadIdx.x + 1 : threadIdx.x;
                    from_right = sX[1][RT ? min(xr, (unsigned)NT - 1) : xr];
                } else {
                    from_left = __shfl_up(fs[1], 1, TX);
                    from_right = __shfl_down(fs[2], 1, TX);
                }
                const float in1 = jx_m >= 0 ? from_left : v2;
                const float in2 = jx_p >= 0 ? from_right : v1;
                v1 = row_tile ? in1 : v1;
                v2 = row_tile ? in2 : v2;
            }
            const float v3 = k.jy_p >= 0 ? fs[3] : bounce(bcy_hi, damp, fs[3], fs[4]);
            const float v4 = k.jy_m >= 0 ? fs[4] : bounce(bcy_lo, damp, fs[4], fs[3]);
            const float v5 = jz_p >= 0 ? fs[5] : bounce(wz_p, damp, fs[5], fs[6]);
            const float v6 = jz_m >= 0 ? fs[6] : bounce(wz_m, damp, fs[6], fs[5]);
            bstp<NTS>(rout, active ? o0 : kOff, fs[0]);
            bstp<NTS>(rout, active ? o1 : kOff, v1);
            bstp<NTS>(rout, active ? o2 : kOff, v2);
            bstp<NTS>(rout, active ? o3 : kOff, v3);
            bstp<NTS>(rout, active ? o4 : kOff, v4);
            bstp<NTS>(rout, active ? o5 : kOff, v5);
            bstp<NTS>(rout, active ? o6 : kOff, v6);
            em = make_float2(cM02, cM22);

            if (more) {
                drive_loaded<SRC>(g, jz_p, ring_on, ring_col, r1);
                // disabled lanes write the sink slot past the end (never read)
                sS[sb ^ 1][ring_on ? ring_lds : kSinkS] = sum7(r1);
                sElo[es2][e_on ? (int)threadIdx.x : TXr + 2] = e1[0];
                sEhi[es2][e_on ? (int)threadIdx.x : TXr + 2] = e1[1];
                sS[sb ^ 1][active ? my_lds : kSinkS] = Sp;
                Sm = Sc;
                Sc = Sp;
            }
        };
        float fz[7];
        for (int z = z0;;) {
            if (z >= z1) break;
            plane_step(std::integral_constant<int, 0>{}, fc, fnx, fz, rA, rB, eA, eB, z);
            if (++z >= z1) break;
            plane_step(std::integral_constant<int, 1>{}, fnx, fz, fc, rB, rC, eB, eC, z);
            if (++z >= z1) break;
            plane_step(std::integral_constant<int, 2>{}, fz, fc, fnx, rC, rA, eC, eA, z);
            ++z;
        }
        __syncthreads();  // LDS reuse by the next tile
    }
}

template <int TX, int NT, bool ROW, bool NTS, bool PERY>
__global__ __launch_bounds__(NT) void step_march_kernel(GeomDev g, ProbeArgs pr, MarchPlan plan,
                                                              const float* __restrict__ fin,
                                                              float* __restrict__ fout) {
    __shared__ float sS[2][lds_s<TX, NT, false>()];
    __shared__ float4 sElo[3][TX + 3];
    __shared__ float4 sEhi[3][TX + 3];
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
    tg.src = nullptr;
    tg.src_map = nullptr;
    tg.src_count = tg.src_zlo = tg.src_zhi = 0;
    tg.src_t = 0;
    const int xcd = blockIdx.x % kXcds;
    const int per_xcd_blocks = gridDim.x / kXcds;
    const int t_begin = (int)(plan.tiles * xcd / kXcds);
    const int t_end = (int)(plan.tiles * (xcd + 1) / kXcds);
    for (int tile = t_begin + (int)blockIdx.x / kXcds; tile < t_end; tile += per_xcd_blocks)
        march_tile<TX, NT, ROW, false, NTS, false, NTS, PERY>(tg, tile, fin, fout, sS, sElo, sEhi);
}

// Batch of geometries advanced by one launch: tiles of all geometries form
// one list (geometry h owns tiles [tile_begin, tile_begin + tiles)), split
// into one contiguous range per XCD.  Block b first records the probes of
// geometries b, b + gridDim.x, ... (one step counter per geometry).
// SECTION: every tile holds whole axis-0 rows of its geometry (run-time
// tile n0 x rty, rty rows chosen per geometry by the host; the whole
// cross-section when it fits), for geometries whose rows a TX-wide tile
// would split or leave mostly idle; TX = NT then only sizes the LDS arrays.
template <int TX, int NT, bool SECTION, bool NTS, bool PERY>
__global__ __launch_bounds__(NT) void step_batch_kernel(const BatchItem* __restrict__ items,
                                                         const int32_t* __restrict__ tile_item, int n_items,
                                                         int64_t tiles_total, BatchProbeArgs bp,
                                                         const float* __restrict__ fin, float* __restrict__ fout) {
    __shared__ float sS[2][lds_s<TX, NT, SECTION>()];
    __shared__ float4 sElo[3][TX + 3];
    __shared__ float4 sEhi[3][TX + 3];
    // this launch's time per geometry: bank `parity`, which no block of it
    // writes (the probe blocks below write the other bank)
    const int64_t* __restrict__ t_now = bp.tcount + (size_t)bp.parity * n_items;
    int64_t* t_next = bp.tcount + (size_t)(bp.parity ^ 1) * n_items;
    for (int h = blockIdx.x; h < n_items; h += gridDim.x) {
        const BatchItem& it = items[h];
        const int64_t t = t_now[h];
        if (t >= 0 && t < bp.t_max) {
            const float* f = fin + it.f_off;
            TileGeom pg;
            pg.n0 = it.n0;
            pg.n1 = it.n1;
            pg.src = bp.src;
            pg.src_map = bp.src_map + it.src_map;
            pg.src_count = bp.src ? it.src_count : 0;
            pg.src_zlo = it.src_zlo;
            pg.src_zhi = it.src_zhi;
            pg.src_t = t;
            for (int p = threadIdx.x; p < it.n_probes; p += blockDim.x) {
                const uint32_t node = (uint32_t)bp.nodes[it.probe_off + p];
                float v[7];
                for (int l = 0; l < 7; ++l) v[l] = f[l * it.N + node];
                const uint32_t i0 = node % (uint32_t)it.n0;
                const uint32_t i2 = node / ((uint32_t)it.n0 * (uint32_t)it.n1);
                // a driven probe node reads its driven value (per lane: not
                // every lane of the block holds a probe)
                if (pg.src_count > 0 && (int)i2 >= it.src_zlo && (int)i2 <= it.src_zhi)
                    drive_loaded<true>(pg, (int)i2, true, node - i2 * ((uint32_t)it.n0 * (uint32_t)it.n1), v);
                double s = 0.0;
                for (int l = 0; l < 7; ++l) s += (double)v[l];
                bp.trace[t * bp.stride + it.probe_off + p] = s / bp.sqrtg[it.sg_off + i0 + (uint32_t)it.n0 * i2];
            }
        }
        if (threadIdx.x == 0) t_next[h] = t + 1;
    }
    const int xcd = blockIdx.x % kXcds;
    const int per_xcd_blocks = gridDim.x / kXcds;
    const int64_t t_begin = tiles_total * xcd / kXcds;
    const int64_t t_end = tiles_total * (xcd + 1) / kXcds;
    for (int64_t tile = t_begin + (int)blockIdx.x / kXcds; tile < t_end; tile += per_xcd_blocks) {
        const int h = tile_item[tile];  // geometry owning this tile
        if (h < 0 || h >= n_items) continue;  // inconsistent table: skip
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
        tg.rtx = it.n0;
        tg.rty = it.rty;
        tg.src = bp.src;
        tg.src_map = bp.src_map + it.src_map;
        tg.src_count = bp.src ? it.src_count : 0;  // (a list being replaced leaves no entries)
        tg.src_zlo = it.src_zlo;
        tg.src_zhi = it.src_zhi;
        tg.src_t = t_now[h];
        march_tile<TX, NT, true, SECTION, NTS, true, false, PERY>(tg, (int)(tile - it.tile_begin), fin + it.f_off,
                                                     fout + it.f_off, sS, sElo, sEhi);
    }
}

}  // namespace

bool march_nts_default(const GeomDev& g) {
    // two population buffers of 4 Q N bytes against the 256 MiB Infinity Cache
    return 2.0 * 4.0 * (2 * g.dim + 1) * (double)g.N > 256.0 * 1024.0 * 1024.0;
}

int march_tx_for(int n0) { return n0 <= 16 ? 16 : (n0 <= 32 ? 32 : 64); }

bool march_shape_ok(int tx, int ty) {
    // 96- and 128-wide rows only with 4 or 8 of them (384 to 1024 threads):
    // the ring needs 2 (tx + ty) loaders
    if (tx == 96 || tx == 128) return ty == 4 || ty == 8;
    return (tx == 16 || tx == 32 || tx == 64) && (tx * ty == 256 || tx * ty == 512);
}

namespace {
template <int TX, int NT>
int blocks_per_cu_of() {
    int nb = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_march_kernel<TX, NT, false, false, false>, NT, 0);
    return e == hipSuccess && nb > 0 ? nb : 1;
}
template <int TX, int NT, bool ROW, bool NTS>
void launch_pery(bool pery, dim3 grid, dim3 block, hipStream_t st, const GeomDev& g, const ProbeArgs& pr,
                 const MarchPlan& plan, const float* fin, float* fout) {
    if (pery)
        hipLaunchKernelGGL((step_march_kernel<TX, NT, ROW, NTS, true>), grid, block, 0, st, g, pr, plan, fin, fout);
    else
        hipLaunchKernelGGL((step_march_kernel<TX, NT, ROW, NTS, false>), grid, block, 0, st, g, pr, plan, fin, fout);
}
template <int TX, int NT>
void launch_of(const GeomDev& g, const ProbeArgs& pr, const MarchPlan& plan, const float* fin, float* fout,
               hipStream_t st) {
    // whole walled rows fit one tile: the variant with the axis-0 lane shift;
    // non-temporal stores as the plan says
    const bool row = g.n0 <= TX && g.bc_lo[0] != LBW_BC_PERIODIC;
    const bool pery = g.bc_lo[1] == LBW_BC_PERIODIC;
    const dim3 grid(plan.blocks), block(NT);
    if (row && plan.nts)
        launch_pery<TX, NT, true, true>(pery, grid, block, st, g, pr, plan, fin, fout);
    else if (row)
        launch_pery<TX, NT, true, false>(pery, grid, block, st, g, pr, plan, fin, fout);
    else if (plan.nts)
        launch_pery<TX, NT, false, true>(pery, grid, block, st, g, pr, plan, fin, fout);
    else
        launch_pery<TX, NT, false, false>(pery, grid, block, st, g, pr, plan, fin, fout);
}
}  // namespace

int march_blocks_per_cu(int tx, int ty) {
    const int nt = tx * ty;
    if (tx == 128) return nt == 1024 ? blocks_per_cu_of<128, 1024>() : blocks_per_cu_of<128, 512>();
    if (tx == 96) return nt == 768 ? blocks_per_cu_of<96, 768>() : blocks_per_cu_of<96, 384>();
    if (nt == 512) return tx == 16 ? blocks_per_cu_of<16, 512>() : tx == 32 ? blocks_per_cu_of<32, 512>()
                                                                            : blocks_per_cu_of<64, 512>();
    return tx == 16 ? blocks_per_cu_of<16, 256>() : tx == 32 ? blocks_per_cu_of<32, 256>() : blocks_per_cu_of<64, 256>();
}

hipError_t launch_step_march(const GeomDev& g, const ProbeArgs& pr, const MarchPlan& plan, const float* fin,
                             float* fout, hipStream_t st) {
    if (!march_shape_ok(plan.tx, plan.ty)) return hipErrorInvalidValue;
    const int nt = plan.tx * plan.ty;
    if (plan.tx == 128 && nt == 1024) {
        launch_of<128, 1024>(g, pr, plan, fin, fout, st);
    } else if (plan.tx == 128) {
        launch_of<128, 512>(g, pr, plan, fin, fout, st);
    } else if (plan.tx == 96 && nt == 768) {
        launch_of<96, 768>(g, pr, plan, fin, fout, st);
    } else if (plan.tx == 96) {
        launch_of<96, 384>(g, pr, plan, fin, fout, st);
    } else if (nt == 512) {
        if (plan.tx == 16) launch_of<16, 512>(g, pr, plan, fin, fout, st);
        else if (plan.tx == 32) launch_of<32, 512>(g, pr, plan, fin, fout, st);
        else launch_of<64, 512>(g, pr, plan, fin, fout, st);
    } else {
        if (plan.tx == 16) launch_of<16, 256>(g, pr, plan, fin, fout, st);
        else if (plan.tx == 32) launch_of<32, 256>(g, pr, plan, fin, fout, st);
        else launch_of<64, 256>(g, pr, plan, fin, fout, st);
    }
    return hipGetLastError();
}

int batch_blocks_per_cu(int tx) {
    int nb = 0;
    hipError_t e =
        tx == 16   ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_batch_kernel<16, kBatchThreads, false, false, false>,
                                                                  kBatchThreads, 0)
        : tx == 32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_batch_kernel<32, kBatchThreads, false, false, false>,
                                                                  kBatchThreads, 0)
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_batch_kernel<64, kBatchThreads, false, false, false>,
                                                                  kBatchThreads, 0);
    return e == hipSuccess && nb > 0 ? nb : 1;
}

int batch_row_tile(int n0, int n1, int nt) {
    if (n0 < 1 || n1 < 1 || n0 + 2 > nt) return 0;
    int r = min(n1, min(nt / n0, nt / 2 - n0));
    return r >= 1 ? r : 0;
}

int batch_section_blocks_per_cu(int nt) {
    int nb = 0;
    hipError_t e =
        nt == 128   ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_batch_kernel<128, 128, true, false, false>, 128, 0)
        : nt == 256 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_batch_kernel<256, 256, true, false, false>, 256, 0)
                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_batch_kernel<512, 512, true, false, false>, 512, 0);
    return e == hipSuccess && nb > 0 ? nb : 1;
}

namespace {
template <bool NTS, bool PERY>
void launch_batch_of(const BatchItem* items, const int32_t* tile_item, int n_items, int64_t tiles_total, int tx,
                     int section_nt, int blocks, const BatchProbeArgs& bp, const float* fin, float* fout,
                     hipStream_t st) {
    const dim3 grid(blocks);
    if (section_nt == 128)
        hipLaunchKernelGGL((step_batch_kernel<128, 128, true, NTS, PERY>), grid, dim3(128), 0, st, items, tile_item, n_items,
                           tiles_total, bp, fin, fout);
    else if (section_nt == 256)
        hipLaunchKernelGGL((step_batch_kernel<256, 256, true, NTS, PERY>), grid, dim3(256), 0, st, items, tile_item, n_items,
                           tiles_total, bp, fin, fout);
    else if (section_nt == 512)
        hipLaunchKernelGGL((step_batch_kernel<512, 512, true, NTS, PERY>), grid, dim3(512), 0, st, items, tile_item, n_items,
                           tiles_total, bp, fin, fout);
    else if (tx == 16)
        hipLaunchKernelGGL((step_batch_kernel<16, kBatchThreads, false, NTS, PERY>), grid, dim3(kBatchThreads), 0, st, items,
                           tile_item, n_items, tiles_total, bp, fin, fout);
    else if (tx == 32)
        hipLaunchKernelGGL((step_batch_kernel<32, kBatchThreads, false, NTS, PERY>), grid, dim3(kBatchThreads), 0, st, items,
                           tile_item, n_items, tiles_total, bp, fin, fout);
    else
        hipLaunchKernelGGL((step_batch_kernel<64, kBatchThreads, false, NTS, PERY>), grid, dim3(kBatchThreads), 0, st, items,
                           tile_item, n_items, tiles_total, bp, fin, fout);
}
}  // namespace

hipError_t launch_step_batch(const BatchItem* items, const int32_t* tile_item, int n_items, int64_t tiles_total,
                             int tx, int section_nt, int blocks, bool nts, bool pery, const BatchProbeArgs& bp,
                             const float* fin, float* fout, hipStream_t st) {
    if (nts && pery)
        launch_batch_of<true, true>(items, tile_item, n_items, tiles_total, tx, section_nt, blocks, bp, fin, fout, st);
    else if (nts)
        launch_batch_of<true, false>(items, tile_item, n_items, tiles_total, tx, section_nt, blocks, bp, fin, fout, st);
    else if (pery)
        launch_batch_of<false, true>(items, tile_item, n_items, tiles_total, tx, section_nt, blocks, bp, fin, fout, st);
    else
        launch_batch_of<false, false>(items, tile_item, n_items, tiles_total, tx, section_nt, blocks, bp, fin, fout, st);
    return hipGetLastError();
}

MarchPlan make_march_plan(const GeomDev& g, int tx, int ty, int lz, int blocks) {
    MarchPlan p{};
    p.nts = march_nts_default(g);
    p.tx = tx;
    p.ty = ty;
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
