// Step for geometries given by their metric (Sec. III: the geometry enters
// the scheme only through sqrt(g), the inverse metric and the contracted
// Christoffel symbols, so any coordinate system runs by supplying them per
// node).  Same arithmetic as the per-node description in step.hip (BGK
// tau = 1/2, corrected equilibrium, Christoffel and metric-gradient forcing,
// push streaming with the wall rules), with all six metric components, each
// varying along every axis.
//
// Coefficients are FP32 planes of N values: c^2 Mhat 00, 11, 22, 01, 02, 12
// and c^2 Gamh / 2 per axis.  For axis d the metric-gradient term is
// (1/4) sum_e [A^{de}(x + e_e) - A^{de}(x - e_e)], A^{de} = c^2 Mhat^{de} S:
// the axis-0 neighbours contribute A^{00}, A^{10}, A^{20}, the axis-1
// neighbours A^{01}, A^{11}, A^{21}, the axis-2 neighbours A^{02}, A^{12},
// A^{22}; beyond a wall the node's own A is mirrored (odd for fixed walls).
//
// Data movement (as the z-marching kernel of the built-in geometries): a
// workgroup of NT = 256 or 512 threads owns a TX x TY tile of (axis 0, axis 1) columns
// and walks a chunk of planes along axis 2.  A thread keeps its column's
// populations, coefficients and the axis-2 products A^{d2} of planes z-1, z
// and z+1 in registers (plane z+2 is loaded while plane z is computed); the
// five products the axis-0 and axis-1 neighbours need (A^{00}, A^{11},
// A^{01}, A^{02}, A^{12}) are staged in LDS for the tile and a one-node ring
// (two plane slots, one barrier per plane), the ring nodes' populations and
// coefficients loaded one plane ahead by the first 2 TX + 2 TY threads.  Workgroup 0 records
// the probes of time t before any population is written and advances the
// step counter.
#include "lbw_internal.h"

namespace lbw {
namespace {

constexpr int kXcd = 8;   // tiles are dealt to XCDs in contiguous ranges

// Buffer loads with 32-bit byte offsets: an offset of kOff lies beyond every
// buffer (the library keeps 4 Q N and 36 N below 2^31), so a disabled lane
// reads 0 without a branch around the load.
constexpr uint32_t kOff = 0x80000000u;
__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ inline float bld(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}

__device__ inline float mirror(int wall, float own) { return wall == LBW_BC_FIXED ? -own : own; }

__device__ inline float bounce_rule(int wall, float damp, float out_l, float own_opposite) {
    return wall == LBW_BC_BOUNCEBACK ? damp * out_l : (wall == LBW_BC_FREE ? own_opposite : -out_l);
}

struct GenPlan {
    int ntx, nty, nch, lz;
};

// one node's populations, coefficients, S and the six products c^2 Mhat^m S
struct Node {
    float f[7];
    float t[9];
    float S;
    float a[6];
};

// node at byte offset nb (4 n), or all zeros when off
__device__ inline void load_node(__amdgpu_buffer_rsrc_t rf, __amdgpu_buffer_rsrc_t rt, uint32_t N4, bool on,
                                 uint32_t nb, Node& v) {
    const uint32_t base = on ? nb : kOff;
    float s = 0.f;
#pragma unroll
    for (int l = 0; l < 7; ++l) {
        v.f[l] = bld(rf, base + (uint32_t)l * N4);
        s += v.f[l];
    }
#pragma unroll
    for (int m = 0; m < 9; ++m) v.t[m] = bld(rt, base + (uint32_t)m * N4);
    v.S = s;
#pragma unroll
    for (int m = 0; m < 6; ++m) v.a[m] = v.t[m] * s;
}

template <int TX, int NT>
__global__ __launch_bounds__(NT) void general_march_kernel(GeomDev g, ProbeArgs pr, GenPlan plan,
                                                            const float* __restrict__ fin,
                                                            float* __restrict__ fout) {
    constexpr int TY = NT / TX;
    constexpr int W = TX + 2;
    constexpr int SLOTS = (TY + 2) * W;
    // LDS products per slot: 0 A^{00}, 1 A^{11}, 2 A^{01}, 3 A^{02}, 4 A^{12}
    __shared__ float sA[2][5][SLOTS + 1];  // + a sink slot

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

    const int n0 = g.n0, n1 = g.n1, n2 = g.n2;
    const int64_t N = g.N, plane = (int64_t)n0 * n1;
    const float* __restrict__ T = g.tab;
    // XCD-contiguous tiles: block b runs on XCD b mod 8 and takes tile
    // (b mod 8) per + b / 8 of that XCD's range, so tiles sharing ring nodes
    // and chunk-boundary planes share an L2; blocks past the last tile exit
    // (block 0, which records the probes, always has tile 0)
    const int per = (int)(((int64_t)plan.ntx * plan.nty * plan.nch + kXcd - 1) / kXcd);
    const int b = (int)(blockIdx.x % kXcd) * per + (int)(blockIdx.x / kXcd);
    if (b >= plan.ntx * plan.nty * plan.nch) return;
    const int tx = b % plan.ntx, ty = (b / plan.ntx) % plan.nty, ch = b / (plan.ntx * plan.nty);
    const int x0 = tx * TX, y0 = ty * TY, z0 = ch * plan.lz;
    const int z1 = min(z0 + plan.lz, n2);
    const int wdt = min(TX, n0 - x0), hgt = min(TY, n1 - y0);
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int x = x0 + lx, y = y0 + ly;
    const bool active = lx < wdt && ly < hgt;
    const int64_t col = (int64_t)x + (int64_t)n0 * y;
    const int my = (ly + 1) * W + lx + 1;
    const uint32_t N4 = (uint32_t)N * 4u, plane4 = (uint32_t)plane * 4u, col4 = (uint32_t)col * 4u;
    const __amdgpu_buffer_rsrc_t rf = rsrc(fin, 7u * N4);
    const __amdgpu_buffer_rsrc_t rt = rsrc(T, 9u * N4);

    int wx_p = 0, wx_m = 0, wy_p = 0, wy_m = 0;
    const int jx_p = link_coord(x, +1, n0, g.bc_lo[0], g.bc_hi[0], &wx_p);
    const int jx_m = link_coord(x, -1, n0, g.bc_lo[0], g.bc_hi[0], &wx_m);
    const int jy_p = link_coord(y, +1, n1, g.bc_lo[1], g.bc_hi[1], &wy_p);
    const int jy_m = link_coord(y, -1, n1, g.bc_lo[1], g.bc_hi[1], &wy_m);

    // ring node of this thread (slot and wrapped column), if any: rows
    // y0 - 1 and y0 + hgt over the tile's columns, columns x0 - 1 and
    // x0 + wdt over its rows, each placed next to the tile's last active
    // column/row so that a node's neighbour slot is always slot +- 1 / +- W
    int ring_slot = -1;
    int64_t ring_col = 0;
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
                ring_slot = sy * W + sx;
                ring_col = (int64_t)gx + (int64_t)n0 * gy;
            }
        }
    }

    // planes z0 - 1 (products only), z0 and z0 + 1
    Node cur, nxt;
    float azm[3] = {0.f, 0.f, 0.f};  // A^{02}, A^{12}, A^{22} at z - 1
    {
        int w = 0;
        const int zm0 = link_coord(z0, -1, n2, g.bc_lo[2], g.bc_hi[2], &w);
        Node v;
        load_node(rf, rt, N4, active && zm0 >= 0, col4 + (uint32_t)zm0 * plane4, v);
        azm[0] = v.a[4];
        azm[1] = v.a[5];
        azm[2] = v.a[2];
        load_node(rf, rt, N4, active, col4 + (uint32_t)z0 * plane4, cur);
        const int zp0 = link_coord(z0, +1, n2, g.bc_lo[2], g.bc_hi[2], &w);
        load_node(rf, rt, N4, active && zp0 >= 0, col4 + (uint32_t)zp0 * plane4, nxt);
    }
    // ring node of plane z: populations and the five coefficient planes the
    // neighbours' products use (loaded one plane ahead)
    float rfv[7], rtv[5];
    const uint32_t ring4 = (uint32_t)ring_col * 4u;
    auto load_ring = [&](int zz) {
        const uint32_t base = ring_slot >= 0 ? ring4 + (uint32_t)zz * plane4 : kOff;
#pragma unroll
        for (int l = 0; l < 7; ++l) rfv[l] = bld(rf, base + (uint32_t)l * N4);
        rtv[0] = bld(rt, base + 0u * N4);
        rtv[1] = bld(rt, base + 1u * N4);
        rtv[2] = bld(rt, base + 3u * N4);
        rtv[3] = bld(rt, base + 4u * N4);
        rtv[4] = bld(rt, base + 5u * N4);
    };
    load_ring(z0);
    Node nn;  // plane z + 2

    int buf = 0;
    for (int z = z0; z < z1; ++z, buf ^= 1) {
        int wz_p = 0, wz_m = 0;
        const int jz_p = link_coord(z, +1, n2, g.bc_lo[2], g.bc_hi[2], &wz_p);
        const int jz_m = link_coord(z, -1, n2, g.bc_lo[2], g.bc_hi[2], &wz_m);
        // plane z + 2 of the own column, consumed one plane later
        {
            int w = 0;
            const int zq = z + 1 < z1 && jz_p >= 0 ? link_coord(jz_p, +1, n2, g.bc_lo[2], g.bc_hi[2], &w) : -1;
            load_node(rf, rt, N4, active && zq >= 0, col4 + (uint32_t)zq * plane4, nn);
        }
        // stage this plane's products for the axis-0/1 neighbours
        if (active) {
            sA[buf][0][my] = cur.a[0];
            sA[buf][1][my] = cur.a[1];
            sA[buf][2][my] = cur.a[3];
            sA[buf][3][my] = cur.a[4];
            sA[buf][4][my] = cur.a[5];
        }
        {
            float s = 0.f;
#pragma unroll
            for (int l = 0; l < 7; ++l) s += rfv[l];
            // lanes without a ring node write a sink slot past the tile
#pragma unroll
            for (int k = 0; k < 5; ++k) sA[buf][k][ring_slot >= 0 ? ring_slot : SLOTS] = rtv[k] * s;
            load_ring(z + 1 < z1 ? z + 1 : z);
        }
        __syncthreads();
        if (active) {
            const float* L0 = sA[buf][0];
            const float* L1 = sA[buf][1];
            const float* L2 = sA[buf][2];
            const float* L3 = sA[buf][3];
            const float* L4 = sA[buf][4];
            // axis 0 neighbours: A^{00}, A^{10} = A^{01}, A^{20} = A^{02}
            const float x00p = jx_p >= 0 ? L0[my + 1] : mirror(wx_p, cur.a[0]);
            const float x00m = jx_m >= 0 ? L0[my - 1] : mirror(wx_m, cur.a[0]);
            const float x10p = jx_p >= 0 ? L2[my + 1] : mirror(wx_p, cur.a[3]);
            const float x10m = jx_m >= 0 ? L2[my - 1] : mirror(wx_m, cur.a[3]);
            const float x20p = jx_p >= 0 ? L3[my + 1] : mirror(wx_p, cur.a[4]);
            const float x20m = jx_m >= 0 ? L3[my - 1] : mirror(wx_m, cur.a[4]);
            // axis 1 neighbours: A^{01}, A^{11}, A^{21} = A^{12}
            const float y01p = jy_p >= 0 ? L2[my + W] : mirror(wy_p, cur.a[3]);
            const float y01m = jy_m >= 0 ? L2[my - W] : mirror(wy_m, cur.a[3]);
            const float y11p = jy_p >= 0 ? L1[my + W] : mirror(wy_p, cur.a[1]);
            const float y11m = jy_m >= 0 ? L1[my - W] : mirror(wy_m, cur.a[1]);
            const float y21p = jy_p >= 0 ? L4[my + W] : mirror(wy_p, cur.a[5]);
            const float y21m = jy_m >= 0 ? L4[my - W] : mirror(wy_m, cur.a[5]);
            // axis 2 neighbours (registers): A^{02}, A^{12}, A^{22}
            const float z02p = jz_p >= 0 ? nxt.a[4] : mirror(wz_p, cur.a[4]);
            const float z02m = jz_m >= 0 ? azm[0] : mirror(wz_m, cur.a[4]);
            const float z12p = jz_p >= 0 ? nxt.a[5] : mirror(wz_p, cur.a[5]);
            const float z12m = jz_m >= 0 ? azm[1] : mirror(wz_m, cur.a[5]);
            const float z22p = jz_p >= 0 ? nxt.a[2] : mirror(wz_p, cur.a[2]);
            const float z22m = jz_m >= 0 ? azm[2] : mirror(wz_m, cur.a[2]);
            const float S = cur.S;
            const float K0 = (cur.f[1] - cur.f[2]) - cur.t[6] * S -
                             0.25f * (((x00p - x00m) + (y01p - y01m)) + (z02p - z02m));
            const float K1 = (cur.f[3] - cur.f[4]) - cur.t[7] * S -
                             0.25f * (((x10p - x10m) + (y11p - y11m)) + (z12p - z12m));
            const float K2 = (cur.f[5] - cur.f[6]) - cur.t[8] * S -
                             0.25f * (((x20p - x20m) + (y21p - y21m)) + (z22p - z22m));
            const float cs = g.c2 * S;
            const float fs0 = g.two_w0 * S - cur.f[0];
            const float fs1 = cs + K0 - cur.f[1], fs2 = cs - K0 - cur.f[2];
            const float fs3 = cs + K1 - cur.f[3], fs4 = cs - K1 - cur.f[4];
            const float fs5 = cs + K2 - cur.f[5], fs6 = cs - K2 - cur.f[6];
            const int64_t n = col + (int64_t)z * plane;
            fout[n] = fs0;
            if (jx_p >= 0) fout[1 * N + n + (jx_p - x)] = fs1;
            else fout[2 * N + n] = bounce_rule(wx_p, g.damp, fs1, fs2);
            if (jx_m >= 0) fout[2 * N + n + (jx_m - x)] = fs2;
            else fout[1 * N + n] = bounce_rule(wx_m, g.damp, fs2, fs1);
            if (jy_p >= 0) fout[3 * N + n + (int64_t)(jy_p - y) * n0] = fs3;
            else fout[4 * N + n] = bounce_rule(wy_p, g.damp, fs3, fs4);
            if (jy_m >= 0) fout[4 * N + n + (int64_t)(jy_m - y) * n0] = fs4;
            else fout[3 * N + n] = bounce_rule(wy_m, g.damp, fs4, fs3);
            if (jz_p >= 0) fout[5 * N + col + (int64_t)jz_p * plane] = fs5;
            else fout[6 * N + n] = bounce_rule(wz_p, g.damp, fs5, fs6);
            if (jz_m >= 0) fout[6 * N + col + (int64_t)jz_m * plane] = fs6;
            else fout[5 * N + n] = bounce_rule(wz_m, g.damp, fs6, fs5);
        }
        // advance one plane: z becomes z - 1, z + 1 becomes z, load z + 2
        azm[0] = cur.a[4];
        azm[1] = cur.a[5];
        azm[2] = cur.a[2];
        cur = nxt;
        nxt = nn;
    }
}

}  // namespace

hipError_t launch_step_general(const GeomDev& g, const ProbeArgs& pr, const MarchPlan& mp, const float* fin,
                               float* fout, hipStream_t st) {
    const int nt = mp.tx * mp.ty;
    if (!((mp.tx == 32 && mp.ty == 8) || (mp.tx == 64 && (mp.ty == 4 || mp.ty == 8))) || mp.lz < 1)
        return hipErrorInvalidValue;
    GenPlan plan;
    plan.ntx = (g.n0 + mp.tx - 1) / mp.tx;
    plan.nty = (g.n1 + mp.ty - 1) / mp.ty;
    plan.nch = (g.n2 + mp.lz - 1) / mp.lz;
    plan.lz = mp.lz;
    const int64_t tiles = (int64_t)plan.ntx * plan.nty * plan.nch;
    if (tiles > 0x7fffffffLL - 8) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)((tiles + kXcd - 1) / kXcd * kXcd);
    if (nt == 512)
        hipLaunchKernelGGL((general_march_kernel<64, 512>), dim3(blocks), dim3(512), 0, st, g, pr, plan, fin, fout);
    else if (mp.tx == 64)
        hipLaunchKernelGGL((general_march_kernel<64, 256>), dim3(blocks), dim3(256), 0, st, g, pr, plan, fin, fout);
    else
        hipLaunchKernelGGL((general_march_kernel<32, 256>), dim3(blocks), dim3(256), 0, st, g, pr, plan, fin, fout);
    return hipGetLastError();
}

}  // namespace lbw
