// Device helpers shared by the z-marching D3Q7 step kernels: buffer
// addressing, wall rules and the per-node collision.  Every kernel that
// updates a node calls collide(), so the per-node arithmetic, and with it
// every result, is the same whichever kernel or launch shape runs it.
#pragma once

#include "lbw_internal.h"

namespace lbw {
namespace march {

constexpr int kXcds = 8;

__device__ inline float sum7(const float v[7]) {
    return v[0] + v[1] + v[2] + v[3] + v[4] + v[5] + v[6];
}

// Buffer addressing: 32-bit byte offsets from a per-geometry base; an offset
// of kOff is outside every range, so such a load returns 0 and such a store
// is dropped by the hardware range check.  Every load and store of a plane
// loop is issued by every lane, disabled ones with kOff, so the loop has no
// branch around a memory operation and the wait counts stay exact.
constexpr uint32_t kOff = 0x80000000u;
constexpr int kRsrcWord3 = 0x00020000;  // raw 32-bit buffer, gfx9-family format word

__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, kRsrcWord3);
}
__device__ inline float bld(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
__device__ inline float4 bld4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
    return make_float4(__int_as_float(v[0]), __int_as_float(v[1]), __int_as_float(v[2]), __int_as_float(v[3]));
}
__device__ inline void bst(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(v), r, (int)off, 0, 0);
}
// the same store, non-temporal when NTS (the gfx950 "nt" cache policy): for
// grids whose populations do not fit the caches, the written plane is not
// read again before a whole pass over memory, so keeping it cached is waste
constexpr int kNontemporal = 2;
template <bool NTS>
__device__ inline void bstp(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(v), r, (int)off, 0, NTS ? kNontemporal : 0);
}
// the 7 populations of the node at byte offset nb, or nothing (all zeros)
// (kOff + 6 N4 stays below 2^32 because 7 N4 < 2^31, so a disabled base
// keeps every population's offset out of range)
__device__ inline void bload7(__amdgpu_buffer_rsrc_t r, uint32_t N4, bool on, uint32_t nb, float v[7]) {
    const uint32_t base = on ? nb : kOff;
#pragma unroll
    for (int l = 0; l < 7; ++l) v[l] = bld(r, base + (uint32_t)l * N4);
}

// Driven node at time t (the sources of Sec. IV.A and IV.C): v holds the
// node's Q populations as loaded and receives the imposed ones.  With
// s = sin(omega t):
//   kind 0 (pressure, at rest): v_0 = a0 s, v_l = a1 s;
//   kind 1 + a (flux along axis a, S = sum_l v_l kept, summed in double):
//   v_0 = (1 - (Q - 1) a1) S, v_l = a1 S plus or minus a0 s on the two links
//   of axis a and a1 S on the others.
// Every kernel that imposes a source calls this, so a driven node gets the
// same bits whichever kernel imposes it.
template <int Q>
__device__ inline void drive_node(int kind, double a0, double a1, double omega, int64_t t, float (&v)[Q]) {
#pragma clang fp contract(off)
    const double s = sin(omega * (double)t);
    if (kind == 0) {
        v[0] = (float)(a0 * s);
        const float u = (float)(a1 * s);
#pragma unroll
        for (int l = 1; l < Q; ++l) v[l] = u;
        return;
    }
    double S = 0.0;
#pragma unroll
    for (int l = 0; l < Q; ++l) S += (double)v[l];
    const double h = a0 * s;
    v[0] = (float)((1.0 - (Q - 1) * a1) * S);
#pragma unroll
    for (int l = 1; l < Q; ++l) {
        double val = a1 * S;
        if ((l - 1) / 2 == kind - 1) val += (l & 1) ? h : -h;
        v[l] = (float)val;
    }
}

// bload7 with the non-temporal hint when NTL
template <bool NTL>
__device__ inline void bload7p(__amdgpu_buffer_rsrc_t r, uint32_t N4, bool on, uint32_t nb, float v[7]) {
    const uint32_t base = on ? nb : kOff;
#pragma unroll
    for (int l = 0; l < 7; ++l)
        v[l] = __int_as_float(
            __builtin_amdgcn_raw_buffer_load_b32(r, (int)(base + (uint32_t)l * N4), 0, NTL ? kNontemporal : 0));
}

// value beyond a wall: mirrored, odd for fixed walls
__device__ inline float ghost(int wall, float v) { return wall == LBW_BC_FIXED ? -v : v; }

// population that a wall returns into the opposite direction at the node:
// bounce-back D f*_l, free f*_{lbar} (the node's own), fixed -f*_l
__device__ inline float bounce(int wall, float damp, float out_l, float own_lb) {
    return wall == LBW_BC_BOUNCEBACK ? damp * out_l : (wall == LBW_BC_FREE ? own_lb : -out_l);
}

// The links of one node: neighbour coordinate along each axis and direction
// (-1 across a wall) and the wall code there.
struct Links {
    int jx_p, jx_m, jy_p, jy_m, jz_p, jz_m;
    int wx_p, wx_m, wy_p, wy_m, wz_p, wz_m;
};

// The axis-1 part of the collision below, f*_3 and f*_4 (the only
// coefficient it needs is c^2 Mhat11; its neighbours are those along axis 1).
// collide() computes its f*_3 and f*_4 by calling this, so a kernel that
// needs only these two gets the same bits.
__device__ __forceinline__ void collide_axis1(float f3, float f4, float S, float cM11, float Syp, float Sym,
                                              const Links& k, float c2, float& fs3, float& fs4) {
#pragma clang fp contract(off)
    const float sp = k.jy_p >= 0 ? Syp : ghost(k.wy_p, S);
    const float sm = k.jy_m >= 0 ? Sym : ghost(k.wy_m, S);
    const float dA = __builtin_fmaf(cM11, sp, -(cM11 * sm));  // A11 above minus below
    const float K1 = __builtin_fmaf(-0.25f, dA, f3 - f4);
    fs3 = __builtin_fmaf(c2, S, K1) - f3;
    fs4 = __builtin_fmaf(c2, S, -K1) - f4;
}

// Collision at one node (Sec. II evolution equation at tau = 1/2 with the
// corrected equilibrium, Christoffel and metric-gradient forcing of
// Sec. III), f* = 2 f^eq - f:
//   A^{de} = c^2 S Mhat^{de}, mirrored beyond walls (odd for fixed walls),
//   K_d = f_{+d} - f_{-d} - (c^2 / 2) S Gamh^d - (1/4) sum_e [A^{de}(x+e_e) - A^{de}(x-e_e)],
//   f*_0 = 2 w_0 S - f_0, f*_{+-d} = c^2 S +- K_d - f_{+-d}.
// fc: the node's populations; S their sum; e_lo / e_hi: the node's table
// record {c^2 Mhat00, 02, 22, 11}, {c^2 Gamh0 / 2, c^2 Gamh2 / 2, 0, 0};
// enp / enm: the low records of the axis-0 neighbours; ezp: that of the
// axis-2 neighbour above; em: (c^2 Mhat02, c^2 Mhat22) of the one below;
// Sx*, Sy*, Sp, Sm: S of the axis-0, axis-1 and axis-2 neighbours (read
// only where the link exists).
__device__ __forceinline__ void collide(const float (&fc)[7], float S, float4 e_lo, float4 e_hi, float4 enp,
                                        float4 enm, float4 ezp, float2 em, float Sxp, float Sxm, float Syp,
                                        float Sym, float Sp, float Sm, const Links& k, float c2, float two_w0,
                                        float (&fs)[7]) {
    // Every rounding is fixed by the source, not by the compiler: fused
    // multiply-adds only where written (each difference of A terms is one
    // product and one fused multiply-add, each K and f* sum takes the
    // products fused), every other product and sum rounded on its own.  So
    // every kernel that calls this gets the same bits for a node.
#pragma clang fp contract(off)
    const float cM00 = e_lo.x, cM02 = e_lo.y, cM22 = e_lo.z, cM11 = e_lo.w;
    const float hG0 = e_hi.x, hG2 = e_hi.y;
    // the neighbour's coefficient and S where the link exists, the node's
    // own coefficient and its mirrored S beyond a wall
    const bool xp = k.jx_p >= 0, xm = k.jx_m >= 0;
    const float sxp = xp ? Sxp : ghost(k.wx_p, S), sxm = xm ? Sxm : ghost(k.wx_m, S);
    const float c00p = xp ? enp.x : cM00, c20p = xp ? enp.y : cM02;
    const float c00m = xm ? enm.x : cM00, c20m = xm ? enm.y : cM02;
    const bool zp = k.jz_p >= 0, zm = k.jz_m >= 0;
    const float szp = zp ? Sp : ghost(k.wz_p, S), szm = zm ? Sm : ghost(k.wz_m, S);
    const float c02p = zp ? ezp.y : cM02, c22p = zp ? ezp.z : cM22;
    const float c02m = zm ? em.x : cM02, c22m = zm ? em.y : cM22;
    const float d00 = __builtin_fmaf(c00p, sxp, -(c00m * sxm));
    const float d20 = __builtin_fmaf(c20p, sxp, -(c20m * sxm));
    const float d02 = __builtin_fmaf(c02p, szp, -(c02m * szm));
    const float d22 = __builtin_fmaf(c22p, szp, -(c22m * szm));
    float K0 = __builtin_fmaf(-hG0, S, fc[1] - fc[2]);
    K0 = __builtin_fmaf(-0.25f, d00, K0);
    K0 = __builtin_fmaf(-0.25f, d02, K0);
    const float K2 = __builtin_fmaf(-0.25f, d22 + d20, __builtin_fmaf(-hG2, S, fc[5] - fc[6]));
    fs[0] = __builtin_fmaf(two_w0, S, -fc[0]);
    fs[1] = __builtin_fmaf(c2, S, K0) - fc[1];
    fs[2] = __builtin_fmaf(c2, S, -K0) - fc[2];
    collide_axis1(fc[3], fc[4], S, cM11, Syp, Sym, k, c2, fs[3], fs[4]);
    fs[5] = __builtin_fmaf(c2, S, K2) - fc[5];
    fs[6] = __builtin_fmaf(c2, S, -K2) - fc[6];
}

}  // namespace march
}  // namespace lbw
