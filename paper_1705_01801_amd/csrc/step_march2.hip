// Two time steps per pass of the D3Q7 z-march (temporal blocking).
//
// The one-step kernels read every population once and write it once per
// step, 56 bytes per node update, and on grids that do not fit the caches
// that is the whole cost.  This kernel advances a tile from t to t+2 in one
// pass over memory, so the populations are read and written once per two
// updates:
//  - a workgroup of TX x (TY + 2) threads owns TY whole axis-0 rows (the
//    grid's walled axis 0 fits one row of TX lanes) over a chunk of planes
//    along axis 2;
//  - step A (t -> t+1) runs plane by plane on the tile and one halo row on
//    either side (TY + 2 rows), with the one-step kernel's data movement:
//    the own column's populations of planes z and z+1 in registers (plane
//    z+2 in flight), S of the plane staged in LDS for the axis-0 and axis-1
//    neighbours.  Its post-collision populations are not stored: along
//    axis 2 they stay in the thread that owns the column (a register carries
//    the +e2 one to the next plane, the -e2 one completes the plane below),
//    along axes 0 and 1 they are handed over through LDS.  The two rows
//    beyond the halo rows send one population each into them (+e1 into the
//    lower halo row, -e1 into the upper one); the first 2 TX threads load
//    those rows and run their collision too, the next 2 TX load the rows
//    beyond them for S only;
//  - a plane's state at t+1 is complete once step A has passed the plane
//    above it, and step B (t+1 -> t+2) also needs S(t+1) of the plane
//    above, so step B runs two planes behind step A, on the tile's own rows,
//    and pushes its populations to memory as the one-step kernel does;
//  - per node both steps call collide() of march_common.h in the same
//    order as a one-step launch would, so the result is that of two single
//    steps, bit for bit;
//  - probes: block 0 records time t from the input; the thread that owns a
//    probe node records time t+1 from the state it assembled; the last
//    workgroup to finish advances the step counter by two, so graph replays
//    need no host input.
// Chunks along axis 2 are extended by two planes of step A either side (the
// state at t+1 of planes z0-1 and z1 is needed), which is the price of the
// chunking besides the two halo rows.
#include "march_common.h"

namespace lbw {
namespace {

using namespace march;

constexpr int kTileProbes = 16;

template <int TX, int TY>
struct M2 {
    static constexpr int NT = TX * (TY + 2);
    static constexpr int W = TX + 2;          // LDS row: one pad entry either side of the axis-0 row
    static constexpr int SROWS = TY + 6;      // S(t) of extended rows -2 .. TY+3
    static constexpr int XROWS = TY + 4;      // populations handed over by rows -1 .. TY+2
    static constexpr int S1ROWS = TY + 2;     // S(t+1) of rows 0 .. TY+1
};

template <int TX, int TY>
struct M2Lds {
    float S[2][M2<TX, TY>::SROWS * M2<TX, TY>::W + 1];     // + a sink slot
    float X[4][M2<TX, TY>::XROWS * M2<TX, TY>::W + 1];
    float S1[2][M2<TX, TY>::S1ROWS * M2<TX, TY>::W + 1];
    float4 Elo[6][M2<TX, TY>::W + 1];                      // coefficient rows, slot = (plane - za0) mod 6
    float4 Ehi[6][M2<TX, TY>::W + 1];
    float B[2][2][TY * TX + 1];                            // step B: +-e0 populations along the row (2 planes)
    int pnode[kTileProbes], px[kTileProbes], py[kTileProbes], pz[kTileProbes];
    int pcount;
};

__device__ inline int wrap(int i, int n) { return ((i % n) + n) % n; }

// The lane's link indices (axis 0, axis 1) and activity flags passed
// through an empty asm statement once per plane: the compiler then derives
// the lane masks it selects with where they are used, instead of keeping
// them all in scalar registers for the whole march (more than the scalar
// file holds: the rest would be spilled to vector lanes and read back twice
// per use).
__device__ __forceinline__ void opaque_jx(Links& k) { asm volatile("" : "+v"(k.jx_p), "+v"(k.jx_m)); }
__device__ __forceinline__ void opaque_jy(Links& k) { asm volatile("" : "+v"(k.jy_p), "+v"(k.jy_m)); }
__device__ __forceinline__ bool opaque_bool(bool b) {
    int v = b;
    asm volatile("" : "+v"(v));
    return v != 0;
}

// PERY, PERZ: axis 1, axis 2 is periodic (every link along it present;
// the wall rules of that axis are compiled out).
template <int TX, int TY, bool PERY, bool PERZ>
__device__ __forceinline__ void march2_tile(const GeomDev& g, const ProbeArgs& pr, int64_t t, int ty, int z0, int z1,
                                            const float* __restrict__ fin, float* __restrict__ fout,
                                            M2Lds<TX, TY>& L) {
    using C = M2<TX, TY>;
    constexpr int W = C::W;
    const int n0 = g.n0, n1 = g.n1, n2 = g.n2;
    const uint32_t N = (uint32_t)g.N;
    const uint32_t plane = (uint32_t)n0 * (uint32_t)n1;
    const float c2 = g.c2, two_w0 = g.two_w0, damp = g.damp;
    const int lx = (int)(threadIdx.x % (unsigned)TX), ly = (int)(threadIdx.x / (unsigned)TX);
    // row tile ty (rows ty TY ..), planes [z0, z1) with 0 <= z0 < z1 <= n2
    const int y0 = ty * TY;
    const int hgt = min(TY, n1 - y0);
    const bool perz = g.bc_lo[2] == LBW_BC_PERIODIC, pery = PERY;
    // step A runs on march planes [za0, za1); the march runs on [za0, z1 + 2)
    const int za0 = perz ? z0 - 2 : max(z0 - 2, 0);
    const int za1 = perz ? z1 + 2 : min(z1 + 2, n2);

    // this thread's node: x = lx on the row of extended row ly (tile row ly - 1)
    const int yr = y0 - 1 + ly;
    const bool ypres = pery || (yr >= 0 && yr < n1);
    const int ya = pery ? wrap(yr, n1) : yr;
    const bool actA = lx < n0 && ypres;
    const bool actB = actA && ly >= 1 && ly <= hgt;
    // waves with no lane on the tile's own rows (all in the halo rows) skip
    // step B altogether (it has no barrier; its hand-over slots are read
    // only by lanes of the same row, which are on the tile's rows)
    const bool waveB = __builtin_amdgcn_ballot_w64(actB) != 0;
    Links kl{};
    kl.jx_p = link_coord(lx, +1, n0, g.bc_lo[0], g.bc_hi[0], &kl.wx_p);
    kl.jx_m = link_coord(lx, -1, n0, g.bc_lo[0], g.bc_hi[0], &kl.wx_m);
    kl.jy_p = ypres ? link_coord(ya, +1, n1, g.bc_lo[1], g.bc_hi[1], &kl.wy_p) : -1;
    kl.jy_m = ypres ? link_coord(ya, -1, n1, g.bc_lo[1], g.bc_hi[1], &kl.wy_m) : -1;
    const uint32_t col4 = actA ? ((uint32_t)lx + (uint32_t)n0 * (uint32_t)ya) * 4u : 0u;
    const int bcx_lo = g.bc_lo[0], bcx_hi = g.bc_hi[0], bcy_lo = g.bc_lo[1], bcy_hi = g.bc_hi[1];
    // byte offsets to the axis-1 neighbours' columns (used where the link exists)
    const uint32_t dyp4 = (uint32_t)((kl.jy_p - ya) * n0) * 4u, dym4 = (uint32_t)((kl.jy_m - ya) * n0) * 4u;

    // ring loader: rows -1 and TY+2 (loaded and collided: they send +e1 / -e1
    // into the halo rows), rows -2 and TY+3 (loaded for S only)
    const int rid = (int)(threadIdx.x / (unsigned)TX);  // 0..3 for loaders
    const int re = rid == 0 ? -1 : rid == 1 ? TY + 2 : rid == 2 ? -2 : TY + 3;
    const int ryr = y0 - 1 + re;
    const bool rpres = rid < 4 && (pery || (ryr >= 0 && ryr < n1));
    const int rya = pery ? wrap(ryr, n1) : ryr;
    const bool ring_on = rpres && lx < n0;
    const bool ring_col = ring_on && rid < 2;  // collides its ring node
    Links kr{};
    kr.jx_p = kl.jx_p;
    kr.jx_m = kl.jx_m;
    kr.wx_p = kl.wx_p;
    kr.wx_m = kl.wx_m;
    kr.jy_p = rpres ? link_coord(rya, +1, n1, g.bc_lo[1], g.bc_hi[1], &kr.wy_p) : -1;
    kr.jy_m = rpres ? link_coord(rya, -1, n1, g.bc_lo[1], g.bc_hi[1], &kr.wy_m) : -1;
    const uint32_t ring4 = ring_on ? ((uint32_t)lx + (uint32_t)n0 * (uint32_t)rya) * 4u : 0u;
    const int my_s = (ly + 2) * W + lx + 1;                  // own S(t) slot
    const int ring_s = ring_on ? (re + 2) * W + lx + 1 : C::SROWS * W;
    const int sinkS = C::SROWS * W;

    // coefficient-row loader: thread t < n0 stages entry t (x = -1 and n0 are
    // beyond the walls and never read)
    const bool erow_on = (int)threadIdx.x < n0;

    const uint32_t N4 = N * 4u, plane4 = plane * 4u;
    const __amdgpu_buffer_rsrc_t rin = make_rsrc(fin, 7u * N4);
    const __amdgpu_buffer_rsrc_t rout = make_rsrc(fout, 7u * N4);
    const __amdgpu_buffer_rsrc_t rtab = make_rsrc(g.tab, (uint32_t)n0 * (uint32_t)n2 * 32u);

    // march plane -> real plane (-1 beyond a wall); in the plane loop the
    // real planes of z - 2, z, z + 2 and z + 3 are carried along and
    // advanced by one plane each (radv: one compare and select, no division)
    auto rplane = [&](int z) -> int { return perz ? wrap(z, n2) : (z >= 0 && z < n2 ? z : -1); };
    // r: real plane of march plane zn - 1; returns that of zn
    auto radv = [&](int r, int zn) -> int {
        const int up = r + 1 == n2 ? 0 : r + 1;
        return perz ? up : (zn >= 0 && zn < n2 ? zn : -1);
    };
    // axis-2 links of real plane r (as link_coord gives them), from the two
    // ends' rules computed once
    const int bz_lo = g.bc_lo[2], bz_hi = g.bc_hi[2];
    const int jzp_end = bz_hi == LBW_BC_PERIODIC ? 0 : -1, wzp_end = bz_hi == LBW_BC_PERIODIC ? 0 : bz_hi;
    const int jzm_end = bz_lo == LBW_BC_PERIODIC ? n2 - 1 : -1, wzm_end = bz_lo == LBW_BC_PERIODIC ? 0 : bz_lo;
    auto zlinks = [&](int r, Links& k) {
        const bool up = r + 1 < n2, dn = r > 0;
        k.jz_p = up ? r + 1 : jzp_end;
        k.wz_p = up ? 0 : wzp_end;
        k.jz_m = dn ? r - 1 : jzm_end;
        k.wz_m = dn ? 0 : wzm_end;
    };
    auto erow_r = [&](int zr, float4& lo, float4& hi) {
        const bool on = erow_on && zr >= 0;
        const uint32_t off = on ? (uint32_t)(threadIdx.x + n0 * zr) * 32u : kOff;
        lo = bld4(rtab, off);
        hi = bld4(rtab, on ? off + 16u : kOff);
    };
    auto stage_erow = [&](int slot, const float4& lo, const float4& hi) {
        if (erow_on) {
            L.Elo[slot][threadIdx.x + 1] = lo;
            L.Ehi[slot][threadIdx.x + 1] = hi;
        }
    };

    // tile probes: those on the tile's own rows and planes record time t+1
    if (threadIdx.x == 0) L.pcount = 0;
    __syncthreads();
    if (t + 1 >= 0 && t + 1 < pr.t_max) {
        for (int p = threadIdx.x; p < pr.n; p += blockDim.x) {
            const int64_t node = pr.nodes[p];
            const int i0 = (int)(node % n0);
            const int i1 = (int)((node / n0) % n1);
            const int i2 = (int)(node / ((int64_t)n0 * n1));
            if (i1 >= y0 && i1 < y0 + hgt && i2 >= z0 && i2 < z1) {
                const int slot = atomicAdd(&L.pcount, 1);
                if (slot < kTileProbes) {
                    L.pnode[slot] = p;
                    L.px[slot] = i0;
                    L.py[slot] = i1;
                    L.pz[slot] = i2;
                }
            }
        }
    }

    __syncthreads();  // the tile's probe list complete
    const int tile_probes = __builtin_amdgcn_readfirstlane(min(L.pcount, kTileProbes));

    // ---- prologue: planes za0 - 1 (S only) and za0 (own column, ring,
    // staged S); coefficient rows za0 - 1 .. za0 + 1; in flight into the
    // loop: own column of plane za0 + 1, ring of plane za0 + 1, coefficient
    // row za0 + 2 ----
    float fA[7], fB[7], fC[7], rA[7], rB[7], rC[7], tmp[7];
    float Sm = 0.f, Sc = 0.f, Sp = 0.f;
    {
        const int zm = rplane(za0 - 1), zc = rplane(za0);
        bload7(rin, N4, actA && zm >= 0, col4 + (uint32_t)zm * plane4, tmp);
        bload7(rin, N4, actA && zc >= 0, col4 + (uint32_t)zc * plane4, fA);
        bload7(rin, N4, ring_on && zc >= 0, ring4 + (uint32_t)zc * plane4, rA);
        float4 a0, b0, a1, b1, a2, b2;
        erow_r(rplane(za0 - 1), a0, b0);
        erow_r(rplane(za0), a1, b1);
        erow_r(rplane(za0 + 1), a2, b2);
        Sm = sum7(tmp);
        Sc = sum7(fA);
        stage_erow(5, a0, b0);  // plane za0 - 1
        stage_erow(0, a1, b1);
        stage_erow(1, a2, b2);
        L.S[0][actA ? my_s : sinkS] = Sc;
        L.S[0][ring_s] = sum7(rA);
    }
    {
        // plane za1 itself is loaded where it exists: S(t) of the plane above
        // the last step-A plane
        const int zn = rplane(za0 + 1);
        const bool on = za0 + 1 <= za1 && zn >= 0;
        bload7(rin, N4, actA && on, col4 + (uint32_t)zn * plane4, fB);
        bload7(rin, N4, ring_on && on, ring4 + (uint32_t)zn * plane4, rB);
    }
    // coefficient rows in flight: eA holds row za0 + 2 for the first plane;
    // each plane stages the row loaded one plane earlier and loads the next
    // into the following slot (period three, by argument order, so no
    // register holding a load in flight is ever copied)
    float4 eA[2], eB[2], eC[2];
    erow_r(rplane(za0 + 2), eA[0], eA[1]);
    // real planes of march planes z, z + 2, z + 3 and z - 2 (carried along)
    int zrr = rplane(za0), zr2 = rplane(za0 + 2), zr3 = rplane(za0 + 3), zrb = rplane(za0 - 2);

    // state at t+1 of planes z-2 (for step B), z-1 and z (being assembled),
    // and S(t+1) of planes z-3 .. z-1
    float fa[7], fb[7], fz[7];
#pragma unroll
    for (int l = 0; l < 7; ++l) fa[l] = fb[l] = fz[l] = 0.f;
    float carry5 = 0.f;
    float S1a = 0.f, S1b = 0.f, S1c = 0.f;  // S(t+1) of planes z-3, z-2, z-1
    // step B's +-e0 stores of the previous plane, done after the next barrier
    // (the row hand-over through LDS then needs no barrier of its own)
    bool pend = false;
    uint32_t pend_nb = 0;
    float pend_v1w = 0.f, pend_v2w = 0.f;
    int pend_slot = 0;
    const int bo = (ly - 1) * TX + lx;  // step B hand-over slot
    auto flush_pending = [&](const Links& k, bool onB) {
        const float* B0 = L.B[pend_slot][0];
        const float* B1 = L.B[pend_slot][1];
        const float from_left = B0[lx > 0 && actB ? bo - 1 : TY * TX];
        const float from_right = B1[lx < TX - 1 && actB ? bo + 1 : TY * TX];
        const float in1 = k.jx_m >= 0 ? from_left : pend_v2w;
        const float in2 = k.jx_p >= 0 ? from_right : pend_v1w;
        bst(rout, pend && onB ? 1u * N4 + pend_nb : kOff, in1);
        bst(rout, pend && onB ? 2u * N4 + pend_nb : kOff, in2);
    };

    const int zend = z1 + 2;
    // One march plane z: step A on z (when z < za1), completion of plane z-1,
    // step B on z-2 (when it is one of the tile's planes).  f2 receives the
    // state at t+1 of plane z, f1 holds plane z-1, f0 plane z-2; fc / fnx /
    // fnn hold the own column at time t of planes z, z+1 and (loading) z+2,
    // rc / rn / rnn the ring's; the caller rotates all of them by argument
    // order (period three), so no register is copied.
    auto march_plane = [&](float (&f0)[7], float (&f1)[7], float (&f2)[7], float (&fc)[7], float (&fnx)[7],
                           float (&fnn)[7], float (&rc)[7], float (&rn)[7], float (&rnn)[7], float4 (&en)[2],
                           float4 (&e3)[2], int z, auto kc) {
        constexpr int K = decltype(kc)::value;  // z - za0 modulo 6 (the loop runs six planes per turn)
        const int sb = K & 1;
        const bool doA = z < za1;
        const int zr = zrr;
        Links kp = kl, krp = kr;
        // a wall code matters only where the link is missing, and there it
        // is that end's code: every lane takes the end codes, uniform, so
        // the wall rules are tested on the scalar unit
        kp.wx_p = bcx_hi;
        kp.wx_m = bcx_lo;
        opaque_jx(kp);
        if constexpr (PERY) {
            kp.jy_p = kp.jy_m = kp.wy_p = kp.wy_m = 0;
            krp.jy_p = krp.jy_m = krp.wy_p = krp.wy_m = 0;
        } else {
            kp.wy_p = krp.wy_p = bcy_hi;
            kp.wy_m = krp.wy_m = bcy_lo;
            opaque_jy(kp);
            opaque_jy(krp);
        }
        const bool pA = opaque_bool(actA), pB = opaque_bool(actB), pR = opaque_bool(ring_on);
        // loads consumed later: own column and ring of plane z+2 (S(t) of
        // plane z+1 comes from fnx), coefficient row z+3
        {
            const int zq = zr2;
            const bool on = z + 2 <= za1 && zq >= 0;
            bload7(rin, N4, pA && on, col4 + (uint32_t)zq * plane4, fnn);
            bload7(rin, N4, pR && on, ring4 + (uint32_t)zq * plane4, rnn);
        }
        erow_r(zr3, e3[0], e3[1]);
        Sp = sum7(fnx);
        const float Srp = sum7(rn);
        __syncthreads();  // S(t) of plane z, coefficient rows up to z+2, step B's hand-over visible
        if (pend) flush_pending(kp, pB);  // uniform
        pend = false;

        if (doA) {
            // (a step-A plane is always a real one: zr >= 0)
            Links k = kp;
            zlinks(zr, k);
            if constexpr (PERZ) k.jz_p = k.jz_m = 0;  // (step A uses only their presence)
            const float* Ls = L.S[sb];
            const float4 e_lo = L.Elo[K % 6][lx + 1], e_hi = L.Ehi[K % 6][lx + 1];
            const float4 enp = L.Elo[K % 6][lx + 2], enm = L.Elo[K % 6][lx];
            const float4 ezp = L.Elo[(K + 1) % 6][lx + 1];
            const float4 ezm = L.Elo[(K + 5) % 6][lx + 1];
            float fs[7];
            collide(fc, Sc, e_lo, e_hi, enp, enm, ezp, make_float2(ezm.y, ezm.z), Ls[my_s + 1], Ls[my_s - 1],
                    Ls[my_s + W], Ls[my_s - W], Sp, Sm, k, c2, two_w0, fs);
            const int xo = (ly + 1) * W + lx + 1;  // hand-over slot of row ly
            L.X[0][xo] = fs[1];
            L.X[1][xo] = fs[2];
            L.X[2][xo] = fs[3];
            L.X[3][xo] = fs[4];
            // the ring rows -1 and TY+2 (threads of the first 2 TX, whole
            // waves) send f*_3 (row -1, into row 0) and f*_4 (row TY+2, into
            // row TY+1): the axis-1 part of their collision
            // (2 TX is a multiple of 64: whole waves, tested as such)
            if (__builtin_amdgcn_readfirstlane((int)threadIdx.x) < 2 * TX) {
                const int ri = (re + 2) * W + lx + 1;
                float rs3, rs4;
                collide_axis1(rc[3], rc[4], sum7(rc), e_lo.w, Ls[ri + W], Ls[ri - W], krp, c2, rs3, rs4);
                const int ro = (re + 1) * W + lx + 1;
                // (row -1 sends f*_3 through X[2], row TY+2 f*_4 through X[3];
                // one store by index, no branch)
                constexpr int xs = C::XROWS * W + 1;
                (&L.X[0][0])[(rid == 0 ? 2 * xs : 3 * xs) + (ring_col ? ro : C::XROWS * W)] = rid == 0 ? rs3 : rs4;
            }
            __syncthreads();  // handed-over populations visible
            f2[0] = fs[0];
            f2[1] = k.jx_m >= 0 ? L.X[0][xo - 1] : bounce(k.wx_m, damp, fs[2], fs[1]);
            f2[2] = k.jx_p >= 0 ? L.X[1][xo + 1] : bounce(k.wx_p, damp, fs[1], fs[2]);
            f2[3] = k.jy_m >= 0 ? L.X[2][xo - W] : bounce(k.wy_m, damp, fs[4], fs[3]);
            f2[4] = k.jy_p >= 0 ? L.X[3][xo + W] : bounce(k.wy_p, damp, fs[3], fs[4]);
            f2[5] = k.jz_m >= 0 ? carry5 : bounce(k.wz_m, damp, fs[6], fs[5]);
            f2[6] = k.jz_p >= 0 ? 0.f : bounce(k.wz_p, damp, fs[5], fs[6]);
            if (k.jz_m >= 0) f1[6] = fs[6];
            carry5 = fs[5];
        }
        // plane z-1 is complete: its S(t+1) for step B's neighbours
        if (z - 1 >= za0 && z - 1 < za1) {
            S1c = sum7(f1);
            L.S1[(K + 1) & 1][actA ? ly * W + lx + 1 : C::S1ROWS * W] = S1c;  // plane z - 1
        }

        // step B on plane zb = z - 2
        const int zb = z - 2;
        if (zb >= z0 && zb < z1 && waveB) {
            const int zbr = zrb;
            Links k = kp;
            zlinks(zbr, k);
            const int jzp = k.jz_p, jzm = k.jz_m;  // the stores' planes
            if constexpr (PERZ) k.jz_p = k.jz_m = 0;
            const float* L1 = L.S1[K & 1];  // plane z - 2
            // (threads off the tile's rows read row 1 instead: every index stays in the array)
            const int s1 = (actB ? ly : 1) * W + lx + 1;
            const float4 e_lo = L.Elo[(K + 4) % 6][lx + 1], e_hi = L.Ehi[(K + 4) % 6][lx + 1];
            const float4 enp = L.Elo[(K + 4) % 6][lx + 2], enm = L.Elo[(K + 4) % 6][lx];
            const float4 ezp = L.Elo[(K + 5) % 6][lx + 1];
            const float4 ezm = L.Elo[(K + 3) % 6][lx + 1];
            float fs[7];
            collide(f0, S1b, e_lo, e_hi, enp, enm, ezp, make_float2(ezm.y, ezm.z), L1[s1 + 1], L1[s1 - 1],
                    L1[s1 + W], L1[s1 - W], S1c, S1a, k, c2, two_w0, fs);
            // probes at t+1 on this plane (the state f0 before step B)
            if (tile_probes > 0) {
                for (int i = 0; i < tile_probes; ++i) {
                    if (actB && L.pz[i] == zbr && L.py[i] == ya && L.px[i] == lx) {
                        double s = 0.0;
                        for (int l = 0; l < 7; ++l) s += (double)f0[l];
                        pr.trace[(t + 1) * pr.n + L.pnode[i]] = s / g.sqrtg[lx + (int64_t)n0 * zbr];
                    }
                }
            }
            // push: +-e0 along the row through LDS, stored after the next
            // barrier (aligned stores); the rest to their destinations (or the
            // wall rules) now
            pend_slot = K & 1;
            L.B[pend_slot][0][actB ? bo : TY * TX] = fs[1];
            L.B[pend_slot][1][actB ? bo : TY * TX] = fs[2];
            const uint32_t nb = col4 + (uint32_t)zbr * plane4;
            pend = true;
            pend_nb = nb;
            pend_v1w = bounce(k.wx_p, damp, fs[1], fs[2]);  // +e0 at the far wall, returned as -e0
            pend_v2w = bounce(k.wx_m, damp, fs[2], fs[1]);  // -e0 at the near wall, returned as +e0
            const uint32_t o3 = k.jy_p >= 0 ? 3u * N4 + nb + dyp4 : 4u * N4 + nb;
            const uint32_t o4 = k.jy_m >= 0 ? 4u * N4 + nb + dym4 : 3u * N4 + nb;
            const uint32_t o5 = k.jz_p >= 0 ? 5u * N4 + col4 + (uint32_t)jzp * plane4 : 6u * N4 + nb;
            const uint32_t o6 = k.jz_m >= 0 ? 6u * N4 + col4 + (uint32_t)jzm * plane4 : 5u * N4 + nb;
            const float v3 = k.jy_p >= 0 ? fs[3] : bounce(k.wy_p, damp, fs[3], fs[4]);
            const float v4 = k.jy_m >= 0 ? fs[4] : bounce(k.wy_m, damp, fs[4], fs[3]);
            const float v5 = k.jz_p >= 0 ? fs[5] : bounce(k.wz_p, damp, fs[5], fs[6]);
            const float v6 = k.jz_m >= 0 ? fs[6] : bounce(k.wz_m, damp, fs[6], fs[5]);
            bst(rout, pB ? nb : kOff, fs[0]);
            bst(rout, pB ? o3 : kOff, v3);
            bst(rout, pB ? o4 : kOff, v4);
            bst(rout, pB ? o5 : kOff, v5);
            bst(rout, pB ? o6 : kOff, v6);
        }
        S1a = S1b;
        S1b = S1c;

        // stage S(t) of plane z+1 and the coefficient row z+2 for the next
        // march plane (their slots were last read two barriers ago)
        if (z + 1 < zend) {
            L.S[sb ^ 1][actA ? my_s : sinkS] = Sp;
            L.S[sb ^ 1][ring_s] = Srp;
            stage_erow((K + 2) % 6, en[0], en[1]);
        }
        Sm = Sc;
        Sc = Sp;
        zrr = radv(zr, z + 1);
        zr2 = radv(zr2, z + 3);
        zr3 = radv(zr3, z + 4);
        zrb = radv(zrb, z - 1);
    };
    for (int z = za0;;) {
        if (z >= zend) break;
        march_plane(fa, fb, fz, fA, fB, fC, rA, rB, rC, eA, eB, z, std::integral_constant<int, 0>{});
        if (++z >= zend) break;
        march_plane(fb, fz, fa, fB, fC, fA, rB, rC, rA, eB, eC, z, std::integral_constant<int, 1>{});
        if (++z >= zend) break;
        march_plane(fz, fa, fb, fC, fA, fB, rC, rA, rB, eC, eA, z, std::integral_constant<int, 2>{});
        if (++z >= zend) break;
        march_plane(fa, fb, fz, fA, fB, fC, rA, rB, rC, eA, eB, z, std::integral_constant<int, 3>{});
        if (++z >= zend) break;
        march_plane(fb, fz, fa, fB, fC, fA, rB, rC, rA, eB, eC, z, std::integral_constant<int, 4>{});
        if (++z >= zend) break;
        march_plane(fz, fa, fb, fC, fA, fB, rC, rA, rB, eC, eA, z, std::integral_constant<int, 5>{});
        ++z;
    }
    __syncthreads();  // the last plane's hand-over visible
    if (pend) flush_pending(kl, actB);
    __syncthreads();  // LDS reuse by the next tile
}

template <int TX, int TY, bool PERY, bool PERZ>
__global__ __launch_bounds__(TX * (TY + 2)) void step_march2_kernel(GeomDev g, ProbeArgs pr, MarchPlan plan,
                                                                    const float* __restrict__ fin,
                                                                    float* __restrict__ fout) {
    __shared__ M2Lds<TX, TY> L;
    const int64_t t = *(volatile const int64_t*)pr.tcount;
    if (blockIdx.x == 0 && t >= 0 && t < pr.t_max) {
        // time t from the input
        for (int p = threadIdx.x; p < pr.n; p += blockDim.x) {
            const int64_t node = pr.nodes[p];
            double s = 0.0;
            for (int l = 0; l < 7; ++l) s += (double)fin[l * g.N + node];
            pr.trace[t * pr.n + p] = s / g.sqrtg[sg_index(g, node)];
        }
    }
    if (plan.lz > 0) {
        // tiles of chunk_z planes, XCD-contiguous ranges of the tile list
        const int xcd = blockIdx.x % kXcds;
        const int per_xcd_blocks = gridDim.x / kXcds;
        const int t_begin = (int)(plan.tiles * xcd / kXcds);
        const int t_end = (int)(plan.tiles * (xcd + 1) / kXcds);
        for (int tile = t_begin + (int)blockIdx.x / kXcds; tile < t_end; tile += per_xcd_blocks) {
            const int ty = tile % plan.nty, z0 = (tile / plan.nty) * plan.lz;
            if (z0 < g.n2) march2_tile<TX, TY, PERY, PERZ>(g, pr, t, ty, z0, min(z0 + plan.lz, g.n2), fin, fout, L);
        }
    } else {
        // balanced: this workgroup's share of the (row tile, plane) pairs,
        // marched as one segment per row tile it touches
        int64_t a = 0, e = 0;
        march2_share(plan.tiles, (int)gridDim.x, (int)blockIdx.x, &a, &e);
        while (a < e) {
            const int ty = (int)(a / g.n2), z0 = (int)(a % g.n2);
            const int z1 = (int)min((int64_t)g.n2, (int64_t)z0 + (e - a));
            march2_tile<TX, TY, PERY, PERZ>(g, pr, t, ty, z0, z1, fin, fout, L);
            a += z1 - z0;
        }
    }
    // the last workgroup to finish advances the step counter by two (every
    // workgroup read it before counting itself done)
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned prev = atomicAdd(pr.tdone, 1u);
        if (prev == gridDim.x - 1) {
            *(volatile int64_t*)pr.tcount = t + 2;
            *(volatile unsigned*)pr.tdone = 0u;
            __threadfence();
        }
    }
}

template <int TX, int TY>
int blocks_per_cu2() {
    int nb = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_march2_kernel<TX, TY, false, false>, TX * (TY + 2), 0);
    return e == hipSuccess && nb > 0 ? nb : 1;
}

}  // namespace

bool march2_shape_ok(int tx, int ty) {
    // 768 threads: the shapes whose registers fit three waves per SIMD
    // without spilling (taller tiles spill at four)
    return (tx == 96 && ty == 6) || (tx == 128 && ty == 4);
}

bool march2_fits(const GeomDev& g, int tx) {
    return g.dim == 3 && !g.sg_node && g.n0 <= tx && g.bc_lo[0] != LBW_BC_PERIODIC;
}

int march2_tile_probes() { return kTileProbes; }

int march2_blocks_per_cu(int tx, int ty) {
    return tx == 96 ? blocks_per_cu2<96, 6>() : blocks_per_cu2<128, 4>();
}

MarchPlan make_march2_plan(const GeomDev& g, int tx, int ty, int lz, int blocks) {
    MarchPlan p{};
    p.tx = tx;
    p.ty = ty;
    p.lz = lz < 0 ? 0 : lz;
    p.ntx = 1;
    p.nty = (g.n1 + ty - 1) / ty;
    // balanced (lz 0): tiles counts the (row tile, plane) pairs shared out
    p.nchunks = p.lz > 0 ? (g.n2 + p.lz - 1) / p.lz : 0;
    p.tiles = p.lz > 0 ? (int64_t)p.nty * p.nchunks : (int64_t)p.nty * g.n2;
    int b = blocks < kXcds ? kXcds : blocks;
    b = (b / kXcds) * kXcds;
    const int64_t cap = ((p.tiles + kXcds - 1) / kXcds) * kXcds;
    if (b > cap) b = (int)cap;
    if (b < kXcds) b = kXcds;
    p.blocks = b;
    return p;
}

namespace {
template <int TX, int TY>
void launch2_of(bool pery, bool perz, dim3 grid, dim3 block, hipStream_t st, const GeomDev& g, const ProbeArgs& pr,
                const MarchPlan& plan, const float* fin, float* fout) {
    if (pery && perz)
        hipLaunchKernelGGL((step_march2_kernel<TX, TY, true, true>), grid, block, 0, st, g, pr, plan, fin, fout);
    else if (pery)
        hipLaunchKernelGGL((step_march2_kernel<TX, TY, true, false>), grid, block, 0, st, g, pr, plan, fin, fout);
    else if (perz)
        hipLaunchKernelGGL((step_march2_kernel<TX, TY, false, true>), grid, block, 0, st, g, pr, plan, fin, fout);
    else
        hipLaunchKernelGGL((step_march2_kernel<TX, TY, false, false>), grid, block, 0, st, g, pr, plan, fin, fout);
}
}  // namespace

hipError_t launch_step_march2(const GeomDev& g, const ProbeArgs& pr, const MarchPlan& plan, const float* fin,
                              float* fout, hipStream_t st) {
    if (!march2_shape_ok(plan.tx, plan.ty) || !march2_fits(g, plan.tx) || !pr.tdone) return hipErrorInvalidValue;
    const dim3 grid(plan.blocks), block(plan.tx * (plan.ty + 2));
    const bool pery = g.bc_lo[1] == LBW_BC_PERIODIC, perz = g.bc_lo[2] == LBW_BC_PERIODIC;
    if (plan.tx == 96)
        launch2_of<96, 6>(pery, perz, grid, block, st, g, pr, plan, fin, fout);
    else
        launch2_of<128, 4>(pery, perz, grid, block, st, g, pr, plan, fin, fout);
    return hipGetLastError();
}

}  // namespace lbw
