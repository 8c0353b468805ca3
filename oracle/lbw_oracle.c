/*
 * FP64 CPU oracle for the curvilinear wave lattice-Boltzmann scheme of
 * Velasco, Munoz and Mendoza, "Lattice Boltzmann model for the simulation of
 * the wave equation in curvilinear coordinates" (arXiv 1705.01801).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; it exists so that the GPU library can be checked against a
 * plain, slow, obviously correct implementation.  It shares no code, header
 * or constant with the HIP library.
 *
 * Layout: populations f[l*N + n], n = i0 + n0*(i1 + n1*i2), l in the order
 *   0: rest, 1: +e0, 2: -e0, 3: +e1, 4: -e1, 5: +e2, 6: -e2.
 * Every routine is written as a sequence of whole-grid passes in the order the
 * paper states the method; there is no fusion or blocking.
 *
 * Readings of the paper taken here (all listed in the design notes):
 *  - weights: w_0 = 1 - D c^2, w_l = c^2/2 (the D3Q7 weight figure is missing;
 *    c_s = c makes the corrected equilibrium's stress c^2 sqrt(g) P delta,
 *    which the forcing term then completes to c^2 sqrt(g) P g^{ij}).
 *  - forcing: the Christoffel term carries sqrt(g) and the gradient term enters
 *    the corrected momentum with a minus sign, as the source of the curvilinear
 *    momentum conservation law requires.
 *  - gradient of A^{ij}: central difference over the two axis neighbours
 *    (the lattice-velocity Taylor formula of the field-derivative appendix on
 *    D3Q7/D2Q5 with w/c_s^2 = 1/2), using pre-collision S of the same step.
 *  - node placement: periodic axis q = qmin + i h; walled axis
 *    q = qmin + (i + 1/2) h, so walls sit half a link outside the end nodes.
 *  - walls: half-way bounce-back with damping (Sec. IV.A, pipe), free
 *    (copy of the boundary node's post-collision population), fixed
 *    (half-way anti-bounce-back, P = 0 on the wall).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_BOX = 0, ORC_POLAR2D = 1, ORC_CYLINDER = 2, ORC_HORN = 3, ORC_TORUS = 4, ORC_BESSEL_HORN = 5 };
enum { ORC_PERIODIC = 0, ORC_BOUNCEBACK = 1, ORC_FREE = 2, ORC_FIXED = 3 };

typedef struct {
    int32_t kind;
    int32_t dim;
    int32_t n[3];
    int32_t bc_lo[3];
    int32_t bc_hi[3];
    int32_t hermite;   /* 1: the Hermite-expansion equilibrium of Sec. II (Cartesian box only) */
    double qmin[3];
    double qmax[3];
    double href;
    double c;
    double damp;
    double par[4];
} orc_geom;

static int64_t orc_nodes(const orc_geom* g) {
    return (int64_t)g->n[0] * g->n[1] * (g->dim == 3 ? g->n[2] : 1);
}

static double orc_h(const orc_geom* g, int a) { return (g->qmax[a] - g->qmin[a]) / g->n[a]; }

static double orc_coord(const orc_geom* g, int a, int i) {
    double h = orc_h(g, a);
    if (g->bc_lo[a] == ORC_PERIODIC) return g->qmin[a] + i * h;
    return g->qmin[a] + (i + 0.5) * h;
}

/* ---------------------------------------------------------------------------
 * Coordinate embeddings X(q) into Euclidean space, with the first (J) and
 * second (H) partial derivatives.
 *   cylinder / polar: Sec. IV.A, cylindrical coordinate transformation
 *   horn:  Sec. IV.B generalised to x = r sigma(z) cos(theta), y = r sigma(z)
 *          sin(theta), z = z; sigma = a + b exp(k z) (exponential flare) or
 *          sigma = (Zmax - z)^(-lambda) (the paper's Bessel horn)
 *   torus: Sec. IV.C, toroidal coordinate transformation (rho, theta major,
 *          phi minor)
 * ------------------------------------------------------------------------- */
static void orc_sigma(const orc_geom* g, double z, double* s, double* s1, double* s2) {
    if (g->kind == ORC_HORN) {
        double a = g->par[0], b = g->par[1], k = g->par[2];
        double e = exp(k * z);
        *s = a + b * e;
        *s1 = b * k * e;
        *s2 = b * k * k * e;
    } else { /* Bessel horn: Z = Zmax - z, sigma = Z^-lambda */
        double lam = g->par[0], zmax = g->par[1];
        double Z = zmax - z;
        *s = pow(Z, -lam);
        *s1 = lam * pow(Z, -lam - 1.0);
        *s2 = lam * (lam + 1.0) * pow(Z, -lam - 2.0);
    }
}

static void orc_embedding(const orc_geom* g, const double q[3], double J[3][3], double H[3][3][3]) {
    memset(J, 0, 9 * sizeof(double));
    memset(H, 0, 27 * sizeof(double));
    switch (g->kind) {
    case ORC_BOX:
        for (int a = 0; a < 3; ++a) J[a][a] = 1.0;
        break;
    case ORC_POLAR2D:
    case ORC_CYLINDER: {
        double r = q[0], ct = cos(q[1]), st = sin(q[1]);
        J[0][0] = ct;  J[0][1] = -r * st;
        J[1][0] = st;  J[1][1] = r * ct;
        J[2][2] = 1.0;
        H[0][0][1] = H[0][1][0] = -st;  H[0][1][1] = -r * ct;
        H[1][0][1] = H[1][1][0] = ct;   H[1][1][1] = -r * st;
        break;
    }
    case ORC_HORN:
    case ORC_BESSEL_HORN: {
        double r = q[0], ct = cos(q[1]), st = sin(q[1]);
        double s, s1, s2;
        orc_sigma(g, q[2], &s, &s1, &s2);
        J[0][0] = s * ct;  J[0][1] = -r * s * st;  J[0][2] = r * s1 * ct;
        J[1][0] = s * st;  J[1][1] = r * s * ct;   J[1][2] = r * s1 * st;
        J[2][2] = 1.0;
        H[0][0][1] = H[0][1][0] = -s * st;
        H[0][0][2] = H[0][2][0] = s1 * ct;
        H[0][1][1] = -r * s * ct;
        H[0][1][2] = H[0][2][1] = -r * s1 * st;
        H[0][2][2] = r * s2 * ct;
        H[1][0][1] = H[1][1][0] = s * ct;
        H[1][0][2] = H[1][2][0] = s1 * st;
        H[1][1][1] = -r * s * st;
        H[1][1][2] = H[1][2][1] = r * s1 * ct;
        H[1][2][2] = r * s2 * st;
        break;
    }
    case ORC_TORUS: {
        double R = g->par[0];
        double p = q[0], ct = cos(q[1]), st = sin(q[1]), cf = cos(q[2]), sf = sin(q[2]);
        double u = R + p * cf;
        J[0][0] = cf * ct;  J[0][1] = -u * st;  J[0][2] = -p * sf * ct;
        J[1][0] = cf * st;  J[1][1] = u * ct;   J[1][2] = -p * sf * st;
        J[2][0] = sf;       J[2][1] = 0.0;      J[2][2] = p * cf;
        H[0][0][1] = H[0][1][0] = -cf * st;
        H[0][0][2] = H[0][2][0] = -sf * ct;
        H[0][1][1] = -u * ct;
        H[0][1][2] = H[0][2][1] = p * sf * st;
        H[0][2][2] = -p * cf * ct;
        H[1][0][1] = H[1][1][0] = cf * ct;
        H[1][0][2] = H[1][2][0] = -sf * st;
        H[1][1][1] = -u * st;
        H[1][1][2] = H[1][2][1] = -p * sf * ct;
        H[1][2][2] = -p * cf * st;
        H[2][0][2] = H[2][2][0] = cf;
        H[2][2][2] = -p * sf;
        break;
    }
    }
}

/* Inverse of a symmetric positive matrix of size d (2 or 3) by cofactors. */
static double orc_inverse(int d, const double m[3][3], double inv[3][3]) {
    memset(inv, 0, 9 * sizeof(double));
    if (d == 2) {
        double det = m[0][0] * m[1][1] - m[0][1] * m[1][0];
        inv[0][0] = m[1][1] / det;  inv[0][1] = -m[0][1] / det;
        inv[1][0] = -m[1][0] / det; inv[1][1] = m[0][0] / det;
        return det;
    }
    double c00 = m[1][1] * m[2][2] - m[1][2] * m[2][1];
    double c01 = m[1][2] * m[2][0] - m[1][0] * m[2][2];
    double c02 = m[1][0] * m[2][1] - m[1][1] * m[2][0];
    double det = m[0][0] * c00 + m[0][1] * c01 + m[0][2] * c02;
    inv[0][0] = c00 / det;
    inv[1][0] = c01 / det;
    inv[2][0] = c02 / det;
    inv[0][1] = (m[0][2] * m[2][1] - m[0][1] * m[2][2]) / det;
    inv[1][1] = (m[0][0] * m[2][2] - m[0][2] * m[2][0]) / det;
    inv[2][1] = (m[0][1] * m[2][0] - m[0][0] * m[2][1]) / det;
    inv[0][2] = (m[0][1] * m[1][2] - m[0][2] * m[1][1]) / det;
    inv[1][2] = (m[0][2] * m[1][0] - m[0][0] * m[1][2]) / det;
    inv[2][2] = (m[0][0] * m[1][1] - m[0][1] * m[1][0]) / det;
    return det;
}

/* Metric quantities at one point, in the coordinates' own units:
 *   g_ij = dX/dq^i . dX/dq^j, G = g^{-1}, sqrtg = sqrt(det g),
 *   Gamma^i_jk = G^{il} (dX/dq^l . d2X/dq^j dq^k)   (Christoffel, 2nd kind),
 *   Gc^i = Gamma^i_jk G^{jk}                         (Sec. III, corrected momentum). */
static void orc_metric_point(const orc_geom* g, const double q[3], double G[3][3], double* sqrtg, double Gc[3]) {
    int d = g->dim;
    double J[3][3], H[3][3][3], gm[3][3];
    orc_embedding(g, q, J, H);
    memset(gm, 0, sizeof(gm));
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            double s = 0.0;
            for (int a = 0; a < d; ++a) s += J[a][i] * J[a][j];
            gm[i][j] = s;
        }
    double det = orc_inverse(d, gm, G);
    *sqrtg = sqrt(det);
    double first[3][3][3]; /* dX/dq^l . d2X/dq^j dq^k */
    memset(first, 0, sizeof(first));
    for (int l = 0; l < d; ++l)
        for (int j = 0; j < d; ++j)
            for (int k = 0; k < d; ++k) {
                double s = 0.0;
                for (int a = 0; a < d; ++a) s += J[a][l] * H[a][j][k];
                first[l][j][k] = s;
            }
    for (int i = 0; i < 3; ++i) Gc[i] = 0.0;
    for (int i = 0; i < d; ++i) {
        double s = 0.0;
        for (int j = 0; j < d; ++j)
            for (int k = 0; k < d; ++k) {
                double gam = 0.0;
                for (int l = 0; l < d; ++l) gam += G[i][l] * first[l][j][k];
                s += gam * G[j][k];
            }
        Gc[i] = s;
    }
}

/* Per-node coefficients in lattice units (one lattice link per coordinate
 * step; h_ref is the physical length of one lattice unit, so that the
 * lattice wave speed is c = c_phys dt / h_ref):
 *   Mhat^{ij} = h_ref^2 G^{ij} / (h_i h_j) - delta^{ij}   stored as 6 planes
 *               in the order 00, 11, 22, 01, 02, 12
 *   Gamh^i    = h_ref^2 Gc^i / h_i                        3 planes
 *   sqrtg     = sqrt(det g) in the coordinates' own units. */
int orc_coeffs(const orc_geom* g, double* sqrtg, double* Mhat, double* Gamh) {
    int d = g->dim;
    int64_t N = orc_nodes(g);
    int n2 = d == 3 ? g->n[2] : 1;
    double h[3] = {1.0, 1.0, 1.0};
    for (int a = 0; a < d; ++a) h[a] = orc_h(g, a);
    double href = g->href;
    static const int ci[6] = {0, 1, 2, 0, 0, 1};
    static const int cj[6] = {0, 1, 2, 1, 2, 2};
    for (int i2 = 0; i2 < n2; ++i2)
        for (int i1 = 0; i1 < g->n[1]; ++i1)
            for (int i0 = 0; i0 < g->n[0]; ++i0) {
                int64_t n = i0 + (int64_t)g->n[0] * (i1 + (int64_t)g->n[1] * i2);
                double q[3] = {orc_coord(g, 0, i0), orc_coord(g, 1, i1), d == 3 ? orc_coord(g, 2, i2) : 0.0};
                double G[3][3], sg, Gc[3];
                orc_metric_point(g, q, G, &sg, Gc);
                sqrtg[n] = sg;
                for (int m = 0; m < 6; ++m) {
                    int i = ci[m], j = cj[m];
                    double v = 0.0;
                    if (i < d && j < d) v = href * href * G[i][j] / (h[i] * h[j]) - (i == j ? 1.0 : 0.0);
                    Mhat[m * N + n] = v;
                }
                for (int i = 0; i < 3; ++i) Gamh[i * N + n] = i < d ? href * href * Gc[i] / h[i] : 0.0;
            }
    return 0;
}

/* The same lattice-unit coefficients from given per-node metric data (a
 * geometry described only by its metric, Sec. III: the scheme needs sqrt(g),
 * the inverse metric and the contracted Christoffel symbols).  given holds
 * 10 planes of N values in the coordinates' own units: sqrt(g), G00, G11,
 * G22, G01, G02, G12, Gc0, Gc1, Gc2. */
int orc_coeffs_given(const orc_geom* g, const double* given, double* sqrtg, double* Mhat, double* Gamh) {
    int d = g->dim;
    int64_t N = orc_nodes(g);
    double h[3] = {1.0, 1.0, 1.0};
    for (int a = 0; a < d; ++a) h[a] = orc_h(g, a);
    double href = g->href;
    static const int ci[6] = {0, 1, 2, 0, 0, 1};
    static const int cj[6] = {0, 1, 2, 1, 2, 2};
    for (int64_t n = 0; n < N; ++n) {
        sqrtg[n] = given[n];
        for (int m = 0; m < 6; ++m) {
            int i = ci[m], j = cj[m];
            double v = 0.0;
            if (i < d && j < d) v = href * href * given[(1 + m) * N + n] / (h[i] * h[j]) - (i == j ? 1.0 : 0.0);
            Mhat[m * N + n] = v;
        }
        for (int i = 0; i < 3; ++i) Gamh[i * N + n] = i < d ? href * href * given[(7 + i) * N + n] / h[i] : 0.0;
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Lattice topology.
 * ------------------------------------------------------------------------- */
static int orc_axis_of(int l) { return (l - 1) / 2; }
static int orc_sign_of(int l) { return (l % 2 == 1) ? +1 : -1; }
static int orc_opposite(int l) { return (l % 2 == 1) ? l + 1 : l - 1; }

/* Neighbour of node idx one link along axis a in direction s.  Returns the
 * node index, wrapping periodic axes; returns -1 when the link crosses a wall
 * and stores that wall's boundary code in *bc. */
static int64_t orc_neighbour(const orc_geom* g, const int idx[3], int a, int s, int* bc) {
    int j[3] = {idx[0], idx[1], idx[2]};
    j[a] += s;
    if (j[a] < 0 || j[a] >= g->n[a]) {
        int code = (s < 0) ? g->bc_lo[a] : g->bc_hi[a];
        if (code == ORC_PERIODIC) {
            j[a] = (j[a] + g->n[a]) % g->n[a];
        } else {
            *bc = code;
            return -1;
        }
    }
    return j[0] + (int64_t)g->n[0] * (j[1] + (int64_t)g->n[1] * j[2]);
}

/* Index maps: mask[n] bit (l-1) is set when the link n -> n + xi_l crosses a
 * wall; pull[l*N + n] is the node that population l is pulled from when it
 * arrives at n (periodic wrap applied), or -(1 + bc) when it arrives through a
 * wall with boundary code bc. */
int orc_maps(const orc_geom* g, uint8_t* mask, int32_t* pull) {
    int d = g->dim, Q = 2 * d + 1;
    int64_t N = orc_nodes(g);
    int n2 = d == 3 ? g->n[2] : 1;
    for (int i2 = 0; i2 < n2; ++i2)
        for (int i1 = 0; i1 < g->n[1]; ++i1)
            for (int i0 = 0; i0 < g->n[0]; ++i0) {
                int idx[3] = {i0, i1, i2};
                int64_t n = i0 + (int64_t)g->n[0] * (i1 + (int64_t)g->n[1] * i2);
                uint8_t m = 0;
                pull[n] = (int32_t)n;
                for (int l = 1; l < Q; ++l) {
                    int bc = 0;
                    if (orc_neighbour(g, idx, orc_axis_of(l), orc_sign_of(l), &bc) < 0) m |= (uint8_t)(1u << (l - 1));
                    int64_t src = orc_neighbour(g, idx, orc_axis_of(l), -orc_sign_of(l), &bc);
                    pull[l * N + n] = src >= 0 ? (int32_t)src : -(1 + bc);
                }
                mask[n] = m;
            }
    return 0;
}

/* Initial populations: the corrected equilibrium (Sec. III) at rest,
 * f_l = w_l sqrt(g) P0, i.e. zero first moment. */
/* Weight of population l in the equilibrium at rest (J = 0) per unit of
 * sqrt(g) P: the corrected equilibrium of Sec. III (w_0 = 1 - D c^2,
 * w = c^2 / 2) or, for the Hermite form of Sec. II, its rest value
 * w [1 + (c^2 - c_s^2)(1 - D c_s^2) / (2 c_s^4)] with f_0 taking the rest. */
static double orc_rest_weight(const orc_geom* g, int l) {
    int d = g->dim;
    double c2 = g->c * g->c;
    if (!g->hermite) return (l == 0) ? 1.0 - d * c2 : 0.5 * c2;
    double cs2 = 1.0 / (d + 1), w = 0.5 * cs2;
    double wl = w * (1.0 + (c2 - cs2) * (1.0 - d * cs2) / (2.0 * cs2 * cs2));
    return (l == 0) ? 1.0 - 2 * d * wl : wl;
}

int orc_init(const orc_geom* g, const double* sqrtg, const double* P0, double* f) {
    int d = g->dim, Q = 2 * d + 1;
    int64_t N = orc_nodes(g);
    for (int l = 0; l < Q; ++l) {
        double w = orc_rest_weight(g, l);
        for (int64_t n = 0; n < N; ++n) f[l * N + n] = w * sqrtg[n] * P0[n];
    }
    return 0;
}

/* Mhat plane holding component (d, e). */
static int orc_mcomp(int d, int e) {
    if (d == e) return d;
    int lo = d < e ? d : e, hi = d < e ? e : d;
    if (lo == 0 && hi == 1) return 3;
    if (lo == 0 && hi == 2) return 4;
    return 5;
}

/* One time step t -> t+1 (BGK with tau = 1/2, Sec. II and III):
 *  pass 1: S = sqrt(g) P = sum_l f_l                     (zeroth moment)
 *  pass 2: K^d = sqrt(g) J'^d = sum_l f_l xi_l^d
 *                 - (1/2) c^2 S Gamh^d
 *                 - (1/2) d_e A^{de},  A^{de} = c^2 S Mhat^{de},
 *          d_e A^{de} = (A^{de}(x+e_e) - A^{de}(x-e_e)) / 2,
 *          f*_l = 2 f^eq_l - f_l with f^eq_0 = w_0 S, f^eq_l = w_l (S + xi_l.K / c^2)
 *  pass 3: pull streaming f_l(x, t+1) = f*_l(x - xi_l) with wall rules.
 * A values beyond a wall are mirrored: even for bounce-back and free walls,
 * odd for fixed (P = 0) walls; periodic axes wrap. */
/* Collision with the Hermite-expansion equilibrium of Sec. II (Cartesian,
 * no forcing), written as printed: the lattice weights of D2Q5/D3Q7
 * (w_0 = c_s^2 = 1 / (D + 1), w = c_s^2 / 2), P = sum_l f_l, J = sum_l f_l xi_l,
 * f_i^eq = w [P + xi_i.J / c_s^2 + P (c^2 - c_s^2)(xi_i^2 - D c_s^2) / (2 c_s^4)]
 * for i >= 1 (the printed 3 c_s^2 is D c_s^2 for D = 3) and
 * f_0^eq = P - sum_{i>=1} f_i^eq; post-collision f* = 2 f^eq - f (tau = 1/2). */
static void orc_collide_hermite(const orc_geom* g, const double* f, double* fs) {
    int d = g->dim, Q = 2 * d + 1;
    int64_t N = orc_nodes(g);
    double cs2 = 1.0 / (d + 1), w = 0.5 * cs2, c2 = g->c * g->c;
    for (int64_t n = 0; n < N; ++n) {
        double P = 0.0, J[3] = {0.0, 0.0, 0.0};
        for (int l = 0; l < Q; ++l) {
            P += f[l * N + n];
            if (l > 0) J[orc_axis_of(l)] += orc_sign_of(l) * f[l * N + n];
        }
        double sum = 0.0;
        for (int l = 1; l < Q; ++l) {
            double xiJ = orc_sign_of(l) * J[orc_axis_of(l)];
            double xi2 = 1.0;
            double feq = w * (P + xiJ / cs2 + P * (c2 - cs2) * (xi2 - d * cs2) / (2.0 * cs2 * cs2));
            sum += feq;
            fs[l * N + n] = 2.0 * feq - f[l * N + n];
        }
        fs[n] = 2.0 * (P - sum) - f[n];
    }
}

int orc_step(const orc_geom* g, const double* Mhat, const double* Gamh, double* f, double* fs, double* S) {
    int d = g->dim, Q = 2 * d + 1;
    int64_t N = orc_nodes(g);
    int n2 = d == 3 ? g->n[2] : 1;
    double c2 = g->c * g->c;
    double w0 = 1.0 - d * c2;

    for (int64_t n = 0; n < N; ++n) {
        double s = 0.0;
        for (int l = 0; l < Q; ++l) s += f[l * N + n];
        S[n] = s;
    }

    if (g->hermite) orc_collide_hermite(g, f, fs);
    else
    for (int i2 = 0; i2 < n2; ++i2)
        for (int i1 = 0; i1 < g->n[1]; ++i1)
            for (int i0 = 0; i0 < g->n[0]; ++i0) {
                int idx[3] = {i0, i1, i2};
                int64_t n = i0 + (int64_t)g->n[0] * (i1 + (int64_t)g->n[1] * i2);
                fs[n] = 2.0 * w0 * S[n] - f[n];
                for (int a = 0; a < d; ++a) {
                    double div = 0.0;
                    for (int e = 0; e < d; ++e) {
                        int mc = orc_mcomp(a, e);
                        double Ahere = c2 * S[n] * Mhat[mc * N + n];
                        double Aside[2];
                        for (int side = 0; side < 2; ++side) {
                            int bc = 0;
                            int64_t m = orc_neighbour(g, idx, e, side == 0 ? +1 : -1, &bc);
                            if (m >= 0) Aside[side] = c2 * S[m] * Mhat[mc * N + m];
                            else Aside[side] = (bc == ORC_FIXED) ? -Ahere : Ahere;
                        }
                        div += 0.5 * (Aside[0] - Aside[1]);
                    }
                    double J = f[(1 + 2 * a) * N + n] - f[(2 + 2 * a) * N + n];
                    double K = J - 0.5 * c2 * S[n] * Gamh[a * N + n] - 0.5 * div;
                    fs[(1 + 2 * a) * N + n] = c2 * S[n] + K - f[(1 + 2 * a) * N + n];
                    fs[(2 + 2 * a) * N + n] = c2 * S[n] - K - f[(2 + 2 * a) * N + n];
                }
            }

    for (int i2 = 0; i2 < n2; ++i2)
        for (int i1 = 0; i1 < g->n[1]; ++i1)
            for (int i0 = 0; i0 < g->n[0]; ++i0) {
                int idx[3] = {i0, i1, i2};
                int64_t n = i0 + (int64_t)g->n[0] * (i1 + (int64_t)g->n[1] * i2);
                f[n] = fs[n];
                for (int l = 1; l < Q; ++l) {
                    int bc = 0;
                    int64_t src = orc_neighbour(g, idx, orc_axis_of(l), -orc_sign_of(l), &bc);
                    if (src >= 0) {
                        f[l * N + n] = fs[l * N + src];
                    } else if (bc == ORC_BOUNCEBACK) {
                        f[l * N + n] = g->damp * fs[orc_opposite(l) * N + n];
                    } else if (bc == ORC_FREE) {
                        f[l * N + n] = fs[l * N + n];
                    } else { /* ORC_FIXED */
                        f[l * N + n] = -fs[orc_opposite(l) * N + n];
                    }
                }
            }
    return 0;
}

/* Probe pressure P = S / sqrt(g) at one node. */
static double orc_probe_value(const orc_geom* g, const double* f, const double* sqrtg, int64_t node) {
    int Q = 2 * g->dim + 1;
    int64_t N = orc_nodes(g);
    double s = 0.0;
    for (int l = 0; l < Q; ++l) s += f[l * N + node];
    return s / sqrtg[node];
}

/* Driven sources (Sec. IV.A and IV.C), imposed at time t on every source
 * node with v = amp sin(omega t):
 *  kind 0, pressure: the node is put at rest at P = v, f_0 = w_0 sqrt(g) P,
 *          f_l = w sqrt(g) P (the initial-state rule, zero first moment);
 *  kind 1 + a, flux along axis a (the oscillating plate of Sec. IV.A,
 *          J'_a = v): the node keeps its S = sum_l f_l and is put at the
 *          corrected equilibrium with sqrt(g) J'_a = sqrt(g) v and the other
 *          components zero, f_0 = w_0 S, f_{+-a} = w S +- sqrt(g) v / 2,
 *          the rest w S. */
static void orc_impose(const orc_geom* g, const double* sqrtg, double* f, int64_t t, const int64_t* src, int ns,
                       double amp, double omega, int kind) {
    int d = g->dim, Q = 2 * d + 1;
    int64_t N = orc_nodes(g);
    double v = amp * sin(omega * (double)t);
    for (int i = 0; i < ns; ++i) {
        int64_t n = src[i];
        double S = 0.0;
        if (kind > 0)
            for (int l = 0; l < Q; ++l) S += f[l * N + n];
        for (int l = 0; l < Q; ++l) {
            double w = orc_rest_weight(g, l);
            if (kind == 0) {
                f[l * N + n] = w * sqrtg[n] * v;
            } else {
                double val = w * S;
                if (l > 0 && orc_axis_of(l) == kind - 1) val += 0.5 * orc_sign_of(l) * sqrtg[n] * v;
                f[l * N + n] = val;
            }
        }
    }
}

/* Runs nsteps steps in place, from time t0.  At each time t = t0 + s the
 * sources (if any) are imposed, then the pressure at every probe is
 * appended, trace[s * np + p] = P(probe_p, t), then the step t -> t+1 runs.
 * work holds (Q + 1) * N doubles. */
int orc_run_driven(const orc_geom* g, const double* Mhat, const double* Gamh, const double* sqrtg, double* f,
                   double* work, int64_t nsteps, const int64_t* probes, int np, double* trace, int64_t t0,
                   const int64_t* src, int ns, double amp, double omega, int kind) {
    int Q = 2 * g->dim + 1;
    int64_t N = orc_nodes(g);
    double* fs = work;
    double* S = work + (int64_t)Q * N;
    for (int64_t s = 0; s < nsteps; ++s) {
        if (ns > 0) orc_impose(g, sqrtg, f, t0 + s, src, ns, amp, omega, kind);
        for (int p = 0; p < np; ++p) trace[s * np + p] = orc_probe_value(g, f, sqrtg, probes[p]);
        orc_step(g, Mhat, Gamh, f, fs, S);
    }
    return 0;
}

/* Undriven run: as orc_run_driven with no sources. */
int orc_run(const orc_geom* g, const double* Mhat, const double* Gamh, const double* sqrtg, double* f,
            double* work, int64_t nsteps, const int64_t* probes, int np, double* trace) {
    return orc_run_driven(g, Mhat, Gamh, sqrtg, f, work, nsteps, probes, np, trace, 0, NULL, 0, 0.0, 0.0, 0);
}

/* Scalar invariant sum_x sqrt(g) P = sum_x sum_l f_l (Sec. III, curvilinear
 * continuity equation). */
double orc_invariant(const orc_geom* g, const double* f) {
    int Q = 2 * g->dim + 1;
    int64_t N = orc_nodes(g);
    double s = 0.0;
    for (int64_t i = 0; i < (int64_t)Q * N; ++i) s += f[i];
    return s;
}

/* Pressure field P = S / sqrt(g) at every node. */
int orc_pressure(const orc_geom* g, const double* f, const double* sqrtg, double* P) {
    int64_t N = orc_nodes(g);
    for (int64_t n = 0; n < N; ++n) P[n] = orc_probe_value(g, f, sqrtg, n);
    return 0;
}
