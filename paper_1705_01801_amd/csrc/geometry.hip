// Geometry coefficient tables, index maps, initial state and pressure.
//
// Coefficients (Sec. III and IV of the paper): sqrt(g), the inverse metric
// g^{ij} and the contracted Christoffel symbols Gamma^i = Gamma^i_jk g^jk,
// from closed forms per coordinate system, in FP64:
//   cylinder / polar (r, theta, z):  sqrt(g) = r, g^thth = 1/r^2,
//                                    Gamma^r = -1/r
//   horn (r, theta, z), radius s(z): sqrt(g) = r s^2,
//        g^rr = (1 + r^2 s'^2)/s^2, g^thth = 1/(r s)^2, g^zz = 1,
//        g^rz = -r s'/s, Gamma^r = -(1 + 2 r^2 s'^2 - r^2 s s'')/(r s^2)
//   torus (rho, theta, phi), u = R + rho cos(phi): sqrt(g) = rho u,
//        g^thth = 1/u^2, g^phph = 1/rho^2,
//        Gamma^rho = -(R + 2 rho cos(phi))/(rho u), Gamma^phi = sin(phi)/(rho u)
// (these follow from the printed metrics of Sec. IV with the torus
// Gamma^r_thth taken as -(R + r cos phi) cos phi).  Every coefficient depends
// on (q0, q2) only, so the tables have n0 x n2 entries.
#include "lbw_internal.h"

namespace lbw {
namespace {

__device__ double node_coord(const lbw_geometry_desc& d, int a, int i) {
    double h = (d.qmax[a] - d.qmin[a]) / d.n[a];
    if (d.bc_lo[a] == LBW_BC_PERIODIC) return d.qmin[a] + i * h;
    return d.qmin[a] + (i + 0.5) * h;
}

__device__ void horn_radius(const lbw_geometry_desc& d, double z, double* s, double* s1, double* s2) {
    if (d.kind == LBW_HORN) {
        double a = d.params[0], b = d.params[1], k = d.params[2];
        double e = exp(k * z);
        *s = a + b * e;
        *s1 = b * k * e;
        *s2 = b * k * k * e;
    } else {
        double lam = d.params[0], Z = d.params[1] - z;
        *s = pow(Z, -lam);
        *s1 = lam * pow(Z, -lam - 1.0);
        *s2 = lam * (lam + 1.0) * pow(Z, -lam - 2.0);
    }
}

__global__ void geometry_tables_kernel(lbw_geometry_desc d, double* __restrict__ tab64, float* __restrict__ tab32) {
    const int n0 = d.n[0];
    const int n2 = d.dim == 3 ? d.n[2] : 1;
    const int E = n0 * n2;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const int i0 = e % n0, i2 = e / n0;
    const double q0 = node_coord(d, 0, i0);
    const double q2 = d.dim == 3 ? node_coord(d, 2, i2) : 0.0;

    double G00 = 1.0, G11 = 1.0, G22 = 1.0, G02 = 0.0;
    double Ga0 = 0.0, Ga1 = 0.0, Ga2 = 0.0, sg = 1.0;
    switch (d.kind) {
    case LBW_POLAR2D:
    case LBW_CYLINDER:
        sg = q0;
        G11 = 1.0 / (q0 * q0);
        Ga0 = -1.0 / q0;
        break;
    case LBW_HORN:
    case LBW_BESSEL_HORN: {
        double s, s1, s2;
        horn_radius(d, q2, &s, &s1, &s2);
        const double r = q0;
        sg = r * s * s;
        G00 = (1.0 + r * r * s1 * s1) / (s * s);
        G11 = 1.0 / (r * r * s * s);
        G02 = -r * s1 / s;
        Ga0 = -(1.0 + 2.0 * r * r * s1 * s1 - r * r * s * s2) / (r * s * s);
        break;
    }
    case LBW_TORUS: {
        const double R = d.params[0], p = q0, cf = cos(q2), sf = sin(q2);
        const double u = R + p * cf;
        sg = p * u;
        G11 = 1.0 / (u * u);
        G22 = 1.0 / (p * p);
        Ga0 = -(R + 2.0 * p * cf) / (p * u);
        Ga2 = sf / (p * u);
        break;
    }
    default:  // LBW_BOX
        break;
    }

    double h[3] = {1.0, 1.0, 1.0};
    for (int a = 0; a < d.dim; ++a) h[a] = (d.qmax[a] - d.qmin[a]) / d.n[a];
    const double hr2 = d.h_ref * d.h_ref;
    const double M00 = hr2 * G00 / (h[0] * h[0]) - 1.0;
    const double M11 = hr2 * G11 / (h[1] * h[1]) - 1.0;
    const double M22 = d.dim == 3 ? hr2 * G22 / (h[2] * h[2]) - 1.0 : 0.0;
    const double M02 = d.dim == 3 ? hr2 * G02 / (h[0] * h[2]) : 0.0;
    const double g0 = hr2 * Ga0 / h[0];
    const double g1 = hr2 * Ga1 / h[1];
    const double g2 = d.dim == 3 ? hr2 * Ga2 / h[2] : 0.0;

    tab64[0 * E + e] = M00;
    tab64[1 * E + e] = M11;
    tab64[2 * E + e] = M22;
    tab64[3 * E + e] = M02;
    tab64[4 * E + e] = g0;
    tab64[5 * E + e] = g1;
    tab64[6 * E + e] = g2;
    tab64[7 * E + e] = sg;

    const double c2 = d.c * d.c;
    float* t = tab32 + (size_t)e * kTabF32;
    t[0] = (float)(c2 * M00);
    t[1] = (float)(c2 * M02);
    t[2] = (float)(c2 * M22);
    t[3] = (float)(c2 * M11);
    t[4] = (float)(0.5 * c2 * g0);
    t[5] = (float)(0.5 * c2 * g2);
    t[6] = 0.0f;
    t[7] = 0.0f;
}

__global__ void index_maps_kernel(GeomDev g, uint8_t* __restrict__ mask, int32_t* __restrict__ pull) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    const int Q = 2 * g.dim + 1;
    int idx[3];
    idx[0] = (int)(n % g.n0);
    const int64_t r = n / g.n0;
    idx[1] = (int)(r % g.n1);
    idx[2] = (int)(r / g.n1);
    const int nn[3] = {g.n0, g.n1, g.n2};
    const int64_t stride[3] = {1, g.n0, (int64_t)g.n0 * g.n1};
    uint8_t m = 0;
    pull[n] = (int32_t)n;
    for (int l = 1; l < Q; ++l) {
        const int a = (l - 1) >> 1;
        const int s = (l & 1) ? 1 : -1;
        int wall = 0;
        if (link_coord(idx[a], s, nn[a], g.bc_lo[a], g.bc_hi[a], &wall) < 0) m |= (uint8_t)(1u << (l - 1));
        const int j = link_coord(idx[a], -s, nn[a], g.bc_lo[a], g.bc_hi[a], &wall);
        pull[l * g.N + n] = j >= 0 ? (int32_t)(n + (int64_t)(j - idx[a]) * stride[a]) : -(1 + wall);
    }
    mask[n] = m;
}

// f_l = w_l sqrt(g) P0 at rest: w_0 = 1 - dim c^2, w_l = c^2 / 2, in FP64,
// rounded once to float.
__global__ void init_kernel(GeomDev g, double c2, const double* __restrict__ p0, float* __restrict__ f) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    const int Q = 2 * g.dim + 1;
    const double sg = g.sqrtg[sg_index(g, n)];
    const double w0 = 1.0 - g.dim * c2, w = 0.5 * c2;
    f[n] = (float)(w0 * sg * p0[n]);
    for (int l = 1; l < Q; ++l) f[l * g.N + n] = (float)(w * sg * p0[n]);
}

__global__ void pressure_kernel(GeomDev g, const float* __restrict__ f, double* __restrict__ p) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    const int Q = 2 * g.dim + 1;
    double s = 0.0;
    for (int l = 0; l < Q; ++l) s += (double)f[l * g.N + n];
    p[n] = s / g.sqrtg[sg_index(g, n)];
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_geometry_tables(const lbw_geometry_desc& d, double* tab64, float* tab32, hipStream_t st) {
    const int64_t E = (int64_t)d.n[0] * (d.dim == 3 ? d.n[2] : 1);
    hipLaunchKernelGGL(geometry_tables_kernel, dim3(blocks_for(E, 128)), dim3(128), 0, st, d, tab64, tab32);
    return hipGetLastError();
}

hipError_t launch_index_maps(const GeomDev& g, uint8_t* mask, int32_t* pull, hipStream_t st) {
    hipLaunchKernelGGL(index_maps_kernel, dim3(blocks_for(g.N, 256)), dim3(256), 0, st, g, mask, pull);
    return hipGetLastError();
}

hipError_t launch_init(const GeomDev& g, const double* p0, float* f, hipStream_t st) {
    hipLaunchKernelGGL(init_kernel, dim3(blocks_for(g.N, 256)), dim3(256), 0, st, g, (double)g.c2_64, p0, f);
    return hipGetLastError();
}

hipError_t launch_pressure(const GeomDev& g, const float* f, double* p, hipStream_t st) {
    hipLaunchKernelGGL(pressure_kernel, dim3(blocks_for(g.N, 256)), dim3(256), 0, st, g, f, p);
    return hipGetLastError();
}

}  // namespace lbw
