// C-ABI entry points declared in include/lbw.h.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "host_util.h"

using lbw::GeomDev;
using lbw::fail;
using lbw::hip_fail;

struct lbw_geometry {
    lbw_geometry_desc d;
    int Q = 0;
    int64_t N = 0;
    int64_t E = 0;  // table entries n0 * n2 (a geometry given by its metric: N)
    bool general = false;  // given by its metric: per-node tables, general step kernel
    double* tab64 = nullptr;
    float* tab32 = nullptr;
    hipStream_t stream = nullptr;
    GeomDev dev{};
    lbw::MarchPlan plan{};  // launch shape of the 3-D step
    lbw::MarchPlan plan2{}; // launch shape of the two-step pass, used when use2
    bool use2 = false;
    int plan_version = 0;   // bumped on every change of plan
};

struct lbw_state {
    lbw_geometry* g = nullptr;
    float* f[2] = {nullptr, nullptr};
    int cur = 0;
    int64_t t = 0;
    int64_t t_max = 0;
    int n_probes = 0;
    double* trace = nullptr;
    int64_t* d_probes = nullptr;
    int64_t* d_tcount = nullptr;
    hipStream_t stream = nullptr;
    double* mode_work = nullptr;
    size_t mode_work_bytes = 0;
    double* mode_out = nullptr;  // device, 2 * mode_k
    int mode_k = 0;
    int64_t* d_scratch_count = nullptr;  // step counter for timing launches
    unsigned* d_done = nullptr;          // workgroups done in a two-step launch (real and timing runs)
    std::vector<int64_t> probes_host;    // probe nodes (tiles of the two-step pass hold at most a few)
    lbw::SourceEntry* d_src = nullptr;   // driven sources, imposed before every step
    int n_src = 0;
    double* d_amp = nullptr;             // response intensities (n_probes)
    // graph-captured step blocks, one per starting buffer parity
    int graph_block = 32;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int graph_version = -1;
    bool graph_two = false;  // the captured blocks are two-step launches
};

namespace {

thread_local std::string g_err;

// tuned launch shapes per grid shape (n0, n1, n2) -> one-step (tile_x, tile_y,
// chunk_z, blocks) and two-step shape (tile_x 0: one-step launches)
struct Tuned {
    int tx, ty, lz, blocks, nts;
    int tx2, ty2, lz2, blocks2;
};
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, Tuned> g_tuned;

bool is_finite(double v) { return std::isfinite(v); }

}  // namespace

namespace lbw {

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    if (e == hipErrorOutOfMemory) return fail(LBW_ENOMEM, "%s: %s", what, hipGetErrorString(e));
    return fail(LBW_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

int device_cus(int* cus) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "device query");
    HIP_TRY(hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev), "device query");
    return LBW_OK;
}

lbw_geometry_desc normalised(const lbw_geometry_desc& in) {
    lbw_geometry_desc d = in;
    if (d.dim == 2) {
        d.n[2] = 1;
        d.bc_lo[2] = d.bc_hi[2] = LBW_BC_PERIODIC;
        d.qmin[2] = 0.0;
        d.qmax[2] = 1.0;
    }
    return d;
}

double lattice_c2(const lbw_geometry_desc& d) {
    const double c2 = d.c * d.c;
    if (d.equilibrium != LBW_EQ_HERMITE) return c2;
    const double cs2 = 1.0 / (d.dim + 1);
    return cs2 + (c2 - cs2) * (1.0 - d.dim * cs2) / (2.0 * cs2);
}

GeomDev make_geomdev(const lbw_geometry_desc& d, const float* tab32, const double* sqrtg) {
    GeomDev v{};
    v.dim = d.dim;
    v.n0 = d.n[0];
    v.n1 = d.n[1];
    v.n2 = d.n[2];
    v.N = (int64_t)d.n[0] * d.n[1] * d.n[2];
    for (int a = 0; a < 3; ++a) {
        v.bc_lo[a] = d.bc_lo[a];
        v.bc_hi[a] = d.bc_hi[a];
    }
    const double c2 = lattice_c2(d);
    v.c2 = (float)c2;
    v.two_w0 = (float)(2.0 * (1.0 - d.dim * c2));
    v.damp = (float)d.damping;
    v.c2_64 = c2;
    v.tab = tab32;
    v.sqrtg = sqrtg;
    return v;
}

int validate_desc(const lbw_geometry_desc* d) {
    if (!d) return fail(LBW_EINVAL, "descriptor is NULL");
    if (d->kind < LBW_BOX || d->kind > LBW_GENERAL) return fail(LBW_EINVAL, "unknown kind %d", d->kind);
    if (d->dim != 2 && d->dim != 3) return fail(LBW_EINVAL, "dim must be 2 or 3 (got %d)", d->dim);
    if (d->kind == LBW_POLAR2D && d->dim != 2) return fail(LBW_EINVAL, "polar2d needs dim 2");
    if (d->kind != LBW_POLAR2D && d->kind != LBW_BOX && d->dim != 3) return fail(LBW_EINVAL, "kind needs dim 3");
    if (d->equilibrium != LBW_EQ_CORRECTED && d->equilibrium != LBW_EQ_HERMITE)
        return fail(LBW_EINVAL, "unknown equilibrium %d", d->equilibrium);
    if (d->equilibrium == LBW_EQ_HERMITE && d->kind != LBW_BOX)
        return fail(LBW_EINVAL, "the Hermite equilibrium applies to Cartesian boxes only");
    int64_t N = 1;
    for (int a = 0; a < d->dim; ++a) {
        if (d->n[a] < 1) return fail(LBW_EINVAL, "n[%d] = %d < 1", a, d->n[a]);
        if (!is_finite(d->qmin[a]) || !is_finite(d->qmax[a]) || !(d->qmax[a] > d->qmin[a]))
            return fail(LBW_EINVAL, "axis %d: need qmin < qmax", a);
        for (int side = 0; side < 2; ++side) {
            int code = side ? d->bc_hi[a] : d->bc_lo[a];
            if (code < LBW_BC_PERIODIC || code > LBW_BC_FIXED) return fail(LBW_EINVAL, "axis %d: bad wall code", a);
        }
        if ((d->bc_lo[a] == LBW_BC_PERIODIC) != (d->bc_hi[a] == LBW_BC_PERIODIC))
            return fail(LBW_EINVAL, "axis %d: periodic faces must be paired", a);
        N *= d->n[a];
    }
    // each population buffer (Q * N floats) is addressed with 32-bit byte offsets
    if (4LL * (2 * d->dim + 1) * N > 2147483647LL)
        return fail(LBW_EINVAL, "too many nodes (%lld): 4 Q N bytes must stay below 2^31", (long long)N);
    if (!is_finite(d->h_ref) || !(d->h_ref > 0.0)) return fail(LBW_EINVAL, "h_ref must be > 0");
    if (!is_finite(d->c) || !(d->c > 0.0)) return fail(LBW_EINVAL, "c must be > 0");
    if (!is_finite(d->damping) || d->damping < 0.0 || d->damping > 1.0) return fail(LBW_EINVAL, "damping outside [0,1]");
    switch (d->kind) {
    case LBW_POLAR2D:
    case LBW_CYLINDER:
        if (!(d->qmin[0] > 0.0)) return fail(LBW_EINVAL, "radius must stay > 0");
        break;
    case LBW_HORN: {
        if (!(d->qmin[0] > 0.0)) return fail(LBW_EINVAL, "radius must stay > 0");
        const double a = d->params[0], b = d->params[1], k = d->params[2];
        for (int end = 0; end < 2; ++end) {
            const double z = end ? d->qmax[2] : d->qmin[2];
            const double s = a + b * std::exp(k * z);
            if (!is_finite(s) || !(s > 0.0)) return fail(LBW_EINVAL, "horn radius must stay > 0");
        }
        if (!(a > 0.0) && !(b > 0.0)) return fail(LBW_EINVAL, "horn radius must stay > 0");
        break;
    }
    case LBW_BESSEL_HORN:
        if (!(d->qmin[0] > 0.0)) return fail(LBW_EINVAL, "radius must stay > 0");
        if (!(d->params[1] > d->qmax[2])) return fail(LBW_EINVAL, "Bessel horn needs Zmax > z range");
        break;
    case LBW_TORUS:
        if (!(d->qmin[0] > 0.0)) return fail(LBW_EINVAL, "rho must stay > 0");
        if (!(d->params[0] > d->qmax[0])) return fail(LBW_EINVAL, "torus needs R > rho_max");
        break;
    default:
        break;
    }
    return LBW_OK;
}

}  // namespace lbw

extern "C" {

const char* lbw_last_error(void) { return g_err.c_str(); }

int lbw_make_geometry(const lbw_geometry_desc* desc, void* stream, lbw_geometry_t* out) {
    if (!out) return fail(LBW_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = lbw::validate_desc(desc);
    if (rc) return rc;
    if (desc->kind == LBW_GENERAL)
        return fail(LBW_EINVAL, "a geometry given by its metric is made with lbw_make_geometry_general");
    lbw_geometry* g = new lbw_geometry();
    g->d = lbw::normalised(*desc);
    const lbw_geometry_desc& d = g->d;
    g->Q = 2 * d.dim + 1;
    g->N = (int64_t)d.n[0] * d.n[1] * d.n[2];
    g->E = (int64_t)d.n[0] * d.n[2];
    g->stream = (hipStream_t)stream;
    int cus = 0;
    hipError_t e = hipMalloc(&g->tab64, sizeof(double) * lbw::kTabF64 * g->E);
    if (e == hipSuccess) e = hipMalloc(&g->tab32, sizeof(float) * lbw::kTabF32 * g->E);
    if (e == hipSuccess) e = lbw::launch_geometry_tables(d, g->tab64, g->tab32, g->stream);
    if (e == hipSuccess && lbw::device_cus(&cus) != LBW_OK) e = hipErrorInvalidDevice;
    if (e != hipSuccess) {
        (void)hipFree(g->tab64);
        (void)hipFree(g->tab32);
        delete g;
        return hip_fail(e, "lbw_make_geometry");
    }
    g->dev = lbw::make_geomdev(d, g->tab32, g->tab64 + 7 * g->E);
    const GeomDev& v = g->dev;
    if (d.dim == 3) {
        const int tx = lbw::march_tx_for(v.n0);
        g->plan = lbw::make_march_plan(v, tx, 256 / tx, 16, cus * lbw::march_blocks_per_cu(tx, 256 / tx));
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(std::make_tuple(v.n0, v.n1, v.n2));
        if (it != g_tuned.end()) {
            const Tuned& c = it->second;
            g->plan = lbw::make_march_plan(v, c.tx, c.ty, c.lz, c.blocks);
            g->plan.nts = c.nts;
            if (c.tx2 > 0 && lbw::march2_fits(v, c.tx2)) {
                g->plan2 = lbw::make_march2_plan(v, c.tx2, c.ty2, c.lz2, c.blocks2);
                g->use2 = true;
            }
        }
    }
    *out = g;
    return LBW_OK;
}

int lbw_make_geometry_general(const lbw_geometry_desc* desc, const double* metric, void* stream,
                              lbw_geometry_t* out) {
    if (!out) return fail(LBW_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = lbw::validate_desc(desc);
    if (rc) return rc;
    if (desc->kind != LBW_GENERAL || desc->dim != 3) return fail(LBW_EINVAL, "kind must be LBW_GENERAL with dim 3");
    if (!metric) return fail(LBW_EINVAL, "metric is NULL");
    const lbw_geometry_desc d = lbw::normalised(*desc);
    const int64_t N = (int64_t)d.n[0] * d.n[1] * d.n[2];
    // the kernel addresses the nine coefficient planes with 32-bit byte offsets
    if (4LL * lbw::kGenF32 * N > 2147483647LL)
        return fail(LBW_EINVAL, "too many nodes (%lld) for per-node coefficients: 36 N bytes must stay below 2^31",
                    (long long)N);
    for (int64_t i = 0; i < lbw::kGenF64 * N; ++i)
        if (!std::isfinite(metric[i])) return fail(LBW_EINVAL, "non-finite metric value (plane %lld)", (long long)(i / N));
    for (int64_t n = 0; n < N; ++n)
        if (!(metric[n] > 0.0)) return fail(LBW_EINVAL, "sqrt(g) must be > 0 (node %lld)", (long long)n);
    // lattice units (Sec. III): Mhat^{ij} = h_ref^2 G^{ij} / (h_i h_j) - delta^{ij},
    // Gamh^i = h_ref^2 Gamma^i / h_i; FP32 planes c^2 Mhat and c^2 Gamh / 2
    double h[3];
    for (int a = 0; a < 3; ++a) h[a] = (d.qmax[a] - d.qmin[a]) / d.n[a];
    static const int ci[6] = {0, 1, 2, 0, 0, 1};
    static const int cj[6] = {0, 1, 2, 1, 2, 2};
    const double hr2 = d.h_ref * d.h_ref, c2 = d.c * d.c;
    std::vector<double> t64((size_t)lbw::kGenF64 * N);
    std::vector<float> t32((size_t)lbw::kGenF32 * N);
    for (int64_t n = 0; n < N; ++n) {
        for (int m = 0; m < 6; ++m) {
            const double v = hr2 * metric[(1 + m) * N + n] / (h[ci[m]] * h[cj[m]]) - (ci[m] == cj[m] ? 1.0 : 0.0);
            t64[m * N + n] = v;
            t32[m * N + n] = (float)(c2 * v);
        }
        for (int a = 0; a < 3; ++a) {
            const double v = hr2 * metric[(7 + a) * N + n] / h[a];
            t64[(6 + a) * N + n] = v;
            t32[(6 + a) * N + n] = (float)(0.5 * c2 * v);
        }
        t64[9 * N + n] = metric[n];
    }
    lbw_geometry* g = new lbw_geometry();
    g->d = d;
    g->Q = 7;
    g->N = N;
    g->E = N;
    g->general = true;
    g->stream = (hipStream_t)stream;
    hipError_t e = hipMalloc(&g->tab64, sizeof(double) * t64.size());
    if (e == hipSuccess) e = hipMalloc(&g->tab32, sizeof(float) * t32.size());
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->tab64, t64.data(), sizeof(double) * t64.size(), hipMemcpyHostToDevice, g->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->tab32, t32.data(), sizeof(float) * t32.size(), hipMemcpyHostToDevice, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);  // host tables go out of scope
    if (e != hipSuccess) {
        (void)hipFree(g->tab64);
        (void)hipFree(g->tab32);
        delete g;
        return hip_fail(e, "lbw_make_geometry_general");
    }
    g->dev = lbw::make_geomdev(d, g->tab32, g->tab64 + 9 * N);
    g->dev.sg_node = 1;
    {
        const int tx = g->dev.n0 > 32 ? 64 : 32;  // 64 x 8 or 32 x 8 tiles, 16 planes
        g->plan = lbw::make_march_plan(g->dev, tx, 8, 16, 8);
        g->plan.blocks = (int)g->plan.tiles;
    }
    *out = g;
    return LBW_OK;
}

int lbw_free_geometry(lbw_geometry_t g) {
    if (!g) return LBW_OK;
    (void)hipStreamSynchronize(g->stream);
    (void)hipFree(g->tab64);
    (void)hipFree(g->tab32);
    delete g;
    return LBW_OK;
}

int lbw_geometry_export(lbw_geometry_t g, int what, void* host_dst, size_t bytes) {
    if (!g || !host_dst) return fail(LBW_EINVAL, "NULL argument");
    size_t need = 0;
    switch (what) {
    case LBW_EXPORT_TABLE_F64: need = sizeof(double) * (g->general ? lbw::kGenF64 : lbw::kTabF64) * g->E; break;
    case LBW_EXPORT_MASK_U8: need = (size_t)g->N; break;
    case LBW_EXPORT_PULL_I32: need = sizeof(int32_t) * g->Q * g->N; break;
    default: return fail(LBW_EINVAL, "unknown export %d", what);
    }
    if (bytes != need) return fail(LBW_EINVAL, "export %d needs %zu bytes, got %zu", what, need, bytes);
    if (what == LBW_EXPORT_TABLE_F64) {
        HIP_TRY(hipMemcpyAsync(host_dst, g->tab64, need, hipMemcpyDeviceToHost, g->stream), "export table");
        HIP_TRY(hipStreamSynchronize(g->stream), "export table");
        return LBW_OK;
    }
    uint8_t* mask = nullptr;
    int32_t* pull = nullptr;
    HIP_TRY(hipMalloc(&mask, g->N), "export maps");
    hipError_t e = hipMalloc(&pull, sizeof(int32_t) * g->Q * g->N);
    if (e == hipSuccess) e = lbw::launch_index_maps(g->dev, mask, pull, g->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(host_dst, what == LBW_EXPORT_MASK_U8 ? (void*)mask : (void*)pull, need,
                           hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    (void)hipFree(mask);
    (void)hipFree(pull);
    if (e != hipSuccess) return hip_fail(e, "export maps");
    return LBW_OK;
}

int lbw_stability_bound(lbw_geometry_t g, double* c_max) {
    if (!g || !c_max) return fail(LBW_EINVAL, "NULL argument");
    std::vector<double> t((size_t)(g->general ? lbw::kGenF64 : lbw::kTabF64) * g->E);
    HIP_TRY(hipMemcpyAsync(t.data(), g->tab64, sizeof(double) * t.size(), hipMemcpyDeviceToHost, g->stream),
            "stability bound");
    HIP_TRY(hipStreamSynchronize(g->stream), "stability bound");
    const int64_t E = g->E;
    double worst = 0.0;
    for (int64_t e = 0; e < E; ++e) {
        double tot = 0.0;
        for (int a = 0; a < g->d.dim; ++a) {
            double m = t[a * E + e];
            if (g->general) {
                // off-diagonal planes 01 (3), 02 (4), 12 (5) touching axis a
                m += a == 0 ? std::fabs(t[3 * E + e]) + std::fabs(t[4 * E + e])
                     : a == 1 ? std::fabs(t[3 * E + e]) + std::fabs(t[5 * E + e])
                              : std::fabs(t[4 * E + e]) + std::fabs(t[5 * E + e]);
            } else if (g->d.dim == 3 && a != 1) {
                m += std::fabs(t[3 * E + e]);
            }
            tot += m <= 1.0 ? 4.0 : (1.0 + m) * (1.0 + m) / m;
        }
        worst = std::fmax(worst, tot);
    }
    *c_max = 2.0 / std::sqrt(worst);
    return LBW_OK;
}

int lbw_set_step_config(lbw_geometry_t g, int tile_x, int tile_y, int chunk_z, int blocks) {
    if (!g) return fail(LBW_EINVAL, "geometry is NULL");
    if (g->dev.dim != 3) return fail(LBW_EINVAL, "step configuration applies to 3-D geometries");
    if (g->general) {
        // general kernel: tiles 32 x 8, 64 x 4 (256 threads) or 64 x 8 (512), one workgroup per tile
        if (!((tile_x == 32 && tile_y == 8) || (tile_x == 64 && (tile_y == 4 || tile_y == 8))) || chunk_z < 1 ||
            blocks != 0)
            return fail(LBW_EINVAL, "geometry given by its metric: tile 32 x 8, 64 x 4 or 64 x 8, chunk_z >= 1, blocks 0");
        g->plan = lbw::make_march_plan(g->dev, tile_x, tile_y, chunk_z, 8);
        g->plan.blocks = (int)g->plan.tiles;
        g->plan_version += 1;
        return LBW_OK;
    }
    if (!lbw::march_shape_ok(tile_x, tile_y))
        return fail(LBW_EINVAL,
                    "tile %d x %d: tile_x must be 16, 32 or 64 with tile_x * tile_y 256 or 512, or the tile "
                    "96 x 4, 96 x 8, 128 x 4 or 128 x 8",
                    tile_x, tile_y);
    if (chunk_z < 1 || blocks < 0) return fail(LBW_EINVAL, "chunk_z must be >= 1 and blocks >= 0");
    if (blocks == 0) {
        int dev = 0, cus = 0;
        HIP_TRY(hipGetDevice(&dev), "lbw_set_step_config");
        HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "lbw_set_step_config");
        blocks = cus * lbw::march_blocks_per_cu(tile_x, tile_y);
    }
    g->plan = lbw::make_march_plan(g->dev, tile_x, tile_y, chunk_z, blocks);
    g->use2 = false;
    g->plan_version += 1;
    return LBW_OK;
}

int lbw_set_step2_config(lbw_geometry_t g, int tile_x, int tile_y, int chunk_z, int blocks) {
    if (!g) return fail(LBW_EINVAL, "geometry is NULL");
    if (tile_x == 0) {
        g->use2 = false;
        g->plan_version += 1;
        return LBW_OK;
    }
    if (g->dev.dim != 3 || g->general) return fail(LBW_EINVAL, "two-step launches apply to built-in 3-D geometries");
    if (!lbw::march2_shape_ok(tile_x, tile_y))
        return fail(LBW_EINVAL, "two-step tile %d x %d: must be 96 x 6 or 128 x 4", tile_x, tile_y);
    if (!lbw::march2_fits(g->dev, tile_x))
        return fail(LBW_EINVAL, "two-step tile of %d lanes: needs n0 <= %d (n0 = %d) and a walled axis 0", tile_x,
                    tile_x, g->dev.n0);
    if (chunk_z < 0 || blocks < 0) return fail(LBW_EINVAL, "chunk_z must be >= 0 (0: balanced) and blocks >= 0");
    if (blocks == 0) {
        int cus = 0;
        if (lbw::device_cus(&cus) != LBW_OK) return LBW_EDEVICE;
        blocks = cus * lbw::march2_blocks_per_cu(tile_x, tile_y);
    }
    g->plan2 = lbw::make_march2_plan(g->dev, tile_x, tile_y, chunk_z, blocks);
    g->use2 = true;
    g->plan_version += 1;
    return LBW_OK;
}

int lbw_get_step2_config(lbw_geometry_t g, int* tile_x, int* tile_y, int* chunk_z, int* blocks) {
    if (!g) return fail(LBW_EINVAL, "geometry is NULL");
    if (tile_x) *tile_x = g->use2 ? g->plan2.tx : 0;
    if (tile_y) *tile_y = g->use2 ? g->plan2.ty : 0;
    if (chunk_z) *chunk_z = g->use2 ? g->plan2.lz : 0;
    if (blocks) *blocks = g->use2 ? g->plan2.blocks : 0;
    return LBW_OK;
}

int lbw_get_step_config(lbw_geometry_t g, int* tile_x, int* tile_y, int* chunk_z, int* blocks) {
    if (!g) return fail(LBW_EINVAL, "geometry is NULL");
    if (g->dev.dim != 3) return fail(LBW_EINVAL, "step configuration applies to 3-D geometries");
    if (tile_x) *tile_x = g->plan.tx;
    if (tile_y) *tile_y = g->plan.ty;
    if (chunk_z) *chunk_z = g->plan.lz;
    if (blocks) *blocks = g->plan.blocks;
    return LBW_OK;
}

int lbw_init(lbw_geometry_t g, const double* p0, float* f_a, float* f_b, const int64_t* probes, int n_probes,
             double* trace, int64_t t_max, void* stream, lbw_state_t* out) {
    if (!out) return fail(LBW_EINVAL, "out is NULL");
    *out = nullptr;
    if (!g || !p0 || !f_a || !f_b) return fail(LBW_EINVAL, "NULL argument");
    if (f_a == f_b) return fail(LBW_EINVAL, "f_a and f_b must be distinct");
    if (n_probes < 0 || t_max < 0) return fail(LBW_EINVAL, "negative n_probes or t_max");
    if (n_probes > 0 && (!probes || (!trace && t_max > 0))) return fail(LBW_EINVAL, "probes need a trace buffer");
    for (int p = 0; p < n_probes; ++p)
        if (probes[p] < 0 || probes[p] >= g->N) return fail(LBW_EINVAL, "probe %d out of range", p);
    lbw_state* s = new lbw_state();
    s->g = g;
    s->f[0] = f_a;
    s->f[1] = f_b;
    s->t_max = n_probes > 0 ? t_max : 0;
    s->n_probes = n_probes;
    s->trace = trace;
    s->stream = (hipStream_t)stream;
    s->probes_host.assign(probes, probes + n_probes);
    hipError_t e = hipMalloc(&s->d_tcount, sizeof(int64_t));
    if (e == hipSuccess) e = hipMalloc(&s->d_scratch_count, sizeof(int64_t));
    if (e == hipSuccess) e = hipMalloc(&s->d_done, 2 * sizeof(unsigned));
    if (e == hipSuccess) e = hipMemsetAsync(s->d_done, 0, 2 * sizeof(unsigned), s->stream);
    if (e == hipSuccess && n_probes > 0) e = hipMalloc(&s->d_probes, sizeof(int64_t) * n_probes);
    if (e == hipSuccess && n_probes > 0)
        e = hipMemcpyAsync(s->d_probes, probes, sizeof(int64_t) * n_probes, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->d_tcount, 0, sizeof(int64_t), s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->d_scratch_count, 0, sizeof(int64_t), s->stream);
    if (e == hipSuccess && s->stream != g->stream) e = hipStreamSynchronize(g->stream);
    if (e == hipSuccess) e = lbw::launch_init(g->dev, p0, f_a, s->stream);
    if (e == hipSuccess && n_probes > 0) e = hipStreamSynchronize(s->stream);  // host probe list may go away
    if (e != hipSuccess) {
        (void)hipFree(s->d_tcount);
        (void)hipFree(s->d_scratch_count);
        (void)hipFree(s->d_done);
        (void)hipFree(s->d_probes);
        delete s;
        return hip_fail(e, "lbw_init");
    }
    *out = s;
    return LBW_OK;
}

namespace {

hipError_t launch_one(lbw_state* s, const lbw::ProbeArgs& pr, int from, hipStream_t st) {
    if (s->n_src > 0) {
        const hipError_t e = lbw::launch_sources(s->d_src, s->n_src, s->d_tcount, s->f[from], st);
        if (e != hipSuccess) return e;
    }
    if (s->g->general)
        return lbw::launch_step_general(s->g->dev, pr, s->g->plan, s->f[from], s->f[1 - from], st);
    if (s->g->dev.dim == 3)
        return lbw::launch_step_march(s->g->dev, pr, s->g->plan, s->f[from], s->f[1 - from], st);
    return lbw::launch_step(s->g->dev, pr, s->f[from], s->f[1 - from], st);
}

// The two-step pass applies: chosen for the geometry, no driven sources
// (they are imposed between steps), and no tile of the pass holds more
// probes than it records.
bool two_step_ok(const lbw_state* s) {
    const lbw_geometry* g = s->g;
    if (!g->use2 || g->general || g->dev.dim != 3 || s->n_src > 0 || !lbw::march2_fits(g->dev, g->plan2.tx))
        return false;
    if (s->n_probes == 0 || s->t >= s->t_max) return true;
    std::map<int64_t, int> per_tile;
    const int64_t n0 = g->dev.n0, n1 = g->dev.n1;
    const lbw::MarchPlan& p = g->plan2;
    for (int64_t node : s->probes_host) {
        const int64_t i1 = (node / n0) % n1, i2 = node / (n0 * n1);
        int64_t tile;
        if (p.lz > 0) {
            tile = i1 / p.ty + (int64_t)p.nty * (i2 / p.lz);
        } else {
            // balanced plan: one segment per (workgroup, row tile); the
            // workgroup is the one whose share holds the probe's pair
            const int64_t pair = (i1 / p.ty) * (int64_t)g->dev.n2 + i2;
            int64_t owner = -1;
            for (int b = 0; b < p.blocks && owner < 0; ++b) {
                int64_t a = 0, e = 0;
                lbw::march2_share(p.tiles, p.blocks, b, &a, &e);
                if (pair >= a && pair < e) owner = b;
            }
            tile = owner * (int64_t)p.nty + i1 / p.ty;
        }
        if (++per_tile[tile] > lbw::march2_tile_probes()) return false;
    }
    return true;
}

hipError_t launch_two(lbw_state* s, int from, hipStream_t st) {
    lbw::ProbeArgs pr{s->d_probes, s->n_probes, s->trace, s->t_max, s->d_tcount, s->d_done};
    return lbw::launch_step_march2(s->g->dev, pr, s->g->plan2, s->f[from], s->f[1 - from], st);
}

void drop_graphs(lbw_state* s) {
    for (auto& gx : s->graph) {
        if (gx) (void)hipGraphExecDestroy(gx);
        gx = nullptr;
    }
}

// Captures graph_block steps (one-step launches, or graph_block / 2
// two-step launches when two) starting from buffer `from` on a private
// stream (capture only records; nothing runs there).
hipError_t build_graph(lbw_state* s, int from, bool two) {
    hipStream_t cap = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    lbw::ProbeArgs pr{s->d_probes, s->n_probes, s->trace, s->t_max, s->d_tcount};
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        int cur = from;
        hipError_t le = hipSuccess;
        const int launches = two ? s->graph_block / 2 : s->graph_block;
        for (int i = 0; i < launches && le == hipSuccess; ++i) {
            le = two ? launch_two(s, cur, cap) : launch_one(s, pr, cur, cap);
            cur ^= 1;
        }
        e = hipStreamEndCapture(cap, &graph);
        if (e == hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&s->graph[from], graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cap);
    return e;
}

}  // namespace

int lbw_step_n(lbw_state_t s, int64_t n) {
    if (!s) return fail(LBW_EINVAL, "state is NULL");
    if (n < 0) return fail(LBW_EINVAL, "negative step count");
    lbw::ProbeArgs pr{s->d_probes, s->n_probes, s->trace, s->t_max, s->d_tcount, s->d_done};
    const bool two = two_step_ok(s);
    // steps per captured block: even for two-step launches
    const int K = two ? s->graph_block & ~1 : s->graph_block;
    if (K > 0 && n >= K) {
        if (s->graph_version != s->g->plan_version || s->graph_two != two) {
            drop_graphs(s);
            s->graph_version = s->g->plan_version;
            s->graph_two = two;
        }
        const int launches = two ? K / 2 : K;
        while (n >= K) {
            if (!s->graph[s->cur]) HIP_TRY(build_graph(s, s->cur, two), "lbw_step_n: graph capture");
            HIP_TRY(hipGraphLaunch(s->graph[s->cur], s->stream), "lbw_step_n: graph launch");
            if (launches & 1) s->cur ^= 1;
            s->t += K;
            n -= K;
        }
    }
    while (two && n >= 2) {
        HIP_TRY(launch_two(s, s->cur, s->stream), "lbw_step_n");
        s->cur ^= 1;
        s->t += 2;
        n -= 2;
    }
    for (int64_t i = 0; i < n; ++i) {
        HIP_TRY(launch_one(s, pr, s->cur, s->stream), "lbw_step_n");
        s->cur ^= 1;
        s->t += 1;
    }
    return LBW_OK;
}

int lbw_set_graph_block(lbw_state_t s, int steps) {
    if (!s) return fail(LBW_EINVAL, "state is NULL");
    if (steps < 0 || steps > 4096) return fail(LBW_EINVAL, "graph block must be in [0, 4096]");
    HIP_TRY(hipStreamSynchronize(s->stream), "lbw_set_graph_block");
    drop_graphs(s);
    s->graph_block = steps;
    return LBW_OK;
}

int lbw_autotune(lbw_state_t s, int reps, double* best_us) {
    if (!s) return fail(LBW_EINVAL, "state is NULL");
    if (reps < 1) return fail(LBW_EINVAL, "reps must be >= 1");
    lbw_geometry* g = s->g;
    if (g->dev.dim != 3 || g->general) return fail(LBW_EINVAL, "autotune applies to built-in 3-D geometries");
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev), "lbw_autotune");
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "lbw_autotune");
    // Candidates are timed on real ping-pong traffic: the first launch reads
    // the current buffer and writes the state's other buffer, later launches
    // alternate between that buffer and a temporary one, so every launch
    // reads what the previous one wrote (as lbw_step_n does) and the current
    // buffer is never written.
    float* tmp = nullptr;
    HIP_TRY(hipMalloc((void**)&tmp, sizeof(float) * g->Q * g->N), "lbw_autotune");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    // Candidates are timed with the state's own probes recorded into a
    // scratch trace (the two-step kernel records its probes inside the tiles
    // that hold them, which is part of its cost); the timing step counter
    // restarts at 0 for each candidate, so every timed launch records.
    const int64_t trows = 6 * (int64_t)reps + 8;  // rows of a candidate's 3 reps + 3 launches, two steps each
    double* ptrace = nullptr;
    if (err == hipSuccess && s->n_probes > 0)
        err = hipMalloc((void**)&ptrace, sizeof(double) * (size_t)trows * (size_t)s->n_probes);
    const int np = ptrace ? s->n_probes : 0;
    lbw::ProbeArgs pr{np ? s->d_probes : nullptr, np, ptrace, np ? trows : 0, s->d_scratch_count};
    auto restart = [&]() {
        if (err == hipSuccess) err = hipMemsetAsync(s->d_scratch_count, 0, sizeof(int64_t), s->stream);
    };
    const lbw::MarchPlan keep = g->plan;
    lbw::MarchPlan best = keep;
    float best_ms = 1e30f;
    float* other = s->f[1 - s->cur];
    // One candidate timed: a launch from the current buffer, two more, then
    // `count` timed launches on the ping-pong pair; milliseconds for them.
    auto time1 = [&](const lbw::MarchPlan& p, int count) -> float {
        float* bufs[2] = {other, tmp};
        int w = 0;
        auto run = [&](int n) {
            for (int r = 0; r < n && err == hipSuccess; ++r, w ^= 1)
                err = lbw::launch_step_march(g->dev, pr, p, bufs[w], bufs[w ^ 1], s->stream);
        };
        restart();
        if (err == hipSuccess) err = lbw::launch_step_march(g->dev, pr, p, s->f[s->cur], other, s->stream);
        run(2);
        if (err == hipSuccess) err = hipEventRecord(e0, s->stream);
        run(count);
        if (err == hipSuccess) err = hipEventRecord(e1, s->stream);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        return ms;
    };
    // two time steps per launch: timed per step (reps launches = 2 reps
    // steps), on the same ping-pong buffers with the timing step counter
    // and its own completion counter
    const lbw::ProbeArgs pr2{pr.nodes, pr.n, pr.trace, pr.t_max, s->d_scratch_count, s->d_done + 1};
    auto time2 = [&](const lbw::MarchPlan& p, int count) -> float {
        float* bufs[2] = {other, tmp};
        int w = 0;
        auto run = [&](int n) {
            for (int r = 0; r < n && err == hipSuccess; ++r, w ^= 1)
                err = lbw::launch_step_march2(g->dev, pr2, p, bufs[w], bufs[w ^ 1], s->stream);
        };
        restart();
        if (err == hipSuccess) err = lbw::launch_step_march2(g->dev, pr2, p, s->f[s->cur], other, s->stream);
        run(2);
        if (err == hipSuccess) err = hipEventRecord(e0, s->stream);
        run(count);
        if (err == hipSuccess) err = hipEventRecord(e1, s->stream);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        return ms;
    };
    std::vector<std::pair<float, lbw::MarchPlan>> cand1, cand2;
    for (int nt : {256, 384, 512, 768, 1024})
    for (int tx : {16, 32, 64, 96, 128}) {
        if (err != hipSuccess) break;
        const int ty = nt / tx;
        if (!lbw::march_shape_ok(tx, ty)) continue;
        const int bpc = lbw::march_blocks_per_cu(tx, ty);
        for (int lz : {4, 8, 16, 32, 64}) {
            if (lz > 2 * g->dev.n2 && lz != 4) continue;
            for (int mult : {1, 2}) {
                const lbw::MarchPlan p = lbw::make_march_plan(g->dev, tx, ty, lz, mult * cus * bpc);
                const float ms = time1(p, reps);
                if (err != hipSuccess) break;
                cand1.push_back({ms, p});
            }
        }
    }
    for (int tx : {96, 128}) {
        const int ty = tx == 96 ? 6 : 4;
        if (err != hipSuccess || !lbw::march2_fits(g->dev, tx)) continue;
        const int bpc = lbw::march2_blocks_per_cu(tx, ty);
        // chunk lengths: besides the plain ones, those whose tile count
        // fills whole waves of resident workgroups (tiles of equal work)
        std::vector<int> lzs{0, 8, 12, 16, 20, 24, 32, 40, 48, 64};  // 0: balanced shares
        for (int waves = 1; waves <= 8; ++waves) {
            const int nty = (g->dev.n1 + ty - 1) / ty;
            const int64_t want = (int64_t)waves * cus * bpc;  // tiles
            if (want % nty) continue;
            const int64_t chunks = want / nty;
            const int lz = (int)((g->dev.n2 + chunks - 1) / chunks);
            if (lz >= 4 && std::find(lzs.begin(), lzs.end(), lz) == lzs.end()) lzs.push_back(lz);
        }
        for (int lz : lzs) {
            if (lz > 2 * g->dev.n2 && lz != 8) continue;
            for (int mult : {1, 2}) {
                const lbw::MarchPlan p = lbw::make_march2_plan(g->dev, tx, ty, lz, mult * cus * bpc);
                const float ms = time2(p, reps);
                if (err != hipSuccess) break;
                cand2.push_back({ms, p});
            }
        }
    }
    // The fastest three of each kind timed again over three times the
    // launches (close candidates timed once can swap places from run to
    // run); times per reps launches.
    auto pick = [&](std::vector<std::pair<float, lbw::MarchPlan>>& c, auto timer, lbw::MarchPlan& bp, float& bms) {
        std::sort(c.begin(), c.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
        for (size_t i = 0; i < c.size() && i < 3 && err == hipSuccess; ++i) {
            const float ms = timer(c[i].second, 3 * reps) / 3.f;
            if (err == hipSuccess && ms < bms) {
                bms = ms;
                bp = c[i].second;
            }
        }
    };
    lbw::MarchPlan best2{};
    float best2_ms = 1e30f;  // per 2 reps steps
    pick(cand1, time1, best, best_ms);
    pick(cand2, time2, best2, best2_ms);
    // the best shape with the other store policy (non-temporal stores pay on
    // grids that do not fit the caches, and cost where they do)
    if (err == hipSuccess) {
        lbw::MarchPlan p = best;
        p.nts = !p.nts;
        const float ms = time1(p, 3 * reps) / 3.f;
        if (err == hipSuccess && ms < best_ms) {
            best_ms = ms;
            best = p;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s->stream);
    (void)hipFree(tmp);
    if (ptrace) (void)hipFree(ptrace);
    g->plan = err == hipSuccess ? best : keep;
    const bool two = err == hipSuccess && best2_ms < 2.f * best_ms;
    g->use2 = two;
    if (two) g->plan2 = best2;
    g->plan_version += 1;
    if (err != hipSuccess) return hip_fail(err, "lbw_autotune");
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[std::make_tuple(g->dev.n0, g->dev.n1, g->dev.n2)] =
            Tuned{best.tx, best.ty, best.lz, best.blocks, best.nts, two ? best2.tx : 0, best2.ty, best2.lz,
                  best2.blocks};
    }
    if (best_us) *best_us = two ? 1e3 * best2_ms / (2 * reps) : 1e3 * best_ms / reps;
    return LBW_OK;
}

int lbw_probe(lbw_state_t s, double* host_dst, int64_t t0, int64_t t1) {
    if (!s || !host_dst) return fail(LBW_EINVAL, "NULL argument");
    const int64_t rows = s->t < s->t_max ? s->t : s->t_max;
    if (t0 < 0 || t1 < t0 || t1 > rows) return fail(LBW_EINVAL, "rows [%lld, %lld) outside [0, %lld)",
                                                    (long long)t0, (long long)t1, (long long)rows);
    const size_t cnt = (size_t)(t1 - t0) * s->n_probes;
    if (cnt) {
        HIP_TRY(hipMemcpyAsync(host_dst, s->trace + t0 * s->n_probes, cnt * sizeof(double), hipMemcpyDeviceToHost,
                               s->stream),
                "lbw_probe");
    }
    HIP_TRY(hipStreamSynchronize(s->stream), "lbw_probe");
    for (size_t i = 0; i < cnt; ++i)
        if (!std::isfinite(host_dst[i])) return fail(LBW_EUNSTABLE, "non-finite probe value at row %lld",
                                                     (long long)(t0 + i / s->n_probes));
    return LBW_OK;
}

int lbw_modes(lbw_state_t s, int k, double* freq_out, double* power_out) {
    if (!s || !freq_out) return fail(LBW_EINVAL, "NULL argument");
    if (k < 1) return fail(LBW_EINVAL, "k must be >= 1");
    if (s->n_probes < 1) return fail(LBW_EINVAL, "state has no probes");
    const int64_t T = s->t < s->t_max ? s->t : s->t_max;
    if (T < 8) return fail(LBW_EINVAL, "need at least 8 recorded rows (have %lld)", (long long)T);
    if (s->n_probes > lbw::modes_max_cols(T)) return fail(LBW_EINVAL, "too many probes for one spectrum");
    const size_t need = lbw::modes_work_bytes(T, s->n_probes, 1);
    if (need > s->mode_work_bytes) {
        (void)hipFree(s->mode_work);
        s->mode_work = nullptr;
        s->mode_work_bytes = 0;
        HIP_TRY(hipMalloc(&s->mode_work, need), "lbw_modes");
        s->mode_work_bytes = need;
    }
    if (k > s->mode_k) {
        (void)hipFree(s->mode_out);
        s->mode_out = nullptr;
        s->mode_k = 0;
        HIP_TRY(hipMalloc(&s->mode_out, sizeof(double) * 2 * k), "lbw_modes");
        s->mode_k = k;
    }
    const int ncols = s->n_probes;
    HIP_TRY(lbw::launch_modes_grouped(s->trace, T, s->n_probes, &ncols, 1, k, s->mode_work, s->mode_work_bytes,
                                      s->mode_out, s->mode_out + k, s->stream),
            "lbw_modes");
    std::vector<double> host(2 * (size_t)k);
    HIP_TRY(hipMemcpyAsync(host.data(), s->mode_out, sizeof(double) * 2 * k, hipMemcpyDeviceToHost, s->stream),
            "lbw_modes");
    HIP_TRY(hipStreamSynchronize(s->stream), "lbw_modes");
    for (int i = 0; i < k; ++i) {
        freq_out[i] = host[i];
        if (power_out) power_out[i] = host[k + i];
    }
    return LBW_OK;
}

int lbw_modes_noalloc(lbw_state_t s, int k, double* freq_dev, double* power_dev) {
    if (!s || !freq_dev || !power_dev) return fail(LBW_EINVAL, "NULL argument");
    if (k < 1) return fail(LBW_EINVAL, "k must be >= 1");
    if (s->n_probes < 1) return fail(LBW_EINVAL, "state has no probes");
    const int64_t T = s->t < s->t_max ? s->t : s->t_max;
    if (T < 8) return fail(LBW_EINVAL, "need at least 8 recorded rows (have %lld)", (long long)T);
    if (lbw::modes_static_cols(T) < 1)
        return fail(LBW_EINVAL, "%lld recorded rows exceed the fixed %zu-byte work space (at most %lld rows)",
                    (long long)T, lbw::kModesScratchBytes, (long long)LBW_MODES_NOALLOC_MAX_ROWS);
    void* scratch = nullptr;
    HIP_TRY(lbw::modes_scratch(&scratch), "lbw_modes_noalloc: work space address");
    HIP_TRY(lbw::launch_modes_static(scratch, s->trace, T, s->n_probes, s->n_probes, k, freq_dev, power_dev,
                                     s->stream),
            "lbw_modes_noalloc");
    return LBW_OK;
}

int lbw_set_sources(lbw_state_t s, const int64_t* nodes, int n, double amplitude, double omega, int kind) {
    if (!s) return fail(LBW_EINVAL, "state is NULL");
    if (n < 0 || (n > 0 && !nodes)) return fail(LBW_EINVAL, "invalid source list");
    if (!std::isfinite(amplitude) || !std::isfinite(omega)) return fail(LBW_EINVAL, "non-finite amplitude or omega");
    lbw_geometry* g = s->g;
    if (kind < 0 || kind > g->dev.dim) return fail(LBW_EINVAL, "source kind %d outside [0, %d]", kind, g->dev.dim);
    for (int i = 0; i < n; ++i)
        if (nodes[i] < 0 || nodes[i] >= g->N) return fail(LBW_EINVAL, "source %d outside the grid", i);
    // sqrt(g) per (i0, i2) entry (FP64 table plane 7) or per node (plane 9)
    std::vector<double> sg(n > 0 ? (size_t)g->E : 0);
    if (n > 0)
        HIP_TRY(hipMemcpyAsync(sg.data(), g->tab64 + (g->general ? 9 : 7) * g->E, sizeof(double) * g->E,
                               hipMemcpyDeviceToHost, s->stream),
                "lbw_set_sources");
    HIP_TRY(hipStreamSynchronize(s->stream), "lbw_set_sources");
    const int d = g->dev.dim;
    const double c2 = g->dev.c2_64;
    const int64_t n0 = g->dev.n0, plane = n0 * g->dev.n1;
    std::vector<lbw::SourceEntry> host((size_t)n);
    for (int i = 0; i < n; ++i) {
        const int64_t node = nodes[i];
        const double sq = sg[(size_t)(g->general ? node : node % n0 + n0 * (node / plane))];
        lbw::SourceEntry e{};
        e.f_off = (uint64_t)node;
        e.N = (uint32_t)g->N;
        e.q = g->Q;
        e.counter = 0;
        e.kind = kind;
        e.a0 = kind ? amplitude * 0.5 * sq : amplitude * (1.0 - d * c2) * sq;
        e.a1 = kind ? 0.5 * c2 : amplitude * 0.5 * c2 * sq;
        e.omega = omega;
        host[(size_t)i] = e;
    }
    drop_graphs(s);
    (void)hipFree(s->d_src);
    s->d_src = nullptr;
    s->n_src = 0;
    if (n > 0) {
        HIP_TRY(hipMalloc((void**)&s->d_src, sizeof(lbw::SourceEntry) * n), "lbw_set_sources");
        HIP_TRY(hipMemcpyAsync(s->d_src, host.data(), sizeof(lbw::SourceEntry) * n, hipMemcpyHostToDevice, s->stream),
                "lbw_set_sources");
        HIP_TRY(hipStreamSynchronize(s->stream), "lbw_set_sources");
        s->n_src = n;
    }
    return LBW_OK;
}

int lbw_amplitude(lbw_state_t s, int64_t t0, int64_t t1, double* out) {
    if (!s || !out) return fail(LBW_EINVAL, "NULL argument");
    if (s->n_probes < 1) return fail(LBW_EINVAL, "state has no probes");
    const int64_t rows = s->t < s->t_max ? s->t : s->t_max;
    if (t0 < 0 || t1 <= t0 || t1 > rows)
        return fail(LBW_EINVAL, "rows [%lld, %lld) empty or outside [0, %lld)", (long long)t0, (long long)t1,
                    (long long)rows);
    if (!s->d_amp) HIP_TRY(hipMalloc((void**)&s->d_amp, sizeof(double) * s->n_probes), "lbw_amplitude");
    HIP_TRY(lbw::launch_amplitude(s->trace, s->n_probes, s->n_probes, t0, t1, s->d_amp, s->stream), "lbw_amplitude");
    HIP_TRY(hipMemcpyAsync(out, s->d_amp, sizeof(double) * s->n_probes, hipMemcpyDeviceToHost, s->stream),
            "lbw_amplitude");
    HIP_TRY(hipStreamSynchronize(s->stream), "lbw_amplitude");
    for (int p = 0; p < s->n_probes; ++p)
        if (!std::isfinite(out[p])) return fail(LBW_EUNSTABLE, "non-finite value at probe %d", p);
    return LBW_OK;
}

int lbw_state_info(lbw_state_t s, int64_t* t, float** f_current) {
    if (!s) return fail(LBW_EINVAL, "state is NULL");
    if (t) *t = s->t;
    if (f_current) *f_current = s->f[s->cur];
    return LBW_OK;
}

int lbw_pressure(lbw_state_t s, double* p_out) {
    if (!s || !p_out) return fail(LBW_EINVAL, "NULL argument");
    HIP_TRY(lbw::launch_pressure(s->g->dev, s->f[s->cur], p_out, s->stream), "lbw_pressure");
    return LBW_OK;
}

int lbw_free_state(lbw_state_t s) {
    if (!s) return LBW_OK;
    (void)hipStreamSynchronize(s->stream);
    drop_graphs(s);
    (void)hipFree(s->d_scratch_count);
    (void)hipFree(s->d_done);
    (void)hipFree(s->d_tcount);
    (void)hipFree(s->d_probes);
    (void)hipFree(s->d_src);
    (void)hipFree(s->d_amp);
    (void)hipFree(s->mode_work);
    (void)hipFree(s->mode_out);
    delete s;
    return LBW_OK;
}

}  // extern "C"
