// C-ABI for batches of D3Q7 geometries advanced by one launch per step.
#include <algorithm>
#include <cmath>
#include <map>
#include <utility>
#include <vector>

#include "host_util.h"

using lbw::fail;
using lbw::hip_fail;

struct lbw_batch {
    int n = 0;
    std::vector<lbw_geometry_desc> d;
    std::vector<int64_t> node_off, probe_off, rec_off, tab64_off;  // prefix sums, n + 1 entries
    double* tab64 = nullptr;
    float* tab32 = nullptr;
    std::vector<lbw::BatchItem> items;
    lbw::BatchItem* d_items = nullptr;
    std::vector<int32_t> tile_item;     // geometry of every tile of the current plan
    int32_t* d_tile_item = nullptr;
    int64_t tile_item_cap = 0;          // entries allocated at d_tile_item
    int tx = 32, lz = 16, blocks = 8;
    int section_nt = 0;  // > 0: whole-row tiles of this many threads (tx unused)
    bool nts = false;    // non-temporal population stores (default: the buffers exceed the Infinity Cache)
    bool pery = false;   // every geometry periodic along axis 1 (the step variant without its wall rules)
    int64_t tiles = 0;
    int plan_version = 0;
    float* f[2] = {nullptr, nullptr};
    int cur = 0;
    int64_t t = 0, t_max = 0;
    int64_t P = 0;  // total probes
    double* trace = nullptr;
    int64_t* d_nodes = nullptr;
    int64_t* d_tcount = nullptr;
    int64_t* d_scratch_count = nullptr;
    hipStream_t stream = nullptr;
    int graph_block = 32;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int graph_version = -1;
    double* mode_work = nullptr;
    size_t mode_work_bytes = 0;
    double* mode_out = nullptr;
    int mode_k = 0;
    // driven nodes, imposed by the step kernel as it loads them: all
    // geometries' entries, and per geometry with driven nodes a map from each
    // node of its driven planes to its entry (or -1); per geometry the count,
    // the first and last driven plane and the map offset
    lbw::BatchSource* d_src = nullptr;
    int32_t* d_src_map = nullptr;
    int n_src = 0;
    // or, where driven nodes span many planes, imposed by a launch of their
    // own before every step (one entry per driven node)
    lbw::SourceEntry* d_entries = nullptr;
    int n_entries = 0;
    std::vector<int> src_count, src_zlo, src_zhi;
    std::vector<uint32_t> src_map_off;
    double* d_amp = nullptr;            // response intensities (P)
};

namespace {

constexpr int kXcdsBatch = 8;  // the batch kernel cuts its tile list into one range per XCD

void release(lbw_batch* b) {
    for (auto& gx : b->graph)
        if (gx) (void)hipGraphExecDestroy(gx);
    (void)hipFree(b->tab64);
    (void)hipFree(b->tab32);
    (void)hipFree(b->d_items);
    (void)hipFree(b->d_tile_item);
    (void)hipFree(b->d_nodes);
    (void)hipFree(b->d_tcount);
    (void)hipFree(b->d_scratch_count);
    (void)hipFree(b->mode_work);
    (void)hipFree(b->mode_out);
    (void)hipFree(b->d_src);
    (void)hipFree(b->d_src_map);
    (void)hipFree(b->d_entries);
    (void)hipFree(b->d_amp);
    delete b;
}

// Tile list for the current (tx, lz), uploaded to d_items.  The stream is
// drained before the host table is rewritten and after the copy: kernels
// already queued read d_items when they run, and their tile count is a
// launch argument, so the device table must not change under them and the
// (pageable) host table must not change while a copy from it is pending.
hipError_t build_items(lbw_batch* b) {
    hipError_t e0 = hipStreamSynchronize(b->stream);
    if (e0 != hipSuccess) return e0;
    const int ty = b->section_nt ? 1 : 256 / b->tx;
    int64_t tile = 0;
    for (int h = 0; h < b->n; ++h) {
        const lbw_geometry_desc& d = b->d[h];
        const lbw::GeomDev v = lbw::make_geomdev(d, nullptr, nullptr);
        lbw::BatchItem& it = b->items[h];
        it.n0 = v.n0;
        it.n1 = v.n1;
        it.n2 = v.n2;
        it.N = (uint32_t)v.N;
        for (int a = 0; a < 3; ++a) {
            it.bc_lo[a] = v.bc_lo[a];
            it.bc_hi[a] = v.bc_hi[a];
        }
        it.c2 = v.c2;
        it.two_w0 = v.two_w0;
        it.damp = v.damp;
        it.rty = b->section_nt ? lbw::batch_row_tile(v.n0, v.n1, b->section_nt) : 0;
        it.ntx = b->section_nt ? 1 : (v.n0 + b->tx - 1) / b->tx;
        it.nty = b->section_nt ? (v.n1 + it.rty - 1) / it.rty : (v.n1 + ty - 1) / ty;
        it.lz = b->lz;
        const int nchunks = (v.n2 + b->lz - 1) / b->lz;
        it.tile_begin = tile;
        it.tiles = (int64_t)it.ntx * it.nty * nchunks;
        tile += it.tiles;
        it.f_off = (uint64_t)(7 * b->node_off[h]);
        it.tab_off = (uint32_t)b->rec_off[h];
        it.sg_off = (uint32_t)(b->tab64_off[h] + 7 * (b->rec_off[h + 1] - b->rec_off[h]));
        it.probe_off = (uint32_t)b->probe_off[h];
        it.n_probes = (int)(b->probe_off[h + 1] - b->probe_off[h]);
        it.src_count = b->src_count[h];
        it.src_zlo = b->src_zlo[h];
        it.src_zhi = b->src_zhi[h];
        it.src_map = b->src_map_off[h];
    }
    b->tiles = tile;
    b->plan_version += 1;
    // tile -> geometry table (the kernel reads one entry per tile instead of
    // searching the geometry list)
    b->tile_item.resize((size_t)tile);
    for (int h = 0; h < b->n; ++h)
        std::fill(b->tile_item.begin() + b->items[h].tile_begin,
                  b->tile_item.begin() + b->items[h].tile_begin + b->items[h].tiles, (int32_t)h);
    hipError_t e = hipSuccess;
    if (tile > b->tile_item_cap) {
        (void)hipFree(b->d_tile_item);
        b->d_tile_item = nullptr;
        b->tile_item_cap = 0;
        e = hipMalloc((void**)&b->d_tile_item, sizeof(int32_t) * (size_t)tile);
        if (e != hipSuccess) return e;
        b->tile_item_cap = tile;
    }
    e = hipMemcpyAsync(b->d_items, b->items.data(), sizeof(lbw::BatchItem) * b->n, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && tile > 0)
        e = hipMemcpyAsync(b->d_tile_item, b->tile_item.data(), sizeof(int32_t) * (size_t)tile,
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    return e;
}

lbw::BatchProbeArgs probe_args(lbw_batch* b, bool record) {
    lbw::BatchProbeArgs bp{};
    bp.nodes = b->d_nodes;
    bp.trace = b->trace;
    bp.stride = b->P;
    bp.t_max = record ? b->t_max : 0;
    bp.tcount = record ? b->d_tcount : b->d_scratch_count;
    bp.sqrtg = b->tab64;
    bp.tab4 = reinterpret_cast<const float4*>(b->tab32);
    bp.src = b->n_src > 0 ? b->d_src : nullptr;
    bp.src_map = b->n_src > 0 ? b->d_src_map : nullptr;
    return bp;
}

// One step.  The counter bank is the step's parity, which is that of the
// buffer read: b->cur flips with every step, from 0 at step 0.
hipError_t launch_batch(lbw_batch* b, lbw::BatchProbeArgs bp, const float* fin, float* fout, hipStream_t st) {
    bp.parity = fin == b->f[1] ? 1 : 0;
    if (b->n_entries > 0 && bp.tcount == b->d_tcount) {
        // sources imposed in memory before the step, at this step's time
        const hipError_t e = lbw::launch_sources(b->d_entries, b->n_entries, b->d_tcount + (size_t)bp.parity * b->n,
                                                 const_cast<float*>(fin), st);
        if (e != hipSuccess) return e;
    }
    return lbw::launch_step_batch(b->d_items, b->d_tile_item, b->n, b->tiles, b->tx, b->section_nt, b->blocks, b->nts,
                                  b->pery, bp, fin, fout, st);
}

hipError_t build_graph(lbw_batch* b, int from) {
    hipStream_t cap = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    const lbw::BatchProbeArgs bp = probe_args(b, true);
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        int cur = from;
        hipError_t le = hipSuccess;
        for (int i = 0; i < b->graph_block && le == hipSuccess; ++i) {
            le = launch_batch(b, bp, b->f[cur], b->f[1 - cur], cap);
            cur ^= 1;
        }
        e = hipStreamEndCapture(cap, &graph);
        if (e == hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->graph[from], graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cap);
    return e;
}

void drop_graphs(lbw_batch* b) {
    for (auto& gx : b->graph) {
        if (gx) (void)hipGraphExecDestroy(gx);
        gx = nullptr;
    }
}


// Lanes allotted over the whole batch by whole-row tiles of nt threads
// (0 if some geometry's rows do not fit them).
double row_slots(const lbw_batch* b, int nt) {
    double slots = 0.0;
    for (int h = 0; h < b->n; ++h) {
        const lbw_geometry_desc& d = b->d[h];
        const int r = lbw::batch_row_tile(d.n[0], d.n[1], nt);
        if (r == 0) return 0.0;
        slots += (double)nt * (double)((d.n[1] + r - 1) / r) * (double)d.n[2];
    }
    return slots;
}

// Workgroup size for whole-row tiles over the whole batch: the one of 128,
// 256 and 512 threads that leaves the fewest lanes idle (ties to the
// larger), or 0 if some geometry's rows fit none.
int section_threads(const lbw_batch* b) {
    int best = 0;
    double best_slots = 0.0;
    for (int nt : {512, 256, 128}) {
        const double sl = row_slots(b, nt);
        if (sl > 0.0 && (best == 0 || sl < best_slots)) {
            best = nt;
            best_slots = sl;
        }
    }
    return best;
}

// Lanes allotted over the whole batch: TX-wide tiles (tile_x > 0) or
// whole-row tiles (tile_x = 0).
double lane_slots(const lbw_batch* b, int tile_x) {
    if (tile_x == 0) return row_slots(b, section_threads(b));
    double slots = 0.0;
    for (int h = 0; h < b->n; ++h) {
        const lbw_geometry_desc& d = b->d[h];
        const int ty = 256 / tile_x;
        slots += (double)((d.n[0] + tile_x - 1) / tile_x * tile_x) * (double)((d.n[1] + ty - 1) / ty * ty) *
                 (double)d.n[2];
    }
    return slots;
}

// Tiles of the whole batch for TX-wide tiles (tile_x > 0) or whole-row
// tiles of nt threads (tile_x = 0) and chunks of lz planes.
int64_t batch_tiles(const lbw_batch* b, int tile_x, int nt, int lz) {
    int64_t tiles = 0;
    for (int h = 0; h < b->n; ++h) {
        const lbw_geometry_desc& d = b->d[h];
        int64_t per_plane;
        if (tile_x == 0) {
            const int r = lbw::batch_row_tile(d.n[0], d.n[1], nt);
            if (r == 0) return 0;
            per_plane = (d.n[1] + r - 1) / r;
        } else {
            const int ty = 256 / tile_x;
            per_plane = (int64_t)((d.n[0] + tile_x - 1) / tile_x) * ((d.n[1] + ty - 1) / ty);
        }
        tiles += per_plane * ((d.n[2] + lz - 1) / lz);
    }
    return tiles;
}

// Chunk lengths the tuner times: 4, 8, 16, 32, 64 and the four others with
// the lowest modelled cost, rounds x (lz + 2) plane steps.  rounds is the
// most tiles one of `blocks` persistent workgroups walks (the tiles are cut
// into one contiguous range per XCD, shared by that XCD's blocks) and the 2
// planes stand for a tile's prologue.  On small batches the fixed lengths can
// leave a last round in which most workgroups idle (476 pipes of 20 x 5 x
// 100 with chunks of 16: 3332 tiles on 1536 workgroups, 3 rounds where 2.2
// would do); the model finds the lengths that avoid it.
std::vector<int> lz_candidates(const lbw_batch* b, int tile_x, int nt, int blocks) {
    std::vector<int> out = {4, 8, 16, 32, 64};
    const int64_t per_xcd = blocks / kXcdsBatch > 0 ? blocks / kXcdsBatch : 1;
    std::vector<std::pair<double, int>> cost;
    for (int lz = 4; lz <= 64; ++lz) {
        const int64_t tiles = batch_tiles(b, tile_x, nt, lz);
        if (tiles == 0) return out;
        const int64_t per_range = (tiles + kXcdsBatch - 1) / kXcdsBatch;
        const int64_t rounds = (per_range + per_xcd - 1) / per_xcd;
        cost.emplace_back((double)rounds * (lz + 2), lz);
    }
    std::stable_sort(cost.begin(), cost.end(),
                     [](const std::pair<double, int>& x, const std::pair<double, int>& y) { return x.first < y.first; });
    int added = 0;
    for (const auto& c : cost) {
        if (added == 4) break;
        if (std::find(out.begin(), out.end(), c.second) == out.end()) {
            out.push_back(c.second);
            ++added;
        }
    }
    return out;
}

int set_config(lbw_batch* b, int tile_x, int chunk_z, int blocks) {
    int cus = 0;
    int rc = lbw::device_cus(&cus);
    if (rc) return rc;
    const int nt = tile_x == 0 ? section_threads(b) : 0;
    if (tile_x == 0 && nt == 0) return fail(LBW_EINVAL, "axis-0 rows too long for whole-row tiles");
    if (blocks == 0) blocks = cus * (nt ? lbw::batch_section_blocks_per_cu(nt) : lbw::batch_blocks_per_cu(tile_x));
    blocks = (blocks / 8) * 8;
    if (blocks < 8) blocks = 8;
    b->tx = tile_x;
    b->section_nt = nt;
    b->lz = chunk_z;
    b->blocks = blocks;
    HIP_TRY(build_items(b), "batch step configuration");
    return LBW_OK;
}

}  // namespace

extern "C" {

int lbw_batch_make(const lbw_geometry_desc* descs, int n, const double* p0, float* f_a, float* f_b,
                   const int64_t* probes, const int32_t* n_probes, double* trace, int64_t t_max, void* stream,
                   lbw_batch_t* out) {
    if (!out) return fail(LBW_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || !descs || !p0 || !f_a || !f_b || !n_probes) return fail(LBW_EINVAL, "invalid batch arguments");
    if (f_a == f_b) return fail(LBW_EINVAL, "f_a and f_b must be distinct");
    if (t_max < 0) return fail(LBW_EINVAL, "negative t_max");
    lbw_batch* b = new lbw_batch();
    b->n = n;
    b->stream = (hipStream_t)stream;
    b->node_off.assign(n + 1, 0);
    b->probe_off.assign(n + 1, 0);
    b->rec_off.assign(n + 1, 0);
    b->tab64_off.assign(n + 1, 0);
    for (int h = 0; h < n; ++h) {
        int rc = lbw::validate_desc(&descs[h]);
        if (rc) {
            delete b;
            return fail(rc, "geometry %d: %s", h, lbw_last_error());
        }
        if (descs[h].dim != 3 || descs[h].kind == LBW_GENERAL) {
            delete b;
            return fail(LBW_EINVAL, "geometry %d: batches hold built-in 3-D geometries", h);
        }
        if (n_probes[h] < 0) {
            delete b;
            return fail(LBW_EINVAL, "geometry %d: negative probe count", h);
        }
        b->d.push_back(lbw::normalised(descs[h]));
        const lbw_geometry_desc& d = b->d.back();
        const int64_t N = (int64_t)d.n[0] * d.n[1] * d.n[2];
        const int64_t E = (int64_t)d.n[0] * d.n[2];
        b->node_off[h + 1] = b->node_off[h] + N;
        b->probe_off[h + 1] = b->probe_off[h] + n_probes[h];
        b->rec_off[h + 1] = b->rec_off[h] + E;
        b->tab64_off[h + 1] = b->tab64_off[h] + lbw::kTabF64 * E;
    }
    b->P = b->probe_off[n];
    if (b->P > 0 && (!probes || (!trace && t_max > 0))) {
        delete b;
        return fail(LBW_EINVAL, "probes need a trace buffer");
    }
    if (b->rec_off[n] > 0xffffffffLL || b->tab64_off[n] > 0xffffffffLL) {
        delete b;
        return fail(LBW_EINVAL, "batch tables too large");
    }
    for (int h = 0; h < n; ++h) {
        const int64_t N = b->node_off[h + 1] - b->node_off[h];
        for (int64_t p = b->probe_off[h]; p < b->probe_off[h + 1]; ++p)
            if (probes[p] < 0 || probes[p] >= N) {
                delete b;
                return fail(LBW_EINVAL, "geometry %d: probe %lld out of range", h, (long long)(p - b->probe_off[h]));
            }
    }
    b->f[0] = f_a;
    b->f[1] = f_b;
    b->nts = 2.0 * 28.0 * (double)b->node_off[n] > 256.0 * 1024.0 * 1024.0;
    b->pery = true;
    for (int h = 0; h < n; ++h)
        if (b->d[h].bc_lo[1] != LBW_BC_PERIODIC || b->d[h].bc_hi[1] != LBW_BC_PERIODIC) b->pery = false;
    b->t_max = b->P > 0 ? t_max : 0;
    b->trace = trace;
    b->items.resize(n);
    b->src_map_off.assign(n, 0);
    b->src_count.assign(n, 0);
    b->src_zlo.assign(n, 0);
    b->src_zhi.assign(n, 0);
    hipError_t e = hipMalloc(&b->tab64, sizeof(double) * b->tab64_off[n]);
    if (e == hipSuccess) e = hipMalloc(&b->tab32, sizeof(float) * lbw::kTabF32 * b->rec_off[n]);
    if (e == hipSuccess) e = hipMalloc(&b->d_items, sizeof(lbw::BatchItem) * n);
    if (e == hipSuccess) e = hipMalloc(&b->d_tcount, sizeof(int64_t) * 2 * n);
    if (e == hipSuccess) e = hipMalloc(&b->d_scratch_count, sizeof(int64_t) * 2 * n);
    if (e == hipSuccess && b->P > 0) e = hipMalloc(&b->d_nodes, sizeof(int64_t) * b->P);
    if (e == hipSuccess && b->P > 0)
        e = hipMemcpyAsync(b->d_nodes, probes, sizeof(int64_t) * b->P, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->d_tcount, 0, sizeof(int64_t) * 2 * n, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->d_scratch_count, 0, sizeof(int64_t) * 2 * n, b->stream);
    for (int h = 0; h < n && e == hipSuccess; ++h) {
        const int64_t E = b->rec_off[h + 1] - b->rec_off[h];
        double* t64 = b->tab64 + b->tab64_off[h];
        float* t32 = b->tab32 + lbw::kTabF32 * b->rec_off[h];
        e = lbw::launch_geometry_tables(b->d[h], t64, t32, b->stream);
        if (e == hipSuccess) {
            const lbw::GeomDev v = lbw::make_geomdev(b->d[h], t32, t64 + 7 * E);
            e = lbw::launch_init(v, p0 + b->node_off[h], f_a + 7 * b->node_off[h], b->stream);
        }
    }
    if (e != hipSuccess) {
        release(b);
        return hip_fail(e, "lbw_batch_make");
    }
    int rc = LBW_OK;
    {
        // default: chunk 16 and the tile with the fewest idle lanes over
        // the whole batch: TX-wide (lanes allotted = sum over geometries of
        // ceil(n0 / TX) TX ceil(n1 / TY) TY n2, ties to the wider tile) or
        // whole rows (workgroup size times the tiles per plane times n2;
        // ties to TX-wide tiles); two waves of resident workgroups for
        // TX-wide tiles (measured best on the 512-horn ensemble among chunks
        // 8..128 and one or two waves), one for whole-row tiles (measured
        // on a 64-horn ensemble: 136 against 152 us per step)
        int cus = 0;
        rc = lbw::device_cus(&cus);
        int tx = 64;
        double best = lane_slots(b, 64);
        for (int cand : {32, 16}) {
            const double sl = lane_slots(b, cand);
            if (sl < best) {
                tx = cand;
                best = sl;
            }
        }
        const int nt = section_threads(b);
        if (nt > 0 && lane_slots(b, 0) < best) tx = 0;
        const int bpc = tx == 0 ? lbw::batch_section_blocks_per_cu(nt) : lbw::batch_blocks_per_cu(tx);
        if (rc == LBW_OK) rc = set_config(b, tx, 16, (tx == 0 ? 1 : 2) * cus * bpc);
    }
    if (rc == LBW_OK && b->P > 0 && hipStreamSynchronize(b->stream) != hipSuccess)
        rc = fail(LBW_EDEVICE, "lbw_batch_make: synchronise");
    if (rc) {
        release(b);
        return rc;
    }
    *out = b;
    return LBW_OK;
}

int lbw_batch_layout(lbw_batch_t b, int64_t* node_offsets, int64_t* probe_offsets) {
    if (!b) return fail(LBW_EINVAL, "batch is NULL");
    for (int h = 0; h <= b->n; ++h) {
        if (node_offsets) node_offsets[h] = b->node_off[h];
        if (probe_offsets) probe_offsets[h] = b->probe_off[h];
    }
    return LBW_OK;
}

int lbw_batch_set_step_config(lbw_batch_t b, int tile_x, int chunk_z, int blocks) {
    if (!b) return fail(LBW_EINVAL, "batch is NULL");
    if (tile_x != 0 && tile_x != 16 && tile_x != 32 && tile_x != 64)
        return fail(LBW_EINVAL, "tile_x must be 0 (whole cross-sections), 16, 32 or 64");
    if (chunk_z < 1 || blocks < 0) return fail(LBW_EINVAL, "chunk_z must be >= 1 and blocks >= 0");
    return set_config(b, tile_x, chunk_z, blocks);
}

int lbw_batch_get_step_config(lbw_batch_t b, int* tile_x, int* chunk_z, int* blocks) {
    if (!b) return fail(LBW_EINVAL, "batch is NULL");
    if (tile_x) *tile_x = b->tx;
    if (chunk_z) *chunk_z = b->lz;
    if (blocks) *blocks = b->blocks;
    return LBW_OK;
}

int lbw_batch_set_graph_block(lbw_batch_t b, int steps) {
    if (!b) return fail(LBW_EINVAL, "batch is NULL");
    if (steps < 0 || steps > 4096) return fail(LBW_EINVAL, "graph block must be in [0, 4096]");
    HIP_TRY(hipStreamSynchronize(b->stream), "lbw_batch_set_graph_block");
    drop_graphs(b);
    b->graph_block = steps;
    return LBW_OK;
}

int lbw_batch_step_n(lbw_batch_t b, int64_t n) {
    if (!b) return fail(LBW_EINVAL, "batch is NULL");
    if (n < 0) return fail(LBW_EINVAL, "negative step count");
    const int K = b->graph_block;
    if (K > 0 && n >= K) {
        if (b->graph_version != b->plan_version) {
            drop_graphs(b);
            b->graph_version = b->plan_version;
        }
        while (n >= K) {
            if (!b->graph[b->cur]) HIP_TRY(build_graph(b, b->cur), "lbw_batch_step_n: graph capture");
            HIP_TRY(hipGraphLaunch(b->graph[b->cur], b->stream), "lbw_batch_step_n: graph launch");
            if (K & 1) b->cur ^= 1;
            b->t += K;
            n -= K;
        }
    }
    const lbw::BatchProbeArgs bp = probe_args(b, true);
    for (int64_t i = 0; i < n; ++i) {
        HIP_TRY(launch_batch(b, bp, b->f[b->cur], b->f[1 - b->cur], b->stream), "lbw_batch_step_n");
        b->cur ^= 1;
        b->t += 1;
    }
    return LBW_OK;
}

int lbw_batch_autotune(lbw_batch_t b, int reps, double* best_us) {
    if (!b) return fail(LBW_EINVAL, "batch is NULL");
    if (reps < 1) return fail(LBW_EINVAL, "reps must be >= 1");
    // Timing launches record nothing: their probe arguments carry t_max = 0
    // and the batch's own scratch step counters (zeroed when the batch is
    // made), so no launch can store into the trace whatever a counter holds.
    int cus = 0;
    int rc = lbw::device_cus(&cus);
    if (rc) return rc;
    float* tmp = nullptr;
    HIP_TRY(hipMalloc((void**)&tmp, sizeof(float) * 7 * b->node_off[b->n]), "lbw_batch_autotune");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    const lbw::BatchProbeArgs bp = probe_args(b, false);
    const int keep_tx = b->tx, keep_lz = b->lz, keep_blocks = b->blocks;
    int best_tx = keep_tx, best_lz = keep_lz, best_blocks = keep_blocks;
    float best_ms = 1e30f;
    float* other = b->f[1 - b->cur];
    const int row_nt = section_threads(b);
    // reps steps of the current configuration on the scratch buffers
    auto time_current = [&]() -> float {
        float* bufs[2] = {other, tmp};
        int w = 0;
        if (err == hipSuccess) err = launch_batch(b, bp, b->f[b->cur], other, b->stream);
        for (int r = 0; r < 2 && err == hipSuccess; ++r, w ^= 1)
            err = launch_batch(b, bp, bufs[w], bufs[w ^ 1], b->stream);
        if (err == hipSuccess) err = hipEventRecord(e0, b->stream);
        for (int r = 0; r < reps && err == hipSuccess; ++r, w ^= 1)
            err = launch_batch(b, bp, bufs[w], bufs[w ^ 1], b->stream);
        if (err == hipSuccess) err = hipEventRecord(e1, b->stream);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        return ms;
    };
    for (int tx : {0, 16, 32, 64}) {  // 0: whole-row tiles, when every geometry's rows fit them
        if (err != hipSuccess) break;
        if (tx == 0 && row_nt == 0) continue;
        const int bpc = tx == 0 ? lbw::batch_section_blocks_per_cu(row_nt) : lbw::batch_blocks_per_cu(tx);
        for (int lz : lz_candidates(b, tx, row_nt, cus * bpc)) {
            for (int mult : {1, 2}) {
                if (set_config(b, tx, lz, mult * cus * bpc) != LBW_OK) {
                    err = hipErrorUnknown;
                    break;
                }
                const float ms = time_current();
                if (err != hipSuccess) break;
                if (ms < best_ms) {
                    best_ms = ms;
                    best_tx = tx;
                    best_lz = lz;
                    best_blocks = b->blocks;
                }
            }
        }
    }
    // the best shape with the other store policy (non-temporal stores pay
    // where the populations do not fit the caches, and cost where they do)
    if (err == hipSuccess && set_config(b, best_tx, best_lz, best_blocks) == LBW_OK) {
        const bool policy = b->nts;
        b->nts = !policy;
        const float ms = time_current();
        if (!(err == hipSuccess && ms < best_ms)) b->nts = policy;
        else best_ms = ms;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(b->stream);
    (void)hipFree(tmp);
    if (err == hipSuccess) rc = set_config(b, best_tx, best_lz, best_blocks);
    else rc = set_config(b, keep_tx, keep_lz, keep_blocks);
    if (err != hipSuccess) return hip_fail(err, "lbw_batch_autotune");
    if (rc) return rc;
    if (best_us) *best_us = 1e3 * best_ms / reps;
    return LBW_OK;
}

int lbw_batch_info(lbw_batch_t b, int64_t* t, float** f_current) {
    if (!b) return fail(LBW_EINVAL, "batch is NULL");
    if (t) *t = b->t;
    if (f_current) *f_current = b->f[b->cur];
    return LBW_OK;
}

int lbw_batch_probe(lbw_batch_t b, double* host_dst, int64_t t0, int64_t t1) {
    if (!b || !host_dst) return fail(LBW_EINVAL, "NULL argument");
    const int64_t rows = b->t < b->t_max ? b->t : b->t_max;
    if (t0 < 0 || t1 < t0 || t1 > rows)
        return fail(LBW_EINVAL, "rows [%lld, %lld) outside [0, %lld)", (long long)t0, (long long)t1, (long long)rows);
    const size_t cnt = (size_t)(t1 - t0) * b->P;
    if (cnt)
        HIP_TRY(hipMemcpyAsync(host_dst, b->trace + t0 * b->P, cnt * sizeof(double), hipMemcpyDeviceToHost, b->stream),
                "lbw_batch_probe");
    HIP_TRY(hipStreamSynchronize(b->stream), "lbw_batch_probe");
    for (size_t i = 0; i < cnt; ++i)
        if (!std::isfinite(host_dst[i]))
            return fail(LBW_EUNSTABLE, "non-finite probe value at row %lld", (long long)(t0 + i / b->P));
    return LBW_OK;
}

int lbw_batch_modes(lbw_batch_t b, int k, double* freq_out, double* power_out) {
    if (!b || !freq_out) return fail(LBW_EINVAL, "NULL argument");
    if (k < 1) return fail(LBW_EINVAL, "k must be >= 1");
    if (b->P < 1) return fail(LBW_EINVAL, "batch has no probes");
    const int64_t T = b->t < b->t_max ? b->t : b->t_max;
    if (T < 8) return fail(LBW_EINVAL, "need at least 8 recorded rows (have %lld)", (long long)T);
    std::vector<int> cols(b->n);
    int max_group = 0;
    for (int h = 0; h < b->n; ++h) {
        cols[h] = (int)(b->probe_off[h + 1] - b->probe_off[h]);
        if (cols[h] > max_group) max_group = cols[h];
    }
    const int cap = lbw::modes_max_cols(T);
    if (max_group > cap) return fail(LBW_EINVAL, "too many probes in one geometry for one spectrum");
    const int chunk_cols = (int)std::min<int64_t>(cap, b->P);
    const size_t need = lbw::modes_work_bytes(T, chunk_cols, b->n);
    if (need > b->mode_work_bytes) {
        (void)hipFree(b->mode_work);
        b->mode_work = nullptr;
        b->mode_work_bytes = 0;
        HIP_TRY(hipMalloc(&b->mode_work, need), "lbw_batch_modes");
        b->mode_work_bytes = need;
    }
    if (k > b->mode_k) {
        (void)hipFree(b->mode_out);
        b->mode_out = nullptr;
        b->mode_k = 0;
        HIP_TRY(hipMalloc(&b->mode_out, sizeof(double) * 2 * (size_t)k * b->n), "lbw_batch_modes");
        b->mode_k = k;
    }
    double* fr = b->mode_out;
    double* pw = b->mode_out + (size_t)k * b->n;
    HIP_TRY(lbw::launch_modes_grouped(b->trace, T, b->P, cols.data(), b->n, k, b->mode_work, b->mode_work_bytes, fr,
                                      pw, b->stream),
            "lbw_batch_modes");
    HIP_TRY(hipMemcpyAsync(freq_out, fr, sizeof(double) * k * b->n, hipMemcpyDeviceToHost, b->stream),
            "lbw_batch_modes");
    if (power_out)
        HIP_TRY(hipMemcpyAsync(power_out, pw, sizeof(double) * k * b->n, hipMemcpyDeviceToHost, b->stream),
                "lbw_batch_modes");
    HIP_TRY(hipStreamSynchronize(b->stream), "lbw_batch_modes");
    return LBW_OK;
}

int lbw_batch_set_sources(lbw_batch_t b, const int64_t* nodes, const int32_t* geom, const double* amplitude,
                          const double* omega, const int32_t* kind, int n) {
    if (!b) return fail(LBW_EINVAL, "batch is NULL");
    if (n < 0 || (n > 0 && (!nodes || !geom || !amplitude || !omega))) return fail(LBW_EINVAL, "invalid source list");
    for (int i = 0; i < n; ++i) {
        if (kind && (kind[i] < 0 || kind[i] > 3)) return fail(LBW_EINVAL, "source %d: kind outside [0, 3]", i);
        if (geom[i] < 0 || geom[i] >= b->n) return fail(LBW_EINVAL, "source %d: geometry out of range", i);
        const int64_t N = b->node_off[geom[i] + 1] - b->node_off[geom[i]];
        if (nodes[i] < 0 || nodes[i] >= N) return fail(LBW_EINVAL, "source %d outside its geometry", i);
        if (!std::isfinite(amplitude[i]) || !std::isfinite(omega[i]))
            return fail(LBW_EINVAL, "source %d: non-finite amplitude or omega", i);
    }
    // sqrt(g) planes (table plane 7) of the geometries that carry sources
    std::map<int, std::vector<double>> sg;
    for (int i = 0; i < n; ++i) {
        const int h = geom[i];
        if (sg.count(h)) continue;
        const int64_t E = b->rec_off[h + 1] - b->rec_off[h];
        std::vector<double>& v = sg[h];
        v.resize((size_t)E);
        HIP_TRY(hipMemcpyAsync(v.data(), b->tab64 + b->tab64_off[h] + 7 * E, sizeof(double) * E,
                               hipMemcpyDeviceToHost, b->stream),
                "lbw_batch_set_sources");
    }
    HIP_TRY(hipStreamSynchronize(b->stream), "lbw_batch_set_sources");
    // sorted by (geometry, node); a node listed twice in one geometry is an error
    std::vector<int> order((size_t)n);
    for (int i = 0; i < n; ++i) order[(size_t)i] = i;
    std::sort(order.begin(), order.end(), [&](int x, int y) {
        return geom[x] != geom[y] ? geom[x] < geom[y] : nodes[x] < nodes[y];
    });
    for (int j = 1; j < n; ++j) {
        const int x = order[(size_t)j - 1], y = order[(size_t)j];
        if (geom[x] == geom[y] && nodes[x] == nodes[y])
            return fail(LBW_EINVAL, "sources %d and %d drive the same node", x, y);
    }
    std::vector<lbw::BatchSource> host((size_t)n);
    std::vector<int> count((size_t)b->n, 0), zlo((size_t)b->n, 0), zhi((size_t)b->n, 0);
    for (int j = 0; j < n; ++j) {
        const int i = order[(size_t)j];
        const int h = geom[i];
        const lbw_geometry_desc& d = b->d[h];
        const int64_t n0 = d.n[0], plane = n0 * d.n[1];
        const double sq = sg[h][(size_t)(nodes[i] % n0 + n0 * (nodes[i] / plane))];
        const double c2 = lbw::lattice_c2(d);
        lbw::BatchSource e{};
        e.node = (uint32_t)nodes[i];
        e.kind = kind ? kind[i] : 0;
        e.a0 = e.kind ? amplitude[i] * 0.5 * sq : amplitude[i] * (1.0 - 3.0 * c2) * sq;
        e.a1 = e.kind ? 0.5 * c2 : amplitude[i] * 0.5 * c2 * sq;
        e.omega = omega[i];
        host[(size_t)j] = e;
        const int z = (int)(nodes[i] / plane);
        if (count[(size_t)h] == 0) zlo[(size_t)h] = z;
        zhi[(size_t)h] = z;
        count[(size_t)h] += 1;
    }
    // Imposed by the step kernel as it loads the populations (a map lookup
    // on every plane of a geometry's driven span) when the driven spans are
    // a small part of the batch's planes; else by a launch of their own.
    // Both use drive_node, so the results are the same bits.
    int64_t span = 0, planes = 0;
    for (int h = 0; h < b->n; ++h) {
        planes += b->d[h].n[2];
        if (count[(size_t)h] > 0) span += zhi[(size_t)h] - zlo[(size_t)h] + 1;
    }
    const bool fused = span * 8 <= planes;
    // node -> entry maps over each geometry's driven planes (sized and
    // checked before anything of the batch changes)
    std::vector<uint32_t> map_off((size_t)b->n, 0);
    int64_t map_len = 0;
    for (int h = 0; fused && h < b->n; ++h) {
        if (count[(size_t)h] == 0) continue;
        const int64_t plane = (int64_t)b->d[h].n[0] * b->d[h].n[1];
        if (map_len > 0x7fffffffLL) return fail(LBW_EINVAL, "driven planes too large for the source map");
        map_off[(size_t)h] = (uint32_t)map_len;
        map_len += plane * (zhi[(size_t)h] - zlo[(size_t)h] + 1);
    }
    if (map_len > 0x7fffffffLL) return fail(LBW_EINVAL, "driven planes too large for the source map");
    drop_graphs(b);
    (void)hipFree(b->d_entries);
    b->d_entries = nullptr;
    b->n_entries = 0;
    if (n > 0 && !fused) {
        std::vector<lbw::SourceEntry> ent((size_t)n);
        for (int j = 0; j < n; ++j) {
            const int i = order[(size_t)j];
            const int h = geom[i];
            lbw::SourceEntry e{};
            e.f_off = (uint64_t)(7 * b->node_off[h] + nodes[i]);
            e.N = (uint32_t)(b->node_off[h + 1] - b->node_off[h]);
            e.q = 7;
            e.counter = h;
            e.kind = host[(size_t)j].kind;
            e.a0 = host[(size_t)j].a0;
            e.a1 = host[(size_t)j].a1;
            e.omega = host[(size_t)j].omega;
            ent[(size_t)j] = e;
        }
        (void)hipFree(b->d_src);
        (void)hipFree(b->d_src_map);
        b->d_src = nullptr;
        b->d_src_map = nullptr;
        b->n_src = 0;
        std::fill(count.begin(), count.end(), 0);
        b->src_count = count;
        HIP_TRY(hipMalloc((void**)&b->d_entries, sizeof(lbw::SourceEntry) * n), "lbw_batch_set_sources");
        HIP_TRY(hipMemcpyAsync(b->d_entries, ent.data(), sizeof(lbw::SourceEntry) * n, hipMemcpyHostToDevice,
                               b->stream),
                "lbw_batch_set_sources");
        b->n_entries = n;
        HIP_TRY(build_items(b), "lbw_batch_set_sources");
        return LBW_OK;
    }
    std::vector<int32_t> map((size_t)map_len, -1);
    for (int j = 0; j < n; ++j) {
        const int i = order[(size_t)j];
        const int h = geom[i];
        const int64_t plane = (int64_t)b->d[h].n[0] * b->d[h].n[1];
        map[(size_t)(map_off[(size_t)h] + nodes[i] - plane * zlo[(size_t)h])] = j;
    }
    (void)hipFree(b->d_src);
    (void)hipFree(b->d_src_map);
    b->d_src = nullptr;
    b->d_src_map = nullptr;
    b->n_src = 0;
    if (n > 0) {
        HIP_TRY(hipMalloc((void**)&b->d_src, sizeof(lbw::BatchSource) * n), "lbw_batch_set_sources");
        HIP_TRY(hipMalloc((void**)&b->d_src_map, sizeof(int32_t) * (size_t)map_len), "lbw_batch_set_sources");
        HIP_TRY(hipMemcpyAsync(b->d_src, host.data(), sizeof(lbw::BatchSource) * n, hipMemcpyHostToDevice, b->stream),
                "lbw_batch_set_sources");
        HIP_TRY(hipMemcpyAsync(b->d_src_map, map.data(), sizeof(int32_t) * (size_t)map_len, hipMemcpyHostToDevice,
                               b->stream),
                "lbw_batch_set_sources");
        b->n_src = n;
    }
    b->src_count = count;
    b->src_zlo = zlo;
    b->src_zhi = zhi;
    b->src_map_off = map_off;
    // the tile list carries the ranges (and waits for the copy above)
    HIP_TRY(build_items(b), "lbw_batch_set_sources");
    return LBW_OK;
}

int lbw_batch_amplitude(lbw_batch_t b, int64_t t0, int64_t t1, double* out) {
    if (!b || !out) return fail(LBW_EINVAL, "NULL argument");
    if (b->P < 1) return fail(LBW_EINVAL, "batch has no probes");
    const int64_t rows = b->t < b->t_max ? b->t : b->t_max;
    if (t0 < 0 || t1 <= t0 || t1 > rows)
        return fail(LBW_EINVAL, "rows [%lld, %lld) empty or outside [0, %lld)", (long long)t0, (long long)t1,
                    (long long)rows);
    if (!b->d_amp) HIP_TRY(hipMalloc((void**)&b->d_amp, sizeof(double) * b->P), "lbw_batch_amplitude");
    HIP_TRY(lbw::launch_amplitude(b->trace, b->P, b->P, t0, t1, b->d_amp, b->stream), "lbw_batch_amplitude");
    HIP_TRY(hipMemcpyAsync(out, b->d_amp, sizeof(double) * b->P, hipMemcpyDeviceToHost, b->stream),
            "lbw_batch_amplitude");
    HIP_TRY(hipStreamSynchronize(b->stream), "lbw_batch_amplitude");
    for (int64_t p = 0; p < b->P; ++p)
        if (!std::isfinite(out[p])) return fail(LBW_EUNSTABLE, "non-finite value at probe %lld", (long long)p);
    return LBW_OK;
}

int lbw_batch_free(lbw_batch_t b) {
    if (!b) return LBW_OK;
    (void)hipStreamSynchronize(b->stream);
    release(b);
    return LBW_OK;
}

}  // extern "C"
