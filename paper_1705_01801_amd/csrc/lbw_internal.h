// Internal declarations shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lbw.h"

namespace lbw {

// Per-entry float table used by the step kernels, 8 floats (32 bytes) per
// (i0, i2) entry: c^2 Mhat00, c^2 Mhat02, c^2 Mhat22, c^2 Mhat11,
// c^2 Gamh0 / 2, c^2 Gamh2 / 2, 0, 0.  The pairs an axis-0 neighbour needs
// (00, 02) and an axis-2 neighbour needs (02, 22) are adjacent.
constexpr int kTabF32 = 8;
// FP64 table planes (exported): Mhat00, Mhat11, Mhat22, Mhat02, Gamh0,
// Gamh1, Gamh2, sqrtg.
constexpr int kTabF64 = 8;

struct GeomDev {
    int dim;
    int n0, n1, n2;   // n2 == 1 for dim 2
    int64_t N;        // nodes
    int bc_lo[3], bc_hi[3];
    float c2;         // c^2
    float two_w0;     // 2 (1 - dim c^2)
    float damp;       // bounce-back damping
    double c2_64;     // c^2 in double (initial state)
    const float* tab;     // kTabF32 floats per entry (general geometries: kGenF32 planes of N floats)
    const double* sqrtg;  // one double per entry (general geometries: per node)
    int sg_node;          // 1: sqrt(g) and coefficients are per node (a geometry given by its metric)
};

// General geometries (given by their metric): FP32 planes of N values used
// by the general step kernel, c^2 Mhat 00, 11, 22, 01, 02, 12 and
// c^2 Gamh / 2 for axes 0, 1, 2; FP64 export planes Mhat (same 6), Gamh (3),
// sqrt(g).
constexpr int kGenF32 = 9;
constexpr int kGenF64 = 10;

// Index of node n's sqrt(g): per (i0, i2) entry, or per node.
__host__ __device__ inline int64_t sg_index(const GeomDev& g, int64_t n) {
    return g.sg_node ? n : n % g.n0 + (int64_t)g.n0 * (n / ((int64_t)g.n0 * g.n1));
}

// Neighbour coordinate one link along an axis; -1 when the link crosses a
// wall, whose code is then stored in *wall.
__host__ __device__ inline int link_coord(int i, int s, int n, int lo, int hi, int* wall) {
    int j = i + s;
    if (j < 0) {
        if (lo == LBW_BC_PERIODIC) return j + n;
        *wall = lo;
        return -1;
    }
    if (j >= n) {
        if (hi == LBW_BC_PERIODIC) return j - n;
        *wall = hi;
        return -1;
    }
    return j;
}

// Kernel launchers (stream-ordered; return hipError_t of the launch).
hipError_t launch_geometry_tables(const lbw_geometry_desc& d, double* tab64, float* tab32, hipStream_t st);
hipError_t launch_index_maps(const GeomDev& g, uint8_t* mask, int32_t* pull, hipStream_t st);
hipError_t launch_init(const GeomDev& g, const double* p0, float* f, hipStream_t st);
hipError_t launch_pressure(const GeomDev& g, const float* f, double* p, hipStream_t st);

struct ProbeArgs {
    const int64_t* nodes;  // device
    int n;
    double* trace;         // device, t_max * n
    int64_t t_max;
    int64_t* tcount;       // device step counter
    unsigned* tdone;       // device, workgroups finished in the current two-step launch (0 between launches)
};
hipError_t launch_step(const GeomDev& g, const ProbeArgs& pr, const float* fin, float* fout, hipStream_t st);
// One step of a geometry given by its metric (3-D, per-node coefficients),
// z-marching tiles (plan.tx x plan.ty = 256 threads, plan.lz planes, one
// workgroup per tile); probes recorded as in the other step kernels.
struct MarchPlan;
hipError_t launch_step_general(const GeomDev& g, const ProbeArgs& pr, const MarchPlan& plan, const float* fin,
                               float* fout, hipStream_t st);

// Launch shape of the z-marching D3Q7 kernel.
struct MarchPlan {
    int tx, ty;          // tile extent along axes 0 and 1 (tx * ty = threads per workgroup, 256 or 512)
    int lz;              // planes per chunk along axis 2
    int ntx, nty, nchunks;
    int64_t tiles;       // ntx * nty * nchunks
    int blocks;          // persistent grid size (multiple of 8)
    int nts;             // 1: non-temporal population stores (one-step kernel)
};
// Default store policy: non-temporal when the two population buffers exceed
// the 256 MiB Infinity Cache.
bool march_nts_default(const GeomDev& g);
MarchPlan make_march_plan(const GeomDev& g, int tx, int ty, int lz, int blocks);
int march_tx_for(int n0);
bool march_shape_ok(int tx, int ty);  // tx in {16, 32, 64}, tx * ty in {256, 512}
int march_blocks_per_cu(int tx, int ty);
hipError_t launch_step_march(const GeomDev& g, const ProbeArgs& pr, const MarchPlan& plan, const float* fin,
                             float* fout, hipStream_t st);

// Two time steps per launch (step_march2.hip): workgroups of tx x (ty + 2)
// threads own ty whole axis-0 rows (n0 <= tx, axis 0 walled) over chunks of
// lz planes, or (lz 0) over balanced shares of all (row tile, plane) pairs;
// plan.ntx is 1.  Shapes: 96 x 6 and 128 x 4 (768 threads).
// The step counter advances by two per launch (needs pr.tdone); the probes
// of both times are recorded, at most march2_tile_probes() per tile.
bool march2_shape_ok(int tx, int ty);
// Balanced two-step plans (lz 0): workgroup b of `blocks` (a multiple of 8)
// takes the pairs [a, e) of the `total` (row tile, plane) pairs, row tile
// major; the workgroups of one XCD (b mod 8) take consecutive shares of one
// eighth of them.  Used by the kernel and by the host's probe check alike.
__host__ __device__ inline void march2_share(int64_t total, int blocks, int b, int64_t* a, int64_t* e) {
    const int xcd = b % 8, per = blocks / 8, k = b / 8;
    const int64_t xs = total * xcd / 8, xe = total * (xcd + 1) / 8;
    *a = xs + (xe - xs) * k / per;
    *e = xs + (xe - xs) * (k + 1) / per;
}
bool march2_fits(const GeomDev& g, int tx);
int march2_tile_probes();
int march2_blocks_per_cu(int tx, int ty);
MarchPlan make_march2_plan(const GeomDev& g, int tx, int ty, int lz, int blocks);
hipError_t launch_step_march2(const GeomDev& g, const ProbeArgs& pr, const MarchPlan& plan, const float* fin,
                              float* fout, hipStream_t st);

// One geometry of a batch (all D3Q7), as read by the batch step kernel.
struct BatchItem {
    int n0, n1, n2;
    uint32_t N;
    int bc_lo[3], bc_hi[3];
    float c2, two_w0, damp;
    int ntx, nty, lz;
    int rty;             // rows per tile when the tiles hold whole rows (run-time tiles)
    int64_t tile_begin;  // first global tile of this geometry
    int64_t tiles;
    uint64_t f_off;      // float offset of the population block (Q * N floats)
    uint32_t tab_off;    // first 32-byte record in the batch float table
    uint32_t sg_off;     // first double in the batch sqrt(g) array
    uint32_t probe_off;  // first probe (global numbering; trace column)
    int n_probes;
    int src_count;             // driven nodes of this geometry (0: none)
    int src_zlo, src_zhi;      // planes (axis 2) of the first and last driven node
    uint32_t src_map;          // first entry of this geometry's map in BatchProbeArgs::src_map
};
// One driven node of a batch geometry (Sec. IV.A / IV.C sources), imposed
// by the step kernel on the populations it loads: kind 0 pressure (a0 =
// amplitude w_0 sqrt(g), a1 = amplitude w sqrt(g)), kind 1 + a flux along
// axis a (a0 = amplitude sqrt(g) / 2, a1 = w); drive_node has the rules.
struct BatchSource {
    uint32_t node;   // node index within its geometry
    int32_t kind;
    double a0, a1, omega;
};
struct BatchProbeArgs {
    const int64_t* nodes;  // device, all probes, node index within its geometry
    double* trace;         // device, t_max rows of `stride` doubles
    int64_t stride;        // total probes (trace row length)
    int64_t t_max;
    // device, two banks of one step counter per geometry: a launch reads
    // bank `parity` (the time of its sources and trace row) and its probe
    // blocks write time + 1 into the other bank, so no block of a launch
    // reads a counter that another block of it changes
    int64_t* tcount;
    int parity;
    const double* sqrtg;   // device, batch sqrt(g) array
    const float4* tab4;    // device, batch float table (2 float4 per record)
    const BatchSource* src;  // device, driven nodes of all geometries (NULL: none)
    // device, per geometry with driven nodes: for every node of planes
    // src_zlo .. src_zhi (plane-major, as the populations) its entry in src,
    // or -1
    const int32_t* src_map;
};
int batch_blocks_per_cu(int tx);
// Rows per whole-row tile of nt threads (128, 256 or 512) for an n0 x n1
// cross-section: the most rows r <= n1 with n0 r <= nt lanes and
// 2 (n0 + r) <= nt ring loaders (and n0 + 2 <= nt row loaders), or 0.
int batch_row_tile(int n0, int n1, int nt);
int batch_section_blocks_per_cu(int nt);
// section_nt > 0 selects whole-row tiles of section_nt threads (the tile
// list must then hold ntx = 1 and nty = ceil(n1 / rty) tiles per chunk).
// tile_item: the geometry of each of the tiles_total tiles (device); nts:
// non-temporal population stores; pery: every geometry of the batch is
// periodic along axis 1 (the variant without that axis's wall rules).
hipError_t launch_step_batch(const BatchItem* items, const int32_t* tile_item, int n_items, int64_t tiles_total,
                             int tx, int section_nt, int blocks, bool nts, bool pery, const BatchProbeArgs& bp,
                             const float* fin, float* fout, hipStream_t st);

// One driven node (Sec. IV.A/IV.C sources): its populations sit at
// f[f_off + l N], l < q; the time is counters[counter].  kind 0 imposes a
// pressure (a0 = amplitude w_0 sqrt(g), a1 = amplitude w sqrt(g)); kind
// 1 + a a flux along axis a (a0 = amplitude sqrt(g) / 2, a1 = w).
struct SourceEntry {
    uint64_t f_off;
    uint32_t N;
    int32_t q;
    int32_t counter;
    int32_t kind;
    double a0, a1, omega;
};
// Imposes every source at its current time (before the step that reads f).
hipError_t launch_sources(const SourceEntry* src, int n, const int64_t* counters, float* f, hipStream_t st);
// out[c] = max over rows [t0, t1) of |trace[t * stride + c]|, c < cols (NaN if any is NaN).
hipError_t launch_amplitude(const double* trace, int64_t stride, int64_t cols, int64_t t0, int64_t t1, double* out,
                            hipStream_t st);

// Spectra of probe groups (consecutive trace columns, one group per
// geometry): fills freq/power (device, groups * k each) from trace rows
// [0, T) of row length `stride`.  Synchronises the stream per chunk.
int64_t modes_nfft(int64_t T);
int modes_max_cols(int64_t T);
size_t modes_work_bytes(int64_t T, int max_cols, int max_groups);
hipError_t launch_modes_grouped(const double* trace, int64_t T, int64_t stride, const int* group_ncols, int groups,
                                int k, double* work, size_t work_bytes, double* freq, double* power, hipStream_t st);
// The same spectrum for one group of ncols columns without allocating: the
// work space is the library's fixed device array (kModesScratchBytes per
// GPU; modes_scratch gives its address on the current device), columns are
// transformed modes_static_cols(T) at a time and their power accumulated.
// Nothing is waited for; freq and power (k doubles each) are device memory.
constexpr size_t kModesScratchBytes = size_t(32) << 20;
hipError_t modes_scratch(void** ptr);
int modes_static_cols(int64_t T);  // 0 when one column does not fit
hipError_t launch_modes_static(void* scratch_ptr, const double* trace, int64_t T, int64_t stride, int ncols, int k,
                               double* freq, double* power, hipStream_t st);

}  // namespace lbw
