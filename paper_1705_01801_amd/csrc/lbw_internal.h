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
    const float* tab;     // kTabF32 floats per entry
    const double* sqrtg;  // one double per entry
};

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
};
hipError_t launch_step(const GeomDev& g, const ProbeArgs& pr, const float* fin, float* fout, hipStream_t st);

// Launch shape of the z-marching D3Q7 kernel.
struct MarchPlan {
    int tx, ty;          // tile extent along axes 0 and 1 (tx * ty = 256)
    int lz;              // planes per chunk along axis 2
    int ntx, nty, nchunks;
    int64_t tiles;       // ntx * nty * nchunks
    int blocks;          // persistent grid size (multiple of 8)
};
MarchPlan make_march_plan(const GeomDev& g, int tx, int lz, int blocks);
int march_tx_for(int n0);
int march_blocks_per_cu(int tx);
hipError_t launch_step_march(const GeomDev& g, const ProbeArgs& pr, const MarchPlan& plan, const float* fin,
                             float* fout, hipStream_t st);

// Spectrum: fills freq/power (device, k each) from trace rows [0, T).
hipError_t launch_modes(const double* trace, int64_t T, int n_probes, int k, double* work, size_t work_bytes,
                        double* freq, double* power, hipStream_t st);
size_t modes_work_bytes(int64_t T, int n_probes);

}  // namespace lbw
