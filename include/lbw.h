/*
 * lbw: curvilinear wave lattice-Boltzmann on AMD Instinct MI355X (gfx950).
 *
 * The method is the lattice-Boltzmann model for the scalar wave equation in
 * curvilinear coordinates of Velasco, Munoz and Mendoza (arXiv 1705.01801):
 * a D3Q7 (or D2Q5) lattice that is uniform in the generalised coordinates,
 * BGK relaxation with tau = 1/2, the corrected equilibrium of Sec. III
 * (f_0 = w_0 sqrt(g) P, f_l = w_l sqrt(g) [P + xi_l.J'/c_s^2]) and the
 * Christoffel and metric-gradient forcing carried in the corrected momentum
 * J' (Sec. III, corrected-momentum equation).  Walls follow Sec. IV.A
 * (bounce-back with damping, free) plus a fixed P = 0 wall.
 *
 * Conventions for every entry point:
 *  - returns LBW_OK (0) or a negative LBW_E* code; lbw_last_error() gives a
 *    message for the calling thread's last failure.  Arguments are validated
 *    on the host before any device work is queued; on error nothing is
 *    queued and no output is written.
 *  - "device" pointers are HIP device memory owned by the caller; "host"
 *    pointers are ordinary host memory.  The library owns only the opaque
 *    geometry/state objects and the small tables and scratch inside them.
 *  - stream arguments are hipStream_t passed as void* (NULL = the null
 *    stream).  All device work is queued on that stream; the calls that
 *    wait for it say so below ("Synchronises", "Waits for the stream").
 *  - populations are stored structure-of-arrays, f[l * N + n] with node
 *    n = i0 + n0 * (i1 + n1 * i2) and l in the order
 *    0: rest, 1: +e0, 2: -e0, 3: +e1, 4: -e1, 5: +e2, 6: -e2 (Q = 2*dim + 1).
 */
#ifndef LBW_H
#define LBW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBW_OK 0
#define LBW_EINVAL (-1)    /* invalid argument */
#define LBW_ENOMEM (-2)    /* device allocation failed */
#define LBW_EDEVICE (-3)   /* HIP runtime error */
#define LBW_EUNSTABLE (-4) /* non-finite value found in a probe trace */
#define LBW_ESTATE (-5)    /* call not valid in the object's current state */

/* Coordinate systems (Sec. IV).  Axis order (q0, q1, q2):
 *  LBW_BOX         Cartesian (x, y, z); 2-D or 3-D
 *  LBW_POLAR2D     (r, theta), 2-D restriction of the cylinder
 *  LBW_CYLINDER    (r, theta, z), Sec. IV.A
 *  LBW_HORN        (r, theta, z), x = r s(z) cos(theta), y = r s(z) sin(theta),
 *                  s(z) = a + b exp(k z); params = {a, b, k}
 *  LBW_TORUS       (rho, theta major, phi minor), Sec. IV.C; params = {R}
 *  LBW_BESSEL_HORN as LBW_HORN with s(z) = (Zmax - z)^(-lambda), the Bessel
 *                  horn of Sec. IV.B; params = {lambda, Zmax}
 *  LBW_GENERAL     any 3-D coordinates, given by their metric per node
 *                  (lbw_make_geometry_general); params unused
 */
enum { LBW_BOX = 0, LBW_POLAR2D = 1, LBW_CYLINDER = 2, LBW_HORN = 3, LBW_TORUS = 4, LBW_BESSEL_HORN = 5,
       LBW_GENERAL = 6 };

/* Wall codes per face.  Walls sit half a link outside the end nodes.
 *  PERIODIC    both faces of the axis must be periodic
 *  BOUNCEBACK  half-way bounce-back, reflected population scaled by the
 *              damping factor D (Sec. IV.A, pipe boundary conditions)
 *  FREE        the incoming population copies the boundary node's own
 *              post-collision population ("copying the values of the
 *              neighbouring cell", Sec. IV.A)
 *  FIXED       half-way anti-bounce-back, pressure P = 0 on the wall */
enum { LBW_BC_PERIODIC = 0, LBW_BC_BOUNCEBACK = 1, LBW_BC_FREE = 2, LBW_BC_FIXED = 3 };

/* Equilibrium.
 *  CORRECTED  the corrected equilibrium of Sec. III, f_0 = w_0 sqrt(g) P,
 *             f_l = w sqrt(g) (P + xi_l.J' / c^2) with c_s = c (every kind)
 *  HERMITE    the Hermite-expansion equilibrium of Sec. II, Cartesian boxes
 *             only: the fixed D2Q5/D3Q7 weights (c_s^2 = 1/(D+1), w = c_s^2/2)
 *             plus the second-order term P (c^2 - c_s^2)(xi^2 - D c_s^2) /
 *             (2 c_s^4), f_0 = P - sum_{l>=1} f_l.  Its second moment is
 *             c_eff^2 P, c_eff^2 = c_s^2 + (c^2 - c_s^2)(1 - D c_s^2) / (2 c_s^2)
 *             (c^2/2 + 1/8 on D3Q7), so it steps exactly as CORRECTED at wave
 *             speed c_eff, which is how the library runs it; the two coincide
 *             at c = c_s. */
enum { LBW_EQ_CORRECTED = 0, LBW_EQ_HERMITE = 1 };

typedef struct {
    int32_t kind;      /* LBW_BOX ... LBW_BESSEL_HORN */
    int32_t dim;       /* 2 -> D2Q5, 3 -> D3Q7 */
    int32_t n[3];      /* nodes per axis (n[2] ignored for dim 2) */
    int32_t bc_lo[3];  /* wall code of the low face of each axis */
    int32_t bc_hi[3];  /* wall code of the high face of each axis */
    int32_t equilibrium; /* LBW_EQ_CORRECTED or LBW_EQ_HERMITE (boxes only) */
    double qmin[3];    /* coordinate range; periodic axis nodes at qmin + i h, */
    double qmax[3];    /* walled axis nodes at qmin + (i + 1/2) h, h = (qmax - qmin) / n */
    double h_ref;      /* physical length of one lattice unit (> 0) */
    double c;          /* lattice wave speed c = c_phys dt / h_ref (c_s = c; for
                          LBW_EQ_HERMITE the c of its formula, see above) */
    double damping;    /* bounce-back damping factor D in [0, 1] */
    double params[4];  /* kind-specific, see above */
} lbw_geometry_desc;

typedef struct lbw_geometry* lbw_geometry_t;
typedef struct lbw_state* lbw_state_t;

/* Builds the per-geometry coefficient tables on the device (Sec. III and IV:
 * sqrt(g), g^{ij} and the contracted Christoffel symbols
 * Gamma^i = Gamma^i_jk g^jk, evaluated in FP64 from closed forms and
 * converted to lattice units: Mhat^{ij} = h_ref^2 g^{ij}/(h_i h_j) - delta^{ij},
 * Gamh^i = h_ref^2 Gamma^i / h_i).  The coefficients of every supported kind
 * depend on (i0, i2) only, so tables are n0 x n2.  Queued on stream; the
 * geometry may be used by later calls on the same stream at once.
 * Errors: LBW_EINVAL for an invalid descriptor (bad kind/dim pairing, n < 1,
 * qmax <= qmin, h_ref <= 0, c <= 0 or not finite, damping outside [0, 1],
 * unpaired periodic faces, radius <= 0, torus rho >= R, horn s(z) <= 0,
 * a population buffer of 2^31 bytes or more, i.e. 4 Q N >= 2^31: the step
 * kernels address it with 32-bit byte offsets; at most 76,695,844 nodes for
 * D3Q7); LBW_ENOMEM; LBW_EDEVICE. */
int lbw_make_geometry(const lbw_geometry_desc* desc, void* stream, lbw_geometry_t* out);

/* A 3-D geometry given by its metric (Sec. III: the scheme needs only
 * sqrt(g), the inverse metric and the contracted Christoffel symbols, so any
 * coordinate system runs by supplying them).  desc->kind is LBW_GENERAL and
 * dim 3; desc->params is unused.  metric (host, read during the call) holds
 * 10 planes of N doubles, node n = i0 + n0 (i1 + n1 i2), in the coordinates'
 * own units: sqrt(g), G^00, G^11, G^22, G^01, G^02, G^12 (G = g^{-1}), and
 * Gamma^0, Gamma^1, Gamma^2 (Gamma^i = Gamma^i_jk G^jk).  They are converted
 * to lattice units as in lbw_make_geometry and kept per node; such a
 * geometry is stepped by a per-node kernel that reads 36 coefficient bytes
 * per node, takes the shapes of lbw_set_step_config listed there but no
 * autotuning, and cannot join a batch.  Waits for the stream.  Errors: as
 * lbw_make_geometry, plus LBW_EINVAL for another kind, NULL metric, a
 * non-finite value, sqrt(g) <= 0, or 36 N >= 2^31 bytes of coefficients
 * (at most 59,652,323 nodes). */
int lbw_make_geometry_general(const lbw_geometry_desc* desc, const double* metric, void* stream,
                              lbw_geometry_t* out);

/* Releases a geometry (waits for its stream first).  NULL is accepted. */
int lbw_free_geometry(lbw_geometry_t g);

/* Exported views, for checking the device tables (synchronises):
 *  LBW_EXPORT_TABLE_F64  8 planes of n0*n2 doubles, entry e = i0 + n0*i2:
 *                        Mhat00, Mhat11, Mhat22, Mhat02, Gamh0, Gamh1, Gamh2, sqrtg;
 *                        for LBW_GENERAL 10 planes of N doubles (per node):
 *                        Mhat00, 11, 22, 01, 02, 12, Gamh0, 1, 2, sqrtg
 *  LBW_EXPORT_MASK_U8    N bytes; bit (l-1) set when the link n -> n + xi_l
 *                        crosses a wall
 *  LBW_EXPORT_PULL_I32   Q*N int32; entry l*N + n is the node population l
 *                        arrives from at n (periodic wrap applied), or
 *                        -(1 + wall code) when it arrives through a wall
 * bytes must equal the exported size exactly (LBW_EINVAL otherwise). */
enum { LBW_EXPORT_TABLE_F64 = 0, LBW_EXPORT_MASK_U8 = 1, LBW_EXPORT_PULL_I32 = 2 };
int lbw_geometry_export(lbw_geometry_t g, int what, void* host_dst, size_t bytes);

/* Frozen-coefficient stability bound of the tau = 1/2 step on this geometry:
 * c_max = 2 / sqrt(max_nodes sum_d B_d), B_d = 4 if m_d <= 1 else
 * (1 + m_d)^2 / m_d, m_d = Mhat^dd (+ |Mhat^02| on axes 0 and 2; for
 * LBW_GENERAL + the |Mhat^de| of both off-diagonal components of axis d).
 * Synchronises.  Errors: LBW_EINVAL for NULL arguments. */
int lbw_stability_bound(lbw_geometry_t g, double* c_max);

/* Launch shape of the 3-D step kernel for this geometry (the per-node
 * arithmetic, and so every result, is the same for every shape; only speed
 * changes).  A workgroup owns a tile_x x tile_y tile of (axis 0, axis 1)
 * columns: tile_x is 16, 32 or 64 and tile_x * tile_y, the workgroup size,
 * is 256 or 512, or the tile is 96 x 4, 96 x 8, 128 x 4 or 128 x 8 (384
 * to 1024 threads; rows of up to 96 or 128 nodes in one tile); chunk_z >= 1
 * planes per tile along axis 2; blocks:
 * persistent grid size, rounded down to a multiple of 8 (0 = one full wave
 * of resident workgroups).  Used by lbw_autotune and by tests.
 * A geometry given by its metric (LBW_GENERAL) has its own kernel: tile
 * 32 x 8, 64 x 4 or 64 x 8, any chunk_z, blocks 0 (one workgroup per tile;
 * default 64 x 8 when n0 > 32, else 32 x 8, chunk 16).
 * Errors: LBW_EINVAL for a 2-D geometry or out-of-range values. */
int lbw_set_step_config(lbw_geometry_t g, int tile_x, int tile_y, int chunk_z, int blocks);
int lbw_get_step_config(lbw_geometry_t g, int* tile_x, int* tile_y, int* chunk_z, int* blocks);

/* Two time steps per launch (temporal blocking) for this geometry: each
 * launch advances the state from t to t+2 with one read and one write of
 * every population, the intermediate state held on chip; the per-node
 * arithmetic is the one-step kernel's, so results are identical bit for bit.
 * A workgroup owns tile_y whole axis-0 rows plus a halo row either side
 * (tile_x = 96 with tile_y = 6, or 128 with 4; 768 threads), chunk_z planes
 * along axis 2, or with chunk_z = 0 an equal share of all (row tile, plane)
 * pairs per workgroup (no workgroup marches two whole chunks while another
 * idles); blocks as in lbw_set_step_config (0 = one wave).  Needs a
 * 3-D built-in geometry with n0 <= tile_x and a walled axis 0.
 * lbw_step_n then runs pairs of steps this way (an odd last step, and
 * states with driven sources or with more than 16 probes in one tile of
 * the pass, use one-step launches).  tile_x = 0 turns it off;
 * lbw_set_step_config also turns it off; lbw_autotune turns it on when
 * its best shape is faster per step.  Errors: LBW_EINVAL (other shapes, a
 * geometry it does not fit, chunk_z < 0, blocks < 0). */
int lbw_set_step2_config(lbw_geometry_t g, int tile_x, int tile_y, int chunk_z, int blocks);
/* The two-step shape in use (tile_x = 0 and the rest 0 when off). */
int lbw_get_step2_config(lbw_geometry_t g, int* tile_x, int* tile_y, int* chunk_z, int* blocks);

/* Creates a simulation state on caller-owned device buffers.
 *  p0        device, N doubles: initial pressure P; populations start at the
 *            corrected equilibrium at rest, f_l = w_l sqrt(g) P0 with
 *            w_0 = 1 - dim c^2, w_l = c^2 / 2 (rounded once to float)
 *  f_a, f_b  device, Q*N floats each, distinct; ping-pong population
 *            buffers, f_a holds the state after init
 *  probes    host, n_probes node indices in [0, N) (copied)
 *  trace     device, t_max * n_probes doubles: row t receives the pressure
 *            P = sum_l f_l / sqrt(g) at every probe before step t
 *  t_max     capacity of trace in rows (>= 0); steps beyond it run but
 *            record nothing
 * The state keeps the buffer pointers; the caller keeps them alive until
 * lbw_free_state.  Errors: LBW_EINVAL (NULL pointers, f_a == f_b,
 * probe out of range, n_probes < 0, n_probes > 0 with trace == NULL),
 * LBW_ENOMEM, LBW_EDEVICE. */
int lbw_init(lbw_geometry_t g, const double* p0, float* f_a, float* f_b, const int64_t* probes, int n_probes,
             double* trace, int64_t t_max, void* stream, lbw_state_t* out);

/* Queues n time steps (BGK, tau = 1/2, fused collide-and-push-stream with
 * walls; Sec. II evolution equation with the Sec. III equilibrium and
 * forcing) and the probe recording; returns without waiting.
 * Errors: LBW_EINVAL for n < 0, LBW_EDEVICE on a launch failure. */
int lbw_step_n(lbw_state_t s, int64_t n);

/* Picks the fastest launch shape of the 3-D step kernel for this state's
 * geometry by timing candidates (tile_x 16/32/64 with workgroups of 256 and
 * 512 threads, and the whole-row tiles 96 x 4, 96 x 8, 128 x 4 and 128 x 8;
 * chunk_z 4, 8, 16, 32, 64 (up to twice n2); one and two waves of resident
 * workgroups) for reps launches each with HIP events.  The
 * candidates run real ping-pong steps (each launch reads what the previous
 * one wrote) from the state's current buffer into its other buffer and a
 * temporary buffer of Q*N floats (allocated for the call), with
 * probe recording off; the current buffer, step count and trace are
 * unchanged.  The best shape is also timed with the other store policy
 * (non-temporal population stores, the default where the two population
 * buffers exceed the 256 MiB Infinity Cache, or cached ones).  Two-step
 * launches (lbw_set_step2_config: tiles 96 x 6 and
 * 128 x 4 where the geometry fits them, chunk_z 0 (balanced) and 8 to 64,
 * one and two waves)
 * are timed per step as well, and used when faster.  The three fastest
 * candidates of each kind are timed again over three times the launches
 * before one is kept; every candidate runs with the state's probes
 * recorded into scratch memory.  The choice is stored in
 * the geometry and in a per-process
 * cache keyed by the grid shape, which later geometries of that shape start
 * from.  Synchronises.  best_us (may be NULL) receives the best time per
 * step in microseconds.  Errors: LBW_EINVAL (2-D or LBW_GENERAL geometry,
 * reps < 1). */
int lbw_autotune(lbw_state_t s, int reps, double* best_us);

/* Number of steps lbw_step_n captures into one HIP graph and replays
 * (0 disables graphs; default 32).  Graphs are rebuilt when the launch
 * shape changes. */
int lbw_set_graph_block(lbw_state_t s, int steps);

/* Copies trace rows [t0, t1) (t1 <= recorded rows) to host memory,
 * n_probes doubles per row.  Synchronises.  Returns LBW_EUNSTABLE (after
 * copying) when a copied value is not finite. */
int lbw_probe(lbw_state_t s, double* host_dst, int64_t t0, int64_t t1);

/* Resonant frequencies of the recorded probe traces, computed on the device
 * in FP64: per probe subtract the mean, apply the symmetric Hann window
 * 1/2 - 1/2 cos(2 pi t/(T-1)), zero-pad to 4 x the next power of two of T,
 * FFT, sum |X_k|^2 over probes; peaks are bins k in [16, nfft/2 - 1] with
 * P[k-1] < P[k] >= P[k+1] and P[k] > 1e-3 max_{k>=16} P (bin 16 is the first
 * outside the window's DC main lobe), refined by a parabola through ln P
 * (no refinement when a neighbour bin is 0); the k lowest, ascending, in
 * cycles per step (NaN-padded).  A trace holding a non-finite value gives
 * no peaks (all NaN).  power_out may be NULL.  The FFT work space (32 nfft
 * bytes per probe, up to 1 GiB per pass) is allocated on first use and kept
 * with the state.  Synchronises.  Errors: LBW_EINVAL (k < 1, fewer than 8
 * recorded rows, no probes, more probes than one 1 GiB pass holds),
 * LBW_ENOMEM, LBW_EDEVICE. */
int lbw_modes(lbw_state_t s, int k, double* freq_out, double* power_out);

/* lbw_modes for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same rule and bit-identical results, but the FFT work space is a fixed
 * 32 MiB array of device memory that the library holds on each GPU it runs
 * on until the process ends (probe columns are transformed a few at a time
 * through it), the results go to device memory and nothing is waited for.
 *  freq_dev, power_dev  device, k doubles each (ascending frequencies in
 *                       cycles per step, NaN-padded; their spectral powers),
 *                       ready once the state's stream reaches this call
 * Calls no allocator.  All calls on one GPU share that array: calls whose
 * work overlaps in time on one GPU (other streams, other threads) race and
 * must be ordered by the caller; the array is fully rewritten by each call,
 * so nothing carries over from the previous one.  Errors: LBW_EINVAL (NULL
 * arguments, k < 1, no probes, fewer than 8 or more than
 * LBW_MODES_NOALLOC_MAX_ROWS recorded rows), LBW_EDEVICE. */
#define LBW_MODES_NOALLOC_MAX_ROWS 131072
int lbw_modes_noalloc(lbw_state_t s, int k, double* freq_dev, double* power_dev);

/* Current step count and the device buffer holding the current populations. */
int lbw_state_info(lbw_state_t s, int64_t* t, float** f_current);

/* Driven sources (Sec. IV.A pipe plate and ring sources, Sec. IV.C torus
 * ring and point sources: a pressure, or a flux, imposed at chosen nodes as a
 * harmonic function of time).  From the next queued step on, at every time t
 * (steps since lbw_init), with v = amplitude * sin(omega t), each node in
 * nodes[0..n) is set before the probes are read and the step t -> t+1 is
 * taken; omega is in radians per step:
 *  kind LBW_SOURCE_PRESSURE: put at rest at the pressure P = v,
 *    f_0 = w_0 sqrt(g) P and f_l = w sqrt(g) P (the rule of lbw_init);
 *  kind LBW_SOURCE_FLUX + a (axis a < dim; the oscillating plate, J'_a = v):
 *    the node keeps S = sum_l f_l and takes the equilibrium with first
 *    moment sqrt(g) v along a, f_0 = w_0 S, f_l = w S + e_l^a sqrt(g) v / 2.
 *    This is sqrt(g) J'_a where the flux definition's force correction
 *    vanishes on axis a (Gamma^a = 0 and g^{aj} = delta^{aj}, as for the
 *    axis of the cylindrical pipe); elsewhere it is the imposed first moment.
 * nodes is host memory, read during the call.  n = 0 removes the sources.
 * Waits for the stream.  Errors: LBW_EINVAL (n < 0, NULL nodes with n > 0, a
 * node outside the grid, non-finite amplitude or omega, kind outside
 * [0, dim]), LBW_ENOMEM, LBW_EDEVICE. */
#define LBW_SOURCE_PRESSURE 0
#define LBW_SOURCE_FLUX 1
int lbw_set_sources(lbw_state_t s, const int64_t* nodes, int n, double amplitude, double omega, int kind);

/* Response intensity of a driven run (the frequency sweeps of Sec. IV.A and
 * IV.C): out (host, n_probes values) receives the largest |P| of each probe
 * over recorded rows [t0, t1).  Waits for the stream.  Errors: LBW_EINVAL
 * (no probes, an empty window or one outside the recorded rows),
 * LBW_EUNSTABLE (a non-finite value in the window; out is still written). */
int lbw_amplitude(lbw_state_t s, int64_t t0, int64_t t1, double* out);

/* Pressure P = sum_l f_l / sqrt(g) of the current state into a device buffer
 * of N doubles (queued on the state's stream). */
int lbw_pressure(lbw_state_t s, double* p_out);

/* Releases a state (waits for its stream first); caller buffers are left
 * untouched.  NULL is accepted. */
int lbw_free_state(lbw_state_t s);

/* ------------------------------------------------------------------------
 * Batches: many D3Q7 geometries (e.g. horns of different profiles and grid
 * sizes) advanced together, one launch per step for the whole batch, with
 * the same per-node arithmetic as lbw_step_n.
 *
 * Layout (caller-owned device buffers):
 *  populations  geometry h occupies floats [7 o_h, 7 o_{h+1}) of f_a and f_b,
 *               SoA inside (f[7 o_h + l N_h + n]), o_h = sum_{j<h} N_j
 *  p0           doubles [o_h, o_{h+1})
 *  probes       host; geometry h's n_probes[h] node indices (local to h)
 *               follow those of geometries < h
 *  trace        device, t_max rows of P = sum_h n_probes[h] doubles; row t,
 *               column (first probe of h) + j is probe j of geometry h
 *               before step t
 * ---------------------------------------------------------------------- */
typedef struct lbw_batch* lbw_batch_t;

/* Builds every geometry's tables (as lbw_make_geometry) into batch tables,
 * initialises every geometry at rest (as lbw_init) into f_a, and prepares
 * the tile list.  Errors: LBW_EINVAL (n < 1, a descriptor invalid or not
 * 3-D, NULL pointers, f_a == f_b, a probe outside its geometry,
 * n_probes[h] < 0), LBW_ENOMEM, LBW_EDEVICE. */
int lbw_batch_make(const lbw_geometry_desc* descs, int n, const double* p0, float* f_a, float* f_b,
                   const int64_t* probes, const int32_t* n_probes, double* trace, int64_t t_max, void* stream,
                   lbw_batch_t* out);

/* Node offsets o_0..o_n and probe offsets (n + 1 values each, host). */
int lbw_batch_layout(lbw_batch_t b, int64_t* node_offsets, int64_t* probe_offsets);

/* Launch shape shared by all geometries of the batch (as
 * lbw_set_step_config, with 256-thread workgroups: tile_y = 256 / tile_x).
 * tile_x = 0 selects whole-row tiles instead: each workgroup (128, 256 or
 * 512 threads, one size for the batch) takes r whole axis-0 rows of one
 * geometry over a chunk of planes, r the most rows with n0 r and
 * 2 (n0 + r) at most the workgroup size (the whole cross-section when it
 * fits); every geometry needs n0 + 2 <= 512 and r >= 1, else LBW_EINVAL.
 * Results are identical for every shape.  The default made by
 * lbw_batch_make is chunk_z 16 and the tile with the fewest idle lanes
 * over all geometries: tile_x = 16, 32 or 64 (lanes: sum of
 * ceil(n0/tile_x) tile_x * ceil(n1/tile_y) tile_y * n2, ties to the wider
 * tile; two waves of resident workgroups) or whole rows (lanes: workgroup
 * size * ceil(n1/r) * n2, ties to TX-wide tiles; one wave of resident
 * workgroups).  lbw_batch_autotune times the candidates instead. */
int lbw_batch_set_step_config(lbw_batch_t b, int tile_x, int chunk_z, int blocks);
int lbw_batch_get_step_config(lbw_batch_t b, int* tile_x, int* chunk_z, int* blocks);
/* Times launch shapes (whole-row tiles when the batch allows them, tile_x
 * 16, 32 and 64; chunk_z 4, 8, 16, 32, 64 and, per tile kind, the four
 * other lengths in 4..64 whose tile count spreads best over the resident
 * workgroups; one or two waves of resident workgroups; then the best shape
 * with the other population store policy: non-temporal stores, the default
 * when the two population buffers exceed 256 MiB, or cached ones) with reps
 * steps each on scratch buffers, recording no probes and leaving
 * populations, step count and trace untouched, and keeps the fastest; best_us (may be NULL) receives its microseconds per step.
 * Synchronises.  Errors: LBW_EINVAL (NULL batch, reps < 1), LBW_ENOMEM,
 * LBW_EDEVICE (the previous shape is kept). */
int lbw_batch_autotune(lbw_batch_t b, int reps, double* best_us);
int lbw_batch_set_graph_block(lbw_batch_t b, int steps);

/* Queues n steps of every geometry (probes recorded) without waiting. */
int lbw_batch_step_n(lbw_batch_t b, int64_t n);

/* Step count and the device buffer holding the current populations. */
int lbw_batch_info(lbw_batch_t b, int64_t* t, float** f_current);

/* Copies trace rows [t0, t1) (all P columns) to host; as lbw_probe. */
int lbw_batch_probe(lbw_batch_t b, double* host_dst, int64_t t0, int64_t t1);

/* Resonant frequencies of every geometry (rule of lbw_modes over that
 * geometry's probes): freq_out and power_out (may be NULL) receive n * k
 * values, geometry-major.  Synchronises.  Errors as lbw_modes. */
int lbw_batch_modes(lbw_batch_t b, int k, double* freq_out, double* power_out);

/* Driven sources of a batch (the rules of lbw_set_sources): source i sits
 * at node nodes[i] of geometry geom[i] with its own amplitude[i], omega[i]
 * and kind[i] (NULL kind: all LBW_SOURCE_PRESSURE), so one batch can sweep
 * many drive frequencies, and both source kinds, over copies of a geometry;
 * t is that geometry's step count.  Where the driven nodes lie on few planes
 * (from each geometry's first to last driven plane, at most an eighth of the
 * batch's planes in all) the batch step imposes them itself, on the
 * populations it loads (nothing written to the input buffer); otherwise a
 * launch of their own does, before every step.  Both use the per-node
 * arithmetic of lbw_set_sources, so a driven copy in a batch and the same
 * copy driven alone give the same bits.
 * All arrays are host memory of n entries, read during the call; n = 0
 * removes the sources.  Waits for the stream.  Errors: LBW_EINVAL (n < 0,
 * NULL nodes, geom, amplitude or omega with n > 0, a geometry index or node
 * out of range, a node listed twice for one geometry, non-finite amplitude
 * or omega, a kind outside [0, 3]), LBW_ENOMEM, LBW_EDEVICE. */
int lbw_batch_set_sources(lbw_batch_t b, const int64_t* nodes, const int32_t* geom, const double* amplitude,
                          const double* omega, const int32_t* kind, int n);

/* Response intensity of every probe of the batch (P values in global probe
 * order) over rows [t0, t1); as lbw_amplitude. */
int lbw_batch_amplitude(lbw_batch_t b, int64_t t0, int64_t t1, double* out);

/* Releases the batch (waits for its stream); caller buffers untouched. */
int lbw_batch_free(lbw_batch_t b);

/* ------------------------------------------------------------------------
 * Surrogate MLP (learned map from horn-profile parameters to resonant
 * frequencies, trained on spectra from the batched LBM).  Dense layers
 * widths[0] -> ... -> widths[n_layers], tanh on hidden layers, linear output.
 * BF16 weights and activations, FP32 accumulation (MFMA), FP32 master
 * weights and Adam.  Parameters are library-owned: FP32, layer by layer,
 * W_l (widths[l+1] x widths[l], row-major) then b_l (widths[l+1]).
 * Device pointers (x, t, w, y, loss, grad) are caller-owned, row-major.
 * ---------------------------------------------------------------------- */
typedef struct lbw_mlp* lbw_mlp_t;

/* Zero parameters; max_batch bounds B of every later call.  Errors:
 * LBW_EINVAL (n_layers outside [1, 16], a width outside [1, 4096],
 * max_batch < 1), LBW_ENOMEM. */
int lbw_mlp_create(const int32_t* widths, int n_layers, int max_batch, void* stream, lbw_mlp_t* out);
int lbw_mlp_param_count(lbw_mlp_t m, int64_t* count);
/* Copies host FP32 parameters in (and resets the Adam state) / out.  Synchronises. */
int lbw_mlp_set_params(lbw_mlp_t m, const float* host_params);
int lbw_mlp_get_params(lbw_mlp_t m, float* host_params);
/* y[B, widths[L]] = network(x[B, widths[0]]) (device, FP32). */
int lbw_mlp_forward(lbw_mlp_t m, const float* x, int B, float* y);
/* Loss sum_ij w_ij (y_ij - t_ij)^2 / weight_sum (w may be NULL: all 1) and
 * its gradient with respect to the FP32 parameters, kept for
 * lbw_mlp_adam_step; loss (1 float) and grad (param_count floats) receive
 * copies when not NULL. */
int lbw_mlp_loss_grad(lbw_mlp_t m, const float* x, const float* t, const float* w, int B, float weight_sum,
                      float* loss, float* grad);
/* One Adam step (bias-corrected) on the last gradient.  Errors: LBW_ESTATE
 * before any lbw_mlp_loss_grad, LBW_EINVAL for bad hyper-parameters. */
int lbw_mlp_adam_step(lbw_mlp_t m, float lr, float beta1, float beta2, float eps);
/* steps full-batch training steps (lbw_mlp_loss_grad then lbw_mlp_adam_step)
 * on the same x, t, w, with the cosine learning rate
 * lr (1 + cos(pi s / steps)) / 2 + lr_floor at step s = 0 .. steps-1 of this
 * call, continuing the network's Adam state.  The rate and the bias
 * corrections are computed on the device from a step counter, in double as
 * a host would, and one step is captured once into a HIP graph and replayed
 * (no per-step host work).  loss (device, 1 float, may be NULL) receives the
 * loss of the last step's forward pass.  Synchronises.  Errors as
 * lbw_mlp_loss_grad and lbw_mlp_adam_step; steps < 1 is LBW_EINVAL. */
int lbw_mlp_train(lbw_mlp_t m, const float* x, const float* t, const float* w, int B, float weight_sum, int steps,
                  double lr, double lr_floor, float beta1, float beta2, float eps, float* loss);
int lbw_mlp_free(lbw_mlp_t m);

/* Message of the calling thread's last error ("" if none). */
const char* lbw_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBW_H */
