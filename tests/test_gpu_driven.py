"""GPU: driven sources and response intensity against the FP64 oracle.

Sources impose amplitude * sin(omega t) at chosen nodes before every step,
as a pressure (Sec. IV.A and IV.C ring and point sources) or as the flux
J'_a of an oscillating plate (Sec. IV.A); the intensity is the largest
|P| per probe over a late window (the frequency sweeps).  The HIP path
keeps populations in FP32, so fields and traces are compared with the field
tolerance of the undriven parity tests (relative L2 1e-5); a probe on a
source node must read the imposed value to FP32 rounding; a batch of copies
driven at different frequencies must match each copy driven alone bit for
bit (same per-node arithmetic; a batch imposes the sources in its step
kernel as it loads the populations, or by a launch of their own where they
span most planes, a single run by that launch, all through the same
per-node rule), and graph replay must match step-by-step launches.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_1705_01801_amd as lbw
import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def cyl():
    geom = W.closed_cylinder(scale=16, c=0.35)      # 8 x 8 x 16, sqrt(g) = r varies
    n0, n1 = geom["n"][0], geom["n"][1]
    ring = [0 + n0 * (i1 + n1 * 0) for i1 in range(n1)]
    src = ring + [5 + n0 * (3 + n1 * 7)]
    probes = [ring[2], src[-1], 4 + n0 * (6 + n1 * 12), 7 + n0 * (1 + n1 * 15)]
    return dict(geom, damp=0.65), src, probes


@pytest.mark.parametrize("case", ["cylinder", "polar2d", "box2d_point"])
def test_driven_run_matches_oracle(case):
    C, w, T = 0.8, 0.07, 300
    if case == "cylinder":
        geom, src, probes = cyl()
    elif case == "box2d_point":                       # the Cartesian point source, 100 x 100
        geom, src, w = W.point_source_box()
        n = geom["n"][0]
        probes = [src[0], src[0] + 7, src[0] + 20 * n, 5 + 5 * n]
        T = 150
    else:
        geom = dict(W.polar_disk(scale=4), damp=0.65)  # 16 x 16, D2Q5 kernel
        n0 = geom["n"][0]
        src = [0 + n0 * i1 for i1 in range(geom["n"][1])]
        probes = [src[3], 9 + n0 * 4, 14 + n0 * 11]
    say("driven", case, W.shape_of(geom), "sources", len(src), "steps", T)
    o = oracle.Oracle(geom)
    f = o.init(np.zeros(o.N))
    _, tr_o = o.run(f, T, probes, sources=src, amplitude=C, omega=w)
    sim = lbw.Simulation(lbw.Geometry(geom), np.zeros(o.N), probes, t_max=T)
    sim.set_sources(src, C, w)
    sim.step(T)                                       # graph blocks of 32 plus single launches
    fg = sim.populations().double().cpu().numpy()
    assert rel_l2(fg, f) <= 1e-5
    tr = sim.probe()
    assert np.abs(tr - tr_o).max() <= 1e-5 * np.abs(tr_o).max()
    # the source probe reads the imposed pressure (FP32 populations)
    assert np.abs(tr[:, 0] - C * np.sin(w * np.arange(T))).max() <= 2e-6 * C
    a = sim.amplitude(T - 100, T)
    assert np.abs(a - o.amplitude(tr_o, T - 100, T)).max() <= 1e-5 * a.max()
    assert np.array_equal(a, np.abs(tr[T - 100:]).max(axis=0))


@pytest.mark.parametrize("case", ["cylinder_plate", "polar2d_radial", "general_duct"])
def test_flux_run_matches_oracle(case):
    if case == "cylinder_plate":
        geom, _, probes = cyl()
        n0, n1 = geom["n"][0], geom["n"][1]
        src, axis = list(range(n0 * n1)), 2               # the whole z = 0 plane
    elif case == "polar2d_radial":
        geom = dict(W.polar_disk(scale=4), damp=0.65)
        n0 = geom["n"][0]
        src, axis = [3 + n0 * i1 for i1 in range(geom["n"][1])], 0
        probes = [src[2], 9 + n0 * 4, 14 + n0 * 11]
    else:
        geom = W.general_duct(n=(12, 10, 16))
        geom = dict(geom, coeffs=W.general_coefficients(geom))
        n0, n1 = geom["n"][0], geom["n"][1]
        src, axis = [4 + n0 * (i1 + n1 * 3) for i1 in range(2, 8)], 1
        probes = [src[0], 7 + n0 * (5 + n1 * 9), 2 + n0 * (8 + n1 * 14)]
    C, w, T = 0.8, 0.07, 300
    say("flux", case, W.shape_of(geom), "sources", len(src), "axis", axis, "steps", T)
    o = oracle.Oracle(geom)
    f = o.init(np.zeros(o.N))
    _, tr_o = o.run(f, T, probes, sources=src, amplitude=C, omega=w, flux_axis=axis)
    assert np.abs(tr_o).max() > 1e-2
    sim = lbw.Simulation(lbw.Geometry(geom), np.zeros(o.N), probes, t_max=T)
    sim.set_sources(src, C, w, flux_axis=axis)
    sim.step(T)
    assert rel_l2(sim.populations().double().cpu().numpy(), f) <= 1e-5
    tr = sim.probe()
    assert np.abs(tr - tr_o).max() <= 1e-5 * np.abs(tr_o).max()


def test_sources_graph_replay_and_removal():
    geom, src, probes = cyl()
    T = 150
    out = []
    for block in (0, 16):
        sim = lbw.Simulation(lbw.Geometry(geom), np.zeros(W.num_nodes(geom)), probes, t_max=2 * T)
        sim.set_graph_block(block)
        sim.set_sources(src, 1.0, 0.11)
        sim.step(T)
        sim.set_sources([], 0.0, 0.0)                 # then free ringing
        sim.step(T)
        out.append((sim.populations().cpu().numpy(), sim.probe()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    o = oracle.Oracle(geom)
    f = o.init(np.zeros(o.N))
    _, t1 = o.run(f, T, probes, sources=src, amplitude=1.0, omega=0.11)
    _, t2 = o.run(f, T, probes, t0=T)
    ref = np.vstack([t1, t2])
    assert np.abs(out[0][1] - ref).max() <= 1e-5 * np.abs(ref).max()


def test_batch_sweep_matches_single_runs():
    geom, src, probes = cyl()
    omegas = [0.02, 0.05, 0.09, 0.13]
    T = 200
    n = len(omegas) + 1                               # the last copy is not driven
    N = W.num_nodes(geom)
    say("driven batch of", n)
    b = lbw.Batch([geom] * n, [np.zeros(N)] * n, [probes] * n, t_max=T)
    b.set_graph_block(16)
    nodes = np.concatenate([src] * len(omegas))
    which = np.repeat(np.arange(len(omegas)), len(src))
    b.set_sources(nodes, which, 0.6, np.repeat(omegas, len(src)))
    b.step(T)
    trace = b.probe()
    amp = b.amplitude(T // 2, T)
    for h in range(n):
        sim = lbw.Simulation(lbw.Geometry(geom), np.zeros(N), probes, t_max=T)
        if h < len(omegas):
            sim.set_sources(src, 0.6, omegas[h])
        sim.step(T)
        assert np.array_equal(b.populations(h).cpu().numpy(), sim.populations().cpu().numpy()), h
        cols = slice(int(b.probe_offsets[h]), int(b.probe_offsets[h + 1]))
        assert np.array_equal(trace[:, cols], sim.probe()), h
        assert np.array_equal(amp[cols], np.abs(sim.probe()[T // 2:]).max(axis=0)), h
    assert not trace[:, -len(probes):].any()          # the undriven copy stays at rest


def test_batch_mixes_source_kinds():
    """Ring (pressure) and plate (flux) copies in one batch, each equal bit
    for bit to the same copy driven alone."""
    geom, src, probes = cyl()
    n0, n1 = geom["n"][0], geom["n"][1]
    plate = list(range(n0 * n1))
    cases = [(src, -1, 0.05), (plate, 2, 0.05), (plate, 2, 0.11), (src[:3], 1, 0.08)]
    N, T = W.num_nodes(geom), 160
    say("mixed-kind batch of", len(cases))
    b = lbw.Batch([geom] * len(cases), [np.zeros(N)] * len(cases), [probes] * len(cases), t_max=T)
    b.set_sources(np.concatenate([c[0] for c in cases]), np.repeat(np.arange(len(cases)), [len(c[0]) for c in cases]),
                  0.7, np.repeat([c[2] for c in cases], [len(c[0]) for c in cases]),
                  np.repeat([c[1] for c in cases], [len(c[0]) for c in cases]))
    b.step(T)
    trace = b.probe()
    for h, (nodes, axis, w) in enumerate(cases):
        sim = lbw.Simulation(lbw.Geometry(geom), np.zeros(N), probes, t_max=T)
        sim.set_sources(nodes, 0.7, w, None if axis < 0 else axis)
        sim.step(T)
        assert np.array_equal(b.populations(h).cpu().numpy(), sim.populations().cpu().numpy()), h
        cols = slice(int(b.probe_offsets[h]), int(b.probe_offsets[h + 1]))
        assert np.array_equal(trace[:, cols], sim.probe()), h


def test_whole_section_tiles_match_wide_tiles():
    """Small cross-sections (pipe 20 x 5, cylinder 8 x 8) default to
    whole-section tiles; the same batch on 32-wide tiles, and on whole
    sections with ragged chunks of 7 planes, gives identical bits (same
    per-node arithmetic, only the lane mapping differs)."""
    geoms = [W.driven_pipe("fixed"), W.driven_pipe("free"), cyl()[0]] * 2
    N = [W.num_nodes(g) for g in geoms]
    rng = np.random.default_rng(5)
    P0 = [rng.uniform(-1, 1, n) for n in N]
    probes = [[0, 7, n - 1] for n in N]
    ring = W.pipe_ring(geoms[0])
    out = []
    for shape in (None, (32, 16, 0), (0, 7, 0)):
        b = lbw.Batch(geoms, P0, probes, t_max=200)
        if shape is None:
            assert b.step_config()[0] == 0                 # whole sections by default
        else:
            b.set_step_config(*shape)
        b.set_graph_block(16)
        b.set_sources(np.concatenate([ring, ring]), np.repeat([0, 3], ring.size), 0.5, 0.02)
        say("batch launch shape", b.step_config())
        b.step(200)
        out.append(([b.populations(h).cpu().numpy() for h in range(len(geoms))], b.probe()))
    for pops, tr in out[1:]:
        for h in range(len(geoms)):
            assert np.array_equal(pops[h], out[0][0][h]), h
        assert np.array_equal(tr, out[0][1])


def test_batch_autotune_with_sources_changes_nothing():
    """Tuning a driven batch (as the sweeps do) imposes no source and records
    no probe: populations, step count and trace stay as they were, and the
    run continues bit for bit as an untuned one."""
    geom, src, probes = cyl()
    N = W.num_nodes(geom)
    out = []
    for tune in (False, True):
        b = lbw.Batch([geom] * 3, [np.zeros(N)] * 3, [probes] * 3, t_max=120)
        b.set_sources(np.concatenate([src] * 3), np.repeat(np.arange(3), len(src)), 0.5, [0.03] * len(src) * 3)
        b.step(20)
        if tune:
            before = [b.populations(h).cpu().numpy().copy() for h in range(3)]
            tr = b.probe().copy()
            assert b.autotune(reps=2) > 0 and b.t == 20
            for h in range(3):
                assert np.array_equal(b.populations(h).cpu().numpy(), before[h])
            assert np.array_equal(b.probe(), tr)
        b.step(100)
        out.append(([b.populations(h).cpu().numpy() for h in range(3)], b.probe()))
    for h in range(3):
        assert np.array_equal(out[0][0][h], out[1][0][h])
    assert np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("spread", ["every_plane", "two_planes"])
def test_driven_nodes_anywhere_in_the_tile_walk(spread):
    """A batch imposes its sources either in the step kernel, on the
    populations it loads (where the driven planes are a small part of the
    batch's planes: a node's own column, the ring of a neighbouring tile, a
    chunk's first and last planes, the periodic axis-2 seam), or by a launch
    of their own before every step (where they span most planes).  A torus
    (periodic axes 1 and 2) and a cylinder with driven nodes scattered over
    every plane (the separate launch), or over the two planes either side of
    a chunk boundary (the step kernel), pressure and flux kinds, several on
    probe nodes, give the same bits as each copy driven alone, on four
    launch shapes."""
    rng = np.random.default_rng(17)
    geoms = [W.torus(scale=16), cyl()[0], W.torus(scale=16)]
    N = [W.num_nodes(g) for g in geoms]
    srcs, kinds, omegas, probes = [], [-1, 2, 1], [0.07, 0.05, 0.12], []
    for g, n in zip(geoms, N):
        n0, n1, n2 = g["n"]
        plane = n0 * n1
        zs = range(n2) if spread == "every_plane" else (n2 // 2 - 1, n2 // 2)
        # two nodes on each chosen plane (ring positions included: x = 0,
        # n0 - 1; y = 0, n1 - 1) and the whole x = 0 column of the first and
        # last chosen planes
        nodes = set()
        for z in zs:
            nodes.update(int(v) for v in rng.choice(plane, size=2, replace=False) + z * plane)
        for z in (zs[0], zs[-1]):
            nodes.update(z * plane + n0 * y for y in range(n1))
        nodes = np.array(sorted(nodes), dtype=np.int64)
        srcs.append(nodes)
        probes.append(np.concatenate([nodes[:3], rng.choice(n, size=3, replace=False)]))
    T = 120
    singles = []
    for h, g in enumerate(geoms):
        sim = lbw.Simulation(lbw.Geometry(g), np.zeros(N[h]), probes[h], t_max=T)
        sim.set_sources(srcs[h], 0.6, omegas[h], None if kinds[h] < 0 else kinds[h])
        sim.step(T)
        singles.append((sim.populations().cpu().numpy(), sim.probe()))
    for shape in (None, (16, 5, 0), (32, 3, 0), (64, 32, 0)):
        b = lbw.Batch(geoms, [np.zeros(n) for n in N], probes, t_max=T)
        if shape is not None:
            b.set_step_config(*shape)
        b.set_graph_block(8)
        which = np.repeat(np.arange(len(geoms)), [len(x) for x in srcs])
        b.set_sources(np.concatenate(srcs), which, 0.6, np.repeat(omegas, [len(x) for x in srcs]),
                      np.repeat(kinds, [len(x) for x in srcs]))
        say("driven nodes", spread, "launch shape", b.step_config())
        b.step(T)
        trace = b.probe()
        for h in range(len(geoms)):
            assert np.array_equal(b.populations(h).cpu().numpy(), singles[h][0]), (shape, h)
            cols = slice(int(b.probe_offsets[h]), int(b.probe_offsets[h + 1]))
            assert np.array_equal(trace[:, cols], singles[h][1]), (shape, h)


def test_source_errors():
    geom, src, probes = cyl()
    N = W.num_nodes(geom)
    sim = lbw.Simulation(lbw.Geometry(geom), np.zeros(N), probes, t_max=10)
    with pytest.raises(lbw.LbwError):
        sim.set_sources([N], 1.0, 0.1)
    with pytest.raises(lbw.LbwError):
        sim.set_sources([-1], 1.0, 0.1)
    with pytest.raises(lbw.LbwError):
        sim.set_sources([0], float("nan"), 0.1)
    with pytest.raises(lbw.LbwError):
        sim.set_sources([0], 1.0, 0.1, flux_axis=3)     # no fourth axis
    with pytest.raises(lbw.LbwError):
        sim.set_sources([0], 1.0, 0.1, flux_axis=-2)
    disk = lbw.Geometry(W.polar_disk(scale=4))
    with pytest.raises(lbw.LbwError):
        lbw.Simulation(disk, np.zeros(disk.N)).set_sources([0], 1.0, 0.1, flux_axis=2)
    with pytest.raises(lbw.LbwError):
        sim.amplitude(0, 1)                          # nothing recorded yet
    sim.step(4)
    with pytest.raises(lbw.LbwError):
        sim.amplitude(2, 2)
    with pytest.raises(lbw.LbwError):
        sim.amplitude(0, 5)
    b = lbw.Batch([geom] * 2, [np.zeros(N)] * 2, [probes] * 2, t_max=10)
    with pytest.raises(lbw.LbwError):
        b.set_sources([0], [2], 1.0, 0.1)
    with pytest.raises(lbw.LbwError):
        b.set_sources([N], [1], 1.0, 0.1)
    with pytest.raises(lbw.LbwError):
        b.set_sources([0], [1], 1.0, 0.1, flux_axis=3)
    with pytest.raises(lbw.LbwError):
        b.set_sources([5, 3, 5], [1, 1, 1], 1.0, 0.1)   # node 5 of geometry 1 twice
    b.set_sources([5, 5], [0, 1], 1.0, 0.1)             # the same node of two geometries


def test_pipe_sweep_point_full_size():
    """One point of the pipe sweep at its full size and length (8400 steps),
    batched with two other drive frequencies, against the oracle.  FP32
    rounding (6e-8 per step) accumulates at most linearly over the run:
    tolerance 8400 x 6e-8 ~ 5e-4 relative."""
    geom = W.driven_pipe("fixed")
    ring, probes = W.pipe_ring(geom), W.pipe_probes(geom)
    N, T = W.num_nodes(geom), W.PIPE_STEPS
    omegas = [0.004, 0.00785, 0.0123]
    say("pipe sweep point, batch of", len(omegas), "steps", T)
    b = lbw.Batch([geom] * 3, [np.zeros(N)] * 3, [probes] * 3, t_max=T)
    b.set_sources(np.concatenate([ring] * 3), np.repeat(np.arange(3), len(ring)), 1.0,
                  np.repeat(omegas, len(ring)))
    b.step(T)
    amp = b.amplitude(T // 2, T).reshape(3, len(probes))
    tr = b.probe()[:, len(probes):2 * len(probes)]
    o = oracle.Oracle(geom)
    f = o.init(np.zeros(o.N))
    _, tr_o = o.run(f, T, probes, sources=ring, amplitude=1.0, omega=omegas[1])
    assert np.abs(tr - tr_o).max() <= 5e-4 * np.abs(tr_o).max()
    a_o = o.amplitude(tr_o, T // 2, T)
    assert np.abs(amp[1] - a_o).max() <= 5e-4 * a_o.max()
    assert rel_l2(b.populations(1).double().cpu().numpy(), f) <= 5e-4


def test_torus_sweep_points_match_oracle():
    """Three points of the torus sweep (Sec. IV.C small ring, 20 x 200 x 30,
    M^phiphi up to 39 near rho_min) batched, 600 steps, the middle one
    against the oracle; FP32 rounding over 600 steps: 600 x 6e-8 ~ 4e-5."""
    geom = W.driven_torus()
    ring = W.torus_sources(geom)["small_ring"]
    probes = np.concatenate([W.torus_probes(geom), ring[[3, 10]] + 2])   # two probes near the ring
    N, T = W.num_nodes(geom), 600
    omegas = [0.03, 0.071, 0.2]
    say("torus sweep points, batch of", len(omegas), "steps", T)
    b = lbw.Batch([geom] * 3, [np.zeros(N)] * 3, [probes] * 3, t_max=T)
    b.set_sources(np.concatenate([ring] * 3), np.repeat(np.arange(3), ring.size), 1.0, np.repeat(omegas, ring.size))
    b.step(T)
    tr = b.probe()[:, len(probes):2 * len(probes)]
    o = oracle.Oracle(geom)
    f = o.init(np.zeros(o.N))
    _, tr_o = o.run(f, T, probes, sources=ring, amplitude=1.0, omega=omegas[1])
    assert np.abs(tr_o).max() > 1e-3
    assert np.abs(tr - tr_o).max() <= 5e-5 * np.abs(tr_o).max()
    assert rel_l2(b.populations(1).double().cpu().numpy(), f) <= 5e-5


def test_radial_wave_matches_oracle():
    """The radial wave of the oracle pin (polar grid 199 x 4, ring drive,
    400 steps) through the 2-D kernel."""
    import math
    n0, nth = 199, 4
    geom = dict(kind="polar2d", dim=2, n=(n0, nth), qmin=(1.0, 0.0), qmax=(1.0 + n0, 2 * math.pi),
                bc_lo=("bounceback", "periodic"), bc_hi=("bounceback", "periodic"), h_ref=1.0, c=0.5, damp=1.0,
                params=())
    src = [n0 * i for i in range(nth)]
    o = oracle.Oracle(geom)
    f = o.init(np.zeros(o.N))
    o.run(f, 400, [], sources=src, amplitude=1.0, omega=0.075)
    sim = lbw.Simulation(lbw.Geometry(geom), np.zeros(o.N), [5, 50], t_max=400)
    sim.set_sources(src, 1.0, 0.075)
    sim.step(400)
    assert rel_l2(sim.populations().double().cpu().numpy(), f) <= 1e-5
