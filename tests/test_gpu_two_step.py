"""Two time steps per launch against one-step launches and the oracle.

The two-step pass holds the state at t+1 on chip and runs the one-step
kernel's per-node arithmetic (the same collide() code) in the same order,
so every population and every probe value must equal the one-step result
bit for bit: on the benchmark's geometries (coarse), on grids with walls of
every kind along axis 1 and axis 2, periodic axes shorter than a tile, rows
narrower than the tile, ragged last tiles, chunk boundaries, odd step
counts (the last step runs alone) and graph-captured blocks.
"""
import math
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


def run(geom, P0, probes, steps, two=None, one=None, graph=None, tmax=None):
    g = lbw.Geometry(geom)
    if one:
        g.set_step_config(*one)
    if two:
        g.set_step2_config(*two)
    sim = lbw.Simulation(g, P0, probes, t_max=steps if tmax is None else tmax)
    if graph is not None:
        sim.set_graph_block(graph)
    sim.step(steps)
    f = sim.populations().cpu().numpy().copy()
    tr = sim.probe()
    assert sim.t == steps
    return f, tr, g


CASES = {
    "cylinder": W.closed_cylinder(scale=4),
    "horn": W.trumpet_horn(scale=4),
    "torus": W.torus(scale=4),
    # axis 1 walled (free, fixed), axis 2 walled with damping, n1 not a multiple of the tile height
    "box_walls": dict(kind="box", dim=3, n=(37, 13, 29), qmin=(0, 0, 0), qmax=(37.0, 11.7, 34.8),
                      bc_lo=("bounceback", "free", "fixed"), bc_hi=("fixed", "bounceback", "free"), h_ref=1.0,
                      c=0.33, damp=0.9, params=()),
    # periodic axes shorter than the tile and than the chunk extension
    "cyl_short": dict(W.closed_cylinder(scale=1), n=(50, 3, 2), bc_lo=("free", "periodic", "periodic"),
                      bc_hi=("bounceback", "periodic", "periodic"), qmax=(1.0, 2 * math.pi, 0.1)),
    # one plane along axis 2, walled
    "cyl_flat": dict(W.closed_cylinder(scale=1), n=(20, 9, 1), qmax=(1.0, 2 * math.pi, 0.05)),
    # axis 1 walled, axis 2 periodic (the kernel variant with only the axis-2 wall rules compiled out)
    "box_walls_zper": dict(kind="box", dim=3, n=(41, 11, 23), qmin=(0, 0, 0), qmax=(41.0, 9.9, 27.6),
                           bc_lo=("free", "fixed", "periodic"), bc_hi=("bounceback", "free", "periodic"),
                           h_ref=1.0, c=0.33, damp=0.85, params=()),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_two_step_bit_identical_to_one_step(name):
    geom = CASES[name]
    N = W.num_nodes(geom)
    rng = np.random.default_rng(11)
    P0 = rng.uniform(-1, 1, N)
    probes = np.unique(rng.integers(0, N, 12))
    steps = 41
    say("two-step", name, geom["n"])
    ref, tr_ref, _ = run(geom, P0, probes, steps)
    n0 = geom["n"][0]
    # (chunk_z 0: balanced shares of the (row tile, plane) pairs, with
    # shares that split row tiles and, at 24 workgroups, many segments)
    shapes = [(96, 6, lz, b) for lz, b in ((16, 0), (5, 8), (64, 16), (0, 0), (0, 24))] if n0 <= 96 else []
    shapes += [(128, 4, lz, b) for lz, b in ((16, 0), (3, 8), (32, 0), (0, 0), (0, 8))]
    for shape in shapes:
        for graph in (0, 32, 7):
            f, tr, g = run(geom, P0, probes, steps, two=shape, graph=graph)
            assert g.step2_config()[:2] == shape[:2]
            assert np.array_equal(f, ref), (name, shape, graph)
            assert np.array_equal(tr, tr_ref), (name, shape, graph)


def test_two_step_matches_oracle_and_keeps_trace_rows():
    w = W.workload(3, scale=4)
    geom, P0, probes = w["geom"], w["P0"], w["probes"]
    say("two-step vs oracle", w["name"], geom["n"])
    f, tr, _ = run(geom, P0, probes, 200, two=(96, 6, 16, 0), tmax=150)
    o = oracle.Oracle(geom)
    fo, tro = o.run(o.init(P0), 200, probes)
    assert np.linalg.norm(f - fo) / np.linalg.norm(fo) <= 1e-5
    assert tr.shape == (150, len(probes))
    assert np.abs(tr - tro[:150]).max() <= 1e-5 * np.abs(tro).max()


def test_two_step_refuses_what_it_does_not_fit():
    g = lbw.Geometry(dict(W.closed_cylinder(scale=1), n=(130, 8, 8)))
    with pytest.raises(lbw.LbwError):
        g.set_step2_config(128, 4, 16, 0)                   # rows longer than the tile
    g2 = lbw.Geometry(CASES["box_walls"])
    for bad in [(96, 8, 16, 0), (64, 4, 16, 0), (96, 6, -1, 0), (128, 6, 16, 0)]:
        with pytest.raises(lbw.LbwError):
            g2.set_step2_config(*bad)
    g2.set_step2_config(96, 6, 16, 0)
    assert g2.step2_config()[0] == 96
    g2.set_step_config(32, 8, 16, 0)                         # a one-step shape turns it off
    assert g2.step2_config() == (0, 0, 0, 0)


def test_two_step_with_sources_runs_one_step_launches():
    geom = CASES["cylinder"]
    N = W.num_nodes(geom)
    P0 = np.zeros(N)
    src = [3, 77]
    out = []
    for two in (None, (128, 4, 16, 0)):
        g = lbw.Geometry(geom)
        if two:
            g.set_step2_config(*two)
        sim = lbw.Simulation(g, P0, [5, 900], t_max=60)
        sim.set_sources(src, 0.7, 0.11)
        sim.step(60)
        out.append((sim.populations().cpu().numpy().copy(), sim.probe()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_autotune_may_pick_two_step_and_results_stay():
    w = W.workload(2, scale=2)
    geom, P0, probes = w["geom"], w["P0"], w["probes"]
    say("autotune two-step", w["name"], geom["n"])
    ref, tr_ref, _ = run(geom, P0, probes, 64)
    g = lbw.Geometry(geom)
    sim = lbw.Simulation(g, P0, probes, t_max=64)
    sim.step(10)
    before = sim.populations().cpu().numpy().copy()
    us = sim.autotune(reps=3)
    assert us > 0 and sim.t == 10
    assert np.array_equal(sim.populations().cpu().numpy(), before)
    say("  picked", g.step_config(), g.step2_config(), "%.1f us/step" % us)
    sim.step(54)
    assert np.array_equal(sim.populations().cpu().numpy(), ref)
    assert np.array_equal(sim.probe(), tr_ref)
