"""GPU: batches of geometries advanced by one launch per step.

Every geometry of a batch runs the same per-node arithmetic as a geometry
stepped alone, so states and traces must be bit-identical to the
single-geometry path; one member is also compared with the FP64 oracle.
Spectra from the batch call equal those of the single-geometry call on the
same traces.
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


def members():
    geoms = [
        W.trumpet_horn(c=0.3, a=0.08, b=0.01, k=2.0, n=(32, 32, 64)),
        W.trumpet_horn(c=0.25, a=0.15, b=0.03, k=4.0, n=(48, 40, 80)),
        W.trumpet_horn(c=0.3, a=0.1, b=0.02, k=3.0, n=(96, 64, 48)),
        dict(W.closed_cylinder(c=0.4), n=(40, 24, 33)),
        dict(W.torus(c=0.1), n=(20, 32, 48)),
        dict(kind="box", dim=3, n=(70, 11, 37), qmin=(0, 0, 0), qmax=(70.0, 8.8, 48.1),
             bc_lo=("periodic", "fixed", "periodic"), bc_hi=("periodic", "free", "periodic"), h_ref=1.0,
             c=0.35, damp=0.9, params=()),
    ]
    rng = np.random.default_rng(21)
    P0s, probes = [], []
    for i, g in enumerate(geoms):
        N = W.num_nodes(g)
        P0s.append(rng.uniform(-1, 1, N))
        probes.append(rng.integers(0, N, size=[3, 0, 5, 1, 4, 2][i]))
    return geoms, P0s, probes


def test_batch_matches_single_geometries_bit_for_bit():
    geoms, P0s, probes = members()
    steps = 90
    say("batch of", len(geoms))
    b = lbw.Batch(geoms, P0s, probes, t_max=steps)
    b.set_graph_block(16)
    b.step(steps)
    trace = b.probe()
    for h, g in enumerate(geoms):
        sim = lbw.Simulation(lbw.Geometry(g), P0s[h], probes[h], t_max=steps)
        sim.step(steps)
        fb = b.populations(h).cpu().numpy()
        fs = sim.populations().cpu().numpy()
        assert np.array_equal(fb, fs), h
        cols = slice(int(b.probe_offsets[h]), int(b.probe_offsets[h + 1]))
        if len(probes[h]):
            assert np.array_equal(trace[:, cols], sim.probe()), h


def test_batch_member_matches_oracle():
    geoms, P0s, probes = members()
    steps = 200
    b = lbw.Batch(geoms, P0s, probes, t_max=steps)
    b.step(steps)
    for h in (2, 4):
        say("batch vs oracle", h)
        o = oracle.Oracle(geoms[h])
        f, tr = o.run(o.init(P0s[h]), steps, probes[h])
        fb = b.populations(h).double().cpu().numpy()
        assert np.linalg.norm(fb - f) / np.linalg.norm(f) <= 1e-5
        cols = slice(int(b.probe_offsets[h]), int(b.probe_offsets[h + 1]))
        assert np.abs(b.probe()[:, cols] - tr).max() <= 1e-5 * np.abs(tr).max()


def test_batch_launch_shapes_autotune_graphs_identical():
    geoms, P0s, probes = members()
    ref = None
    for cfg in [(32, 16, 0), (64, 5, 8), (32, 64, 24), "tune"]:
        say("batch shape", cfg)
        b = lbw.Batch(geoms, P0s, probes, t_max=70)
        b.step(3)
        if cfg == "tune":
            before = b.populations(2).cpu().numpy().copy()
            assert b.autotune(reps=2) > 0 and b.t == 3
            assert np.array_equal(b.populations(2).cpu().numpy(), before)
            b.set_graph_block(7)
        else:
            b.set_step_config(*cfg)
            b.set_graph_block(0)
        b.step(67)
        out = [b.populations(h).cpu().numpy().copy() for h in range(len(geoms))], b.probe()
        if ref is None:
            ref = out
        else:
            for x, y in zip(out[0], ref[0]):
                assert np.array_equal(x, y)
            assert np.array_equal(out[1], ref[1])


def test_batch_modes_equal_single_modes():
    geoms, P0s, probes = members()
    steps = 600
    b = lbw.Batch(geoms, P0s, probes, t_max=steps)
    b.step(steps)
    k = 6
    fb, pb = b.modes(k)
    for h, g in enumerate(geoms):
        if not len(probes[h]):
            assert np.isnan(fb[h]).all()
            continue
        sim = lbw.Simulation(lbw.Geometry(g), P0s[h], probes[h], t_max=steps)
        sim.step(steps)
        fs, ps = sim.modes(k)
        assert np.array_equal(np.isnan(fs), np.isnan(fb[h]))
        ok = ~np.isnan(fs)
        assert np.array_equal(fs[ok], fb[h][ok]) and np.array_equal(ps[ok], pb[h][ok])
        fo, _ = oracle.modes(sim.probe(), k)
        assert np.abs(fs[ok] / fo[ok] - 1).max() <= 1e-10


def test_batch_launch_shapes_and_graphs_identical():
    """Launch shapes and graph blocks change nothing (no autotuning)."""
    geoms, P0s, probes = members()
    ref = None
    for cfg, block in [((32, 16, 0), 0), ((64, 5, 8), 16), ((32, 64, 24), 7), ((16, 16, 0), 32), ((16, 9, 16), 5),
                       ((0, 16, 0), 8), ((0, 5, 16), 3)]:
        say("batch shape", cfg, block)
        b = lbw.Batch(geoms, P0s, probes, t_max=70)
        b.set_step_config(*cfg)
        b.set_graph_block(block)
        b.step(70)
        out = [b.populations(h).cpu().numpy().copy() for h in range(len(geoms))], b.probe()
        if ref is None:
            ref = out
        else:
            for x, y in zip(out[0], ref[0]):
                assert np.array_equal(x, y)
            assert np.array_equal(out[1], ref[1])


def test_batch_rejects_bad_input():
    geoms, P0s, probes = members()
    bad = [list(p) for p in probes]
    bad[2] = [W.num_nodes(geoms[2])]
    with pytest.raises(lbw.LbwError):
        lbw.Batch(geoms, P0s, bad, t_max=10)
    with pytest.raises(lbw.LbwError):
        lbw.Batch([W.polar_disk()], [np.zeros(64 * 64)], [[0]], t_max=10)
