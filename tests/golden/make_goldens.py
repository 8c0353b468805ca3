"""Writes the stored oracle results that the full-size GPU parity tests use.

Calls only the FP64 oracle (``oracle/``) on the seeded inputs of
``workloads``; nothing here comes from the HIP library.  Run from the
repository root (one process per case, CPU only):

    python tests/golden/make_goldens.py full 1 2 3     # 1000 steps, full grids
    python tests/golden/make_goldens.py modes 1 2 3    # 4x coarser grids, configured step counts
    python tests/golden/make_goldens.py ensemble 80 222 # training-ensemble horns, configured run
    python tests/golden/make_goldens.py full 4          # the duct given by its metric, 1000 steps
    python tests/golden/make_goldens.py sweep 0         # one torus sweep point, full length

Files (numpy .npz, no pickled objects):

* ``full_<name>_1000.npz``: ``trace`` (1000 x probes, FP64 pressure at every
  probe before each step), ``nodes`` (65,536 distinct node indices drawn
  with a seeded generator), ``f`` (7 x 65,536: the populations at those
  nodes after 1000 steps, stored as float32, whose rounding is 6e-8
  relative, far below the 1e-5 bar), ``invariant`` (sum of all populations
  = sum sqrt(g) P at t = 0 and t = 1000) and ``input_digest`` (SHA-256 of
  the geometry description, P0 and the probes, so a changed input is caught);
* ``modes_<name>_coarse4.npz``: ``freq``, ``power`` (the first 10 spectral
  peaks of the probe traces by the oracle's extractor, cycles per step),
  ``steps``, ``input_digest``, and ``norm`` (L2 norm of the populations at
  t = 0 and at the end);
* ``ensemble_<i>.npz``: horn i of the training ensemble on its own grid,
  with c = 0.9 of the frozen-coefficient stability bound computed from the
  oracle's coefficients (c^2 rounded down to a multiple of 2^-16), run from
  the plane pulse for the configured 30,000 steps: ``c``, ``freq`` and
  ``power`` (the first 10 spectral peaks of its 8 probes, cycles per step),
  ``trace`` (every 10th row of the probe traces), ``input_digest``;
* ``sweep_torus_small_ring.npz``: one point of the torus sweep (the small
  ring driven at omega = 0.071 rad/step from rest) over the sweep's full
  length: ``trace`` (every 10th row), ``amplitude`` (largest |P| per probe
  over the second half), ``nodes`` / ``f`` (populations at 16,384 seeded
  nodes at the end, float32), ``sources``, ``omega``, ``input_digest``.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
FULL_STEPS = 1000
SAMPLE = 65536
MODES_K = 10
COARSE = 4


def input_digest(w) -> str:
    h = hashlib.sha256()
    geom = {k: v for k, v in w["geom"].items() if k != "coeffs"}
    h.update(json.dumps(geom, sort_keys=True, default=float).encode())
    if "coeffs" in w["geom"]:                     # a geometry given by its metric: the per-node planes
        h.update(np.ascontiguousarray(w["geom"]["coeffs"], dtype=np.float64).tobytes())
    h.update(np.ascontiguousarray(w["P0"], dtype=np.float64).tobytes())
    h.update(np.ascontiguousarray(w["probes"], dtype=np.int64).tobytes())
    return h.hexdigest()


def sample_nodes(idx: int, N: int) -> np.ndarray:
    rng = np.random.default_rng(W.SEED_BASE + 1000 + idx)
    return np.sort(rng.choice(N, size=min(SAMPLE, N), replace=False)).astype(np.int64)


def full_name(idx: int) -> str:
    return "general_duct_d3q7_128x128x128" if idx == 4 else W.NAMES[idx]


def full_path(idx: int) -> str:
    return os.path.join(HERE, "full_%s_%d.npz" % (full_name(idx), FULL_STEPS))


def modes_path(idx: int) -> str:
    return os.path.join(HERE, "modes_%s_coarse%d.npz" % (W.NAMES[idx], COARSE))


def make_full(idx: int):
    w = W.general_workload() if idx == 4 else W.workload(idx)
    o = oracle.Oracle(w["geom"])
    f = o.init(w["P0"])
    inv0 = o.invariant(f)
    t0 = time.time()
    _, trace = o.run(f, FULL_STEPS, w["probes"])
    nodes = sample_nodes(idx, o.N)
    np.savez(full_path(idx), trace=trace, nodes=nodes, f=f[:, nodes].astype(np.float32),
             invariant=np.array([inv0, o.invariant(f)]), input_digest=np.array(input_digest(w)))
    print("full %s: %d steps in %.0f s" % (w["name"], FULL_STEPS, time.time() - t0), flush=True)


ENSEMBLE_TRACE_STRIDE = 10


def ensemble_path(i: int) -> str:
    return os.path.join(HERE, "ensemble_%d.npz" % i)


def stability_bound(o) -> float:
    """2 / sqrt(max over nodes of sum_d B_d), B_d = 4 for m_d <= 1 and
    (1 + m_d)^2 / m_d otherwise, m_d = Mhat^dd plus |Mhat^02| on axes 0
    and 2: the frozen-coefficient bound of the tau = 1/2 scheme."""
    tot = np.zeros(o.N)
    for a in range(o.dim):
        m = o.Mhat[a] + (np.abs(o.Mhat[4]) if o.dim == 3 and a in (0, 2) else 0.0)
        tot += np.where(m <= 1.0, 4.0, (1.0 + m) ** 2 / np.maximum(m, 1e-300))
    return 2.0 / float(np.sqrt(tot.max()))


def ensemble_member(i: int):
    """Horn i of the training ensemble with its wave speed, pulse and probes."""
    m = W.ensemble(512)[i]
    geom = dict(m["geom"], c=0.1)
    cmax = stability_bound(oracle.Oracle(geom))   # Mhat does not depend on c
    c2 = np.floor((0.9 * cmax) ** 2 * 65536.0) / 65536.0
    geom["c"] = float(np.sqrt(c2))
    return dict(geom=geom, P0=W.horn_pulse(geom), probes=np.asarray(m["probes"], dtype=np.int64))


def make_ensemble(i: int):
    w = ensemble_member(i)
    o = oracle.Oracle(w["geom"])
    f = o.init(w["P0"])
    t0 = time.time()
    _, trace = o.run(f, W.ENSEMBLE_STEPS, w["probes"])
    freq, power = oracle.modes(trace, W.ENSEMBLE_MODES)
    np.savez(ensemble_path(i), c=np.array(w["geom"]["c"]), freq=freq, power=power,
             trace=trace[::ENSEMBLE_TRACE_STRIDE], input_digest=np.array(input_digest(w)))
    print("ensemble horn %d %s c %.6f: %d steps in %.0f s, freq %s" % (
        i, w["geom"]["n"], w["geom"]["c"], W.ENSEMBLE_STEPS, time.time() - t0, freq), flush=True)


SWEEP_OMEGA = 0.071
SWEEP_SAMPLE = 16384


def sweep_path() -> str:
    return os.path.join(HERE, "sweep_torus_small_ring.npz")


def sweep_inputs():
    """The torus sweep's geometry, its small-ring source nodes and probes
    (the sweep's probe and two next to the ring), from rest."""
    geom = W.driven_torus()
    ring = np.asarray(W.torus_sources(geom)["small_ring"], dtype=np.int64)
    probes = np.concatenate([W.torus_probes(geom), ring[[3, 10]] + 2]).astype(np.int64)
    return dict(geom=geom, P0=np.zeros(W.num_nodes(geom)), probes=probes), ring


def make_sweep(_=0):
    w, ring = sweep_inputs()
    o = oracle.Oracle(w["geom"])
    f = o.init(w["P0"])
    T = W.TORUS_STEPS
    t0 = time.time()
    _, trace = o.run(f, T, w["probes"], sources=ring, amplitude=1.0, omega=SWEEP_OMEGA)
    rng = np.random.default_rng(W.SEED_BASE + 2000)
    nodes = np.sort(rng.choice(o.N, size=SWEEP_SAMPLE, replace=False)).astype(np.int64)
    np.savez(sweep_path(), trace=trace[::ENSEMBLE_TRACE_STRIDE], amplitude=o.amplitude(trace, T // 2, T),
             nodes=nodes, f=f[:, nodes].astype(np.float32), sources=ring, omega=np.array(SWEEP_OMEGA),
             steps=np.array(T), input_digest=np.array(input_digest(w)))
    print("torus sweep point omega %.3f: %d steps in %.0f s" % (SWEEP_OMEGA, T, time.time() - t0), flush=True)


def make_modes(idx: int):
    w = W.workload(idx, scale=COARSE)
    o = oracle.Oracle(w["geom"])
    f = o.init(w["P0"])
    n0 = float(np.linalg.norm(f))
    t0 = time.time()
    _, trace = o.run(f, w["steps"], w["probes"])
    freq, power = oracle.modes(trace, MODES_K)
    np.savez(modes_path(idx), freq=freq, power=power, steps=np.array(w["steps"]),
             norm=np.array([n0, float(np.linalg.norm(f))]), input_digest=np.array(input_digest(w)))
    print("modes %s x%d: %d steps in %.0f s, freq %s" % (w["name"], COARSE, w["steps"], time.time() - t0, freq),
          flush=True)


if __name__ == "__main__":
    what = sys.argv[1]
    for i in (int(v) for v in sys.argv[2:]):
        {"full": make_full, "modes": make_modes, "ensemble": make_ensemble, "sweep": make_sweep}[what](i)
