"""Writes the stored oracle results that the full-size GPU parity tests use.

Calls only the FP64 oracle (``oracle/``) on the seeded inputs of
``workloads``; nothing here comes from the HIP library.  Run from the
repository root (one process per case, CPU only):

    python tests/golden/make_goldens.py full 1 2 3     # 1000 steps, full grids
    python tests/golden/make_goldens.py modes 1 2 3    # 4x coarser grids, configured step counts

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
  t = 0 and at the end).
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
    h.update(json.dumps(w["geom"], sort_keys=True, default=float).encode())
    h.update(np.ascontiguousarray(w["P0"], dtype=np.float64).tobytes())
    h.update(np.ascontiguousarray(w["probes"], dtype=np.int64).tobytes())
    return h.hexdigest()


def sample_nodes(idx: int, N: int) -> np.ndarray:
    rng = np.random.default_rng(W.SEED_BASE + 1000 + idx)
    return np.sort(rng.choice(N, size=min(SAMPLE, N), replace=False)).astype(np.int64)


def full_path(idx: int) -> str:
    return os.path.join(HERE, "full_%s_%d.npz" % (W.NAMES[idx], FULL_STEPS))


def modes_path(idx: int) -> str:
    return os.path.join(HERE, "modes_%s_coarse%d.npz" % (W.NAMES[idx], COARSE))


def make_full(idx: int):
    w = W.workload(idx)
    o = oracle.Oracle(w["geom"])
    f = o.init(w["P0"])
    inv0 = o.invariant(f)
    t0 = time.time()
    _, trace = o.run(f, FULL_STEPS, w["probes"])
    nodes = sample_nodes(idx, o.N)
    np.savez(full_path(idx), trace=trace, nodes=nodes, f=f[:, nodes].astype(np.float32),
             invariant=np.array([inv0, o.invariant(f)]), input_digest=np.array(input_digest(w)))
    print("full %s: %d steps in %.0f s" % (w["name"], FULL_STEPS, time.time() - t0), flush=True)


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
        (make_full if what == "full" else make_modes)(i)
