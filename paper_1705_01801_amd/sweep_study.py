"""Frequency sweeps of the driven pipe (the ring and plate sources of
Sec. IV.A): every (source, drive frequency) pair is one copy of the pipe in
one batch, all advanced together; the response intensity at a probe is
plotted against the drive frequency and its peaks are compared with the
pipe's resonances.  The ring imposes the pressure on the inner-radius ring
of the closed end, the plate the flux J'_z on the whole closed-end plane.

    python -m paper_1705_01801_amd.sweep_study --out sweep.json
    python -m paper_1705_01801_amd.sweep_study --torus --out torus.json

The torus sweep (Sec. IV.C) drives the small ring at rho_min, theta = 0 of
a 20 x 200 x 30 torus at 499 frequencies and reads the intensity opposite
the source on the major circle.

Closed form used for the comparison: axisymmetric modes of the annulus
r in [1, 25] with reflecting (zero normal derivative) walls have radial
wavenumbers zeta_j (zeta_0 = 0 and the roots of
J_1(zeta a) Y_1(zeta b) - J_1(zeta b) Y_1(zeta a)); a pipe closed at z = 0 and
open at z = L has axial wavenumbers (2n + 1) pi / (2L), one closed at both
ends n pi / L; omega = c sqrt(zeta_j^2 + k_z^2).  Every numerical step of the
sweep runs in the HIP library; this script only sets it up and reads back
the intensities.
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

import workloads as W

from . import Batch, Simulation, Geometry


def radial_wavenumbers(a: float, b: float, kmax: float) -> list:
    from scipy.optimize import brentq
    from scipy.special import j1, y1

    def f(z):
        return j1(z * a) * y1(z * b) - j1(z * b) * y1(z * a)

    roots = [0.0]
    zs = np.linspace(1e-4, kmax, 4000)
    v = f(zs)
    for i in range(len(zs) - 1):
        if np.sign(v[i]) != np.sign(v[i + 1]):
            roots.append(brentq(f, zs[i], zs[i + 1]))
    return roots


def resonances(c: float, L: float, a: float, b: float, wmax: float, closed_open: bool) -> list:
    out = []
    for zeta in radial_wavenumbers(a, b, wmax / c):
        for n in range(0, 200):
            kz = (2 * n + 1) * math.pi / (2 * L) if closed_open else n * math.pi / L
            w = c * math.hypot(zeta, kz)
            if w > wmax:
                break
            if w > 0:
                out.append(w)
    return sorted(out)


def peaks(omega: np.ndarray, amp: np.ndarray, rel: float = 0.02) -> list:
    """Local maxima above rel * max, refined by a parabola through the three
    samples around each."""
    out = []
    top = amp.max()
    for i in range(1, len(amp) - 1):
        if amp[i] > amp[i - 1] and amp[i] >= amp[i + 1] and amp[i] > rel * top:
            y0, y1, y2 = amp[i - 1], amp[i], amp[i + 1]
            d = 0.5 * (y0 - y2) / (y0 - 2 * y1 + y2)
            out.append(float(omega[i] + d * (omega[1] - omega[0])))
    return out


def match(expected: list, found: list, tol: float):
    """Nearest found peak per expected resonance within tol (absolute)."""
    rows = []
    for w in expected:
        if not found:
            break
        j = int(np.argmin([abs(p - w) for p in found]))
        if abs(found[j] - w) <= tol:
            rows.append((w, found[j], found[j] / w - 1))
    return rows


def source_nodes(geom, source: str):
    """(nodes, flux axis or -1 for a pressure source) of a pipe source."""
    if source == "ring":
        return W.pipe_ring(geom), -1
    if source == "plate":
        return W.pipe_plate(geom), 2
    raise ValueError("source must be 'ring' or 'plate'")


def run(points: int = 119, steps: int = W.PIPE_STEPS, plain: int = 4, ends=("fixed", "free"),
        sources=("ring",), launch=None) -> dict:
    """The sweep: one batch with a copy of the pipe per (source, open end,
    drive frequency); returns the measurements and the peak comparison
    (response[source][end]).  The points run one at a time repeat the first
    source and end."""
    import torch
    omegas = W.sweep_omegas(points)
    combos = [(src, e) for src in sources for e in ends]
    geoms = [W.driven_pipe(e) for _, e in combos for _ in omegas]
    N = W.num_nodes(geoms[0])
    probes = W.pipe_probes(geoms[0])
    T = int(steps)
    b = Batch(geoms, [np.zeros(N)] * len(geoms), [probes] * len(geoms), t_max=T)
    nodes, which, om, axis = [], [], [], []
    for k, (src, _) in enumerate(combos):
        sn, ax = source_nodes(geoms[0], src)
        for i, w in enumerate(omegas):
            nodes.append(sn)
            which.append(np.full(sn.size, k * len(omegas) + i))
            om.append(np.full(sn.size, w))
            axis.append(np.full(sn.size, ax))
    b.set_sources(np.concatenate(nodes), np.concatenate(which), 1.0, np.concatenate(om), np.concatenate(axis))
    if launch:                                   # launch shape only: results are the same for every shape
        b.set_step_config(*launch)
    else:
        b.autotune(reps=10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(T)
    torch.cuda.synchronize()
    t_step = time.perf_counter() - t0
    t1 = time.perf_counter()
    amp = b.amplitude(T // 2, T).reshape(len(combos), len(omegas), len(probes))
    t_amp = time.perf_counter() - t1
    rep = {"workload": "driven pipe 20x5x100 (r, theta, z), %s source, c %.2f, damping %.2f"
                       % (" and ".join(sources), W.PIPE_C, W.PIPE_DAMP),
           "points": len(geoms), "omegas": [float(omegas[0]), float(omegas[-1]), len(omegas)], "steps": T,
           "nodes": int(N * len(geoms)), "launch": list(b.step_config()),
           "batched": {"seconds": t_step + t_amp, "step_seconds": t_step,
                       "points_per_s": len(geoms) / (t_step + t_amp),
                       "glups": N * len(geoms) * T / t_step / 1e9}}
    # a few points one at a time (same graph-replayed single-geometry path)
    if plain > 0:
        idx = np.linspace(0, len(omegas) - 1, plain).astype(int)
        same = True
        sn, ax = source_nodes(geoms[0], combos[0][0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in idx:
            sim = Simulation(Geometry(geoms[i]), np.zeros(N), probes, t_max=T)
            sim.set_sources(sn, 1.0, float(omegas[i]), None if ax < 0 else ax)
            sim.step(T)
            a = sim.amplitude(T // 2, T)
            same = same and bool(np.array_equal(a, amp[0, i]))
            sim.close()
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        rep["plain"] = {"points": len(idx), "seconds": tp, "points_per_s": len(idx) / tp,
                        "identical_to_batched": same}
        rep["batched_vs_plain"] = rep["batched"]["points_per_s"] / rep["plain"]["points_per_s"]
    geom = geoms[0]
    a_in, b_out = geom["qmin"][0], geom["qmax"][0]
    L = geom["qmax"][2]
    # compared: the plane-wave band below the first radial cutoff, where the
    # resonances are pi c / L apart and a peak within 0.4 of that spacing is
    # unambiguous; above it both families interleave
    cutoff = W.PIPE_C * radial_wavenumbers(a_in, b_out, 1.0)[1]
    wmax = min(float(omegas[-1]), cutoff)
    tol = 0.4 * math.pi * W.PIPE_C / L
    rep["compared_band"] = [float(omegas[0]), wmax]
    rep["response"] = {src: {} for src in sources}
    for e, (src, end) in enumerate(combos):
        found = peaks(omegas, amp[e, :, 0])
        res = {"peaks": found}
        for label, co in (("closed_open", True), ("closed_closed", False)):
            exp = resonances(W.PIPE_C, L, a_in, b_out, wmax, co)
            m = match(exp, found, tol)
            res[label] = {"expected": exp, "matched": len(m),
                          "rms_rel": float(np.sqrt(np.mean([r[2] ** 2 for r in m]))) if m else None,
                          "max_rel": float(max(abs(r[2]) for r in m)) if m else None,
                          "pairs": [[r[0], r[1]] for r in m]}
        res["intensity_probe0"] = amp[e, :, 0].tolist()
        rep["response"][src][end] = res
    b.close()
    return rep


def run_torus(points: int = 499, steps: int = W.TORUS_STEPS, modes: int = 400, plain: int = 2) -> dict:
    """The torus sweep of Sec. IV.C: the small ring (rho_min, theta = 0, all
    phi) driven at every frequency, one torus copy per frequency in one
    batch, intensity opposite the source on the major circle.  The paper has
    no closed form for the torus, so the peaks are compared with the
    resonances of the same torus found another way: the spectral peaks
    (lbw_modes) of a lossless ring-down from a unit pressure on the small
    ring, recorded at the same probe for the same number of steps."""
    import torch
    omegas = W.torus_omegas(points)
    geom = W.driven_torus()
    N = W.num_nodes(geom)
    ring, probes = W.torus_sources(geom)["small_ring"], W.torus_probes(geom)
    T = int(steps)
    b = Batch([geom] * len(omegas), [np.zeros(N)] * len(omegas), [probes] * len(omegas), t_max=T)
    b.set_sources(np.concatenate([ring] * len(omegas)), np.repeat(np.arange(len(omegas)), ring.size), 1.0,
                  np.repeat(omegas, ring.size))
    b.autotune(reps=5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(T)
    torch.cuda.synchronize()
    t_step = time.perf_counter() - t0
    amp = b.amplitude(T // 2, T).reshape(len(omegas), len(probes))
    b.close()
    plain_rep = None
    if plain > 0:                                    # a few points one at a time
        idx = np.linspace(0, len(omegas) - 1, plain).astype(int)
        same = True
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in idx:
            sim = Simulation(Geometry(geom), np.zeros(N), probes, t_max=T)
            sim.set_sources(ring, 1.0, float(omegas[i]))
            sim.step(T)
            same = same and bool(np.array_equal(sim.amplitude(T // 2, T), amp[i]))
            sim.close()
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        plain_rep = {"points": len(idx), "seconds": tp, "points_per_s": len(idx) / tp, "identical_to_batched": same}
    rep = {"workload": "driven torus 20x200x30 (rho, theta, phi), R 640, rho in [5.12, 409.6], small-ring source, "
                       "c %.2f, damping %.2f" % (geom["c"], geom["damp"]),
           "points": len(omegas), "omegas": [float(omegas[0]), float(omegas[-1]), len(omegas)], "steps": T,
           "nodes": int(N * len(omegas)),
           "batched": {"step_seconds": t_step, "points_per_s": len(omegas) / t_step,
                       "glups": N * len(omegas) * T / t_step / 1e9}}
    if plain_rep:
        rep["plain"] = plain_rep
        rep["batched_vs_plain"] = rep["batched"]["points_per_s"] / plain_rep["points_per_s"]
    # the same torus without losses, rung down from the small ring
    lossless = dict(geom, damp=1.0)
    P0 = np.zeros(N)
    P0[ring] = 1.0
    sim = Simulation(Geometry(lossless), P0, probes[:1], t_max=T)
    sim.step(T)
    f_ring, p_ring = sim.modes(modes)
    sim.close()
    ring_down = sorted(float(2 * math.pi * f) for f, p in zip(f_ring, p_ring) if f > 0)
    found = peaks(omegas, amp[:, 0])
    a0 = amp[:, 0]
    top = sorted(sorted(found, key=lambda w: -float(np.interp(w, omegas, a0)))[:5])
    spacing = float(omegas[1] - omegas[0])
    # every sweep peak inside the ring-down's range against its nearest mode
    diffs = [min(abs(r - w) for r in ring_down) for w in found if ring_down and w <= ring_down[-1]]
    above = np.nonzero(a0 >= 0.1 * a0.max())[0]
    rep["response"] = {"peaks": found, "ring_down_modes": ring_down, "five_largest_peaks": top,
                       "compared_peaks": len(diffs),
                       "matched_within_1.5_spacing": int(sum(d <= 1.5 * spacing for d in diffs)),
                       "median_abs_diff": float(np.median(diffs)) if diffs else None,
                       "cutoff_10pct": float(omegas[above[-1]]) if above.size else None,
                       "intensity": a0.tolist()}
    return rep


def main():
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--points", type=int, default=None, help="drive frequencies (pipe 119, torus 499)")
    ap.add_argument("--steps", type=int, default=None, help="steps per point (pipe 8400, torus 8000)")
    ap.add_argument("--plain", type=int, default=4, help="sweep points also run one at a time")
    ap.add_argument("--sources", default="ring,plate", help="comma-separated: ring, plate")
    ap.add_argument("--torus", action="store_true", help="the torus sweep instead of the pipe's")
    ap.add_argument("--launch", default=None,
                    help="tile_x,chunk_z,blocks of the batch step (pipe sweep; default: tuned)")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    torch.cuda.set_device(0)
    if args.torus:
        rep = run_torus(args.points or 499, args.steps or W.TORUS_STEPS)
    else:
        launch = tuple(int(v) for v in args.launch.split(",")) if args.launch else None
        rep = run(args.points or 119, args.steps or W.PIPE_STEPS, args.plain, sources=tuple(args.sources.split(",")),
                  launch=launch)
    line = json.dumps(rep)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
