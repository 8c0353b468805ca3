"""Benchmark: fused collide-and-stream step of the curvilinear wave LBM on
one MI355X, on the 3-D closed cylinder (D3Q7, 128 x 128 x 256 nodes, FP32
populations, 16 probes recorded every step).

Prints one JSON line.  value = whole-job MLUPS (node updates per second / 1e6)
with the state resident in HBM; roofline = algorithmic bytes per launch
(56 B per node: 7 float populations read and written) over the measured
average launch duration, against 8 TB/s; cpu_baseline = the FP64 oracle on
the host for a bounded number of steps of the same grid.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS & % HBM peak; shape-spectra/sec batched+surrogate vs plain LBM"
HBM_PEAK_GBS = 8000.0
# committed counter summaries per configuration, and the kernel sources they cover
_MARCH = ("step_march.hip", "step.hip", "lbw_internal.h")
TRAFFIC = {1: ("traffic_step_cylinder_128x128x256.txt", _MARCH),
           2: ("traffic_step_horn_128x128x512.txt", _MARCH),
           3: ("traffic_step_torus_96x256x512.txt", _MARCH),
           4: ("traffic_step_general_duct_128x128x128.txt", ("step_general.hip", "lbw_internal.h"))}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash(config: int = 1):
    h = hashlib.sha256()
    for name in TRAFFIC[config][1]:
        with open(os.path.join(ROOT, "paper_1705_01801_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(config: int = 1):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this configuration, if it was taken on the current kernel source."""
    if config not in TRAFFIC:
        return None
    path = os.path.join(ROOT, "profiles", TRAFFIC[config][0])
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash(config):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(w, steps):
    import numpy as np

    import oracle
    o = oracle.Oracle(w["geom"])
    f = o.init(w["P0"])
    t0 = time.perf_counter()
    o.run(f, steps, w["probes"])
    dt = time.perf_counter() - t0
    return {"value": o.N * steps / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": "%d steps of the full %s grid (FP64, single thread, %.1f s; host has %d cores)"
                      % (steps, w["name"], dt, os.cpu_count() or 0)}


def spectra_leg(n_horns, n_plain=4):
    """Shape-spectra per second of the batched LBM (n_horns ensemble horns in
    one launch per step) and of the per-shape LBM (the first n_plain of them,
    one after another), 30000 steps and 10 modes each."""
    import numpy as np

    import workloads as W
    from paper_1705_01801_amd import surrogate as S
    members = S.with_wave_speeds(W.ensemble(n_horns, stream=2))
    p0s = [W.horn_pulse(m["geom"]) for m in members]
    steps, k = W.ENSEMBLE_STEPS, W.ENSEMBLE_MODES
    log("bench: spectra leg, %d horns batched, %d per shape" % (n_horns, n_plain))
    f_b, t_step, t_modes = S.run_batch(members, p0s, steps, k)
    f_p, t_plain = S.run_plain(members[:n_plain], p0s[:n_plain], steps, k)
    same = np.isfinite(f_p) & np.isfinite(f_b[:n_plain])
    nodes = int(sum(np.prod(m["geom"]["n"]) for m in members))
    batched = n_horns / (t_step + t_modes)
    plain = n_plain / t_plain
    return {"unit": "spectra/s", "batched": round(batched, 3), "plain": round(plain, 3),
            "batched_vs_plain": round(batched / plain, 2), "horns": n_horns, "plain_horns": n_plain,
            "nodes": nodes, "steps": steps, "modes": k,
            "max_rel_diff_plain_vs_batched": float(np.max(np.abs(f_p[same] / f_b[:n_plain][same] - 1.0)))
            if same.any() else None,
            "note": "surrogate + LBM fallback rate comes from the surrogate study (python -m "
                    "paper_1705_01801_amd.surrogate_study), which trains the surrogate first"}


def sweep_leg(points):
    """Driven-pipe frequency sweep (ring source, Sec. IV.A): sweep points per
    second with every drive frequency a copy in one batch, against two
    points run one at a time; 8400 steps per point."""
    from paper_1705_01801_amd import sweep_study
    log("bench: sweep leg, %d drive frequencies batched" % points)
    r = sweep_study.run(points=points, plain=2, ends=("fixed",))
    m = r["response"]["ring"]["fixed"]["closed_open"]
    return {"unit": "sweep points/s", "batched": round(r["batched"]["points_per_s"], 2),
            "plain": round(r["plain"]["points_per_s"], 3), "batched_vs_plain": round(r["batched_vs_plain"], 1),
            "points": r["points"], "steps": r["steps"], "nodes": r["nodes"], "glups": round(r["batched"]["glups"], 2),
            "identical_to_plain": r["plain"]["identical_to_batched"],
            "closed_open_peaks_matched": m["matched"], "closed_open_rms_rel": m["rms_rel"],
            "workload": r["workload"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--cpu-steps", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--launch", default="auto",
                    help="'auto' (autotune) or TILE_X,TILE_Y,CHUNK_Z,BLOCKS to fix the step kernel's launch shape")
    ap.add_argument("--config", type=int, default=1, choices=(1, 2, 3, 4),
                    help="3-D workload to time: 1 cylinder 128x128x256 (the benchmark), 2 horn 128x128x512, "
                         "3 torus 96x256x512, 4 duct 128x128x128 given by its metric (per-node kernel)")
    ap.add_argument("--spectra-horns", type=int, default=64,
                    help="horns in the batched-vs-plain spectra leg (0 skips it)")
    ap.add_argument("--sweep-points", type=int, default=119,
                    help="drive frequencies in the driven-pipe sweep leg (0 skips it)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU; the library has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1705_01801_amd as lbw
    import workloads as W

    torch.cuda.set_device(0)
    w = W.general_workload() if args.config == 4 else W.workload(args.config)
    geom = w["geom"]
    N = W.num_nodes(geom)
    g = lbw.Geometry(geom)
    sim = lbw.Simulation(g, w["P0"], w["probes"], t_max=args.warmup + args.steps)
    general = args.config == 4          # per-node kernel: no launch shapes to tune
    if general:
        tuned_us = float("nan")
    elif args.launch == "auto":
        tuned_us = sim.autotune(reps=20)
    else:
        sim.geometry.set_step_config(*(int(v) for v in args.launch.split(",")))
        tuned_us = float("nan")
    tile = g.step_config()  # the general kernel: its default shape, one workgroup per tile
    log("bench: %s, %d nodes, warmup %d, steps %d, launch shape %s (tuner %.2f us)" % (w["name"], N, args.warmup,
                                                                                   args.steps, tile, tuned_us))
    sim.step(args.warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    sim.probe(0, min(sim.t, sim.t_max))  # raises on a non-finite trace
    ms_per_step = ms / args.steps
    mlups = N * args.steps / (ms / 1e3) / 1e6
    # algorithmic bytes per node update: 7 populations read and written, plus
    # 9 float coefficients read per node for a geometry given by its metric
    bytes_per_launch = (92.0 if general else 56.0) * N
    achieved = bytes_per_launch / (ms_per_step / 1e3) / 1e9
    traffic = read_traffic(args.config)
    # practical ceiling: a device-to-device copy moving the same bytes
    src = torch.empty(7 * N, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(50):
        dst.copy_(src)
    c1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 56.0 * N / (c0.elapsed_time(c1) / 50 / 1e3) / 1e9
    del src, dst
    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w["name"], "nodes": N, "lattice": "D3Q7", "probes": int(len(w["probes"])),
                   "c": geom["c"], "launch": {"tile_x": tile[0], "tile_y": tile[1], "chunk_z": tile[2],
                                              "blocks": tile[3], "graph_block": 32}},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic},
        "copy_ceiling": {"achieved": round(copy_gbs, 1), "unit": "GB/s",
                         "note": "device copy of the same 56 B/node, torch copy_"},
    }
    if args.spectra_horns > 0:
        out["spectra"] = spectra_leg(args.spectra_horns)
    if args.sweep_points > 0:
        out["sweep"] = sweep_leg(args.sweep_points)
    if not args.no_cpu_baseline:
        log("bench: oracle baseline, %d steps" % args.cpu_steps)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
