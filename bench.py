"""Benchmark: fused collide-and-stream step of the curvilinear wave LBM on
one MI355X.  The headline is the largest single-GPU configuration, the
torus (D3Q7, 96 x 256 x 512 = 12.6 M nodes, FP32 populations, 64 probes
recorded every step); the closed cylinder (128 x 128 x 256, whose 235 MB
working set fits the 256 MB Infinity Cache) and the horn (128 x 128 x 512)
are timed as extra legs.

Prints one JSON line.  value = whole-job MLUPS (node updates per second / 1e6)
with the state resident in device memory, after the library's autotuner has
chosen the launch (one step per launch, or two with the temporally blocked
kernel where that is faster); roofline = algorithmic bytes per launch (56 B
per node update: 7 float populations read and written, times the updates a
launch makes) over the measured average launch duration, against 8 TB/s,
beside the HBM bytes per launch the committed counters measured for that
kernel (about half the algorithmic ones for two steps per launch); surrogate = shape-spectra
per second of the plain per-shape LBM, the batched LBM and the trained
surrogate with every fallback candidate simulated; cpu_baseline = the FP64
oracle on the host for a bounded number of steps of the headline grid.
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
# committed counter summaries per configuration and steps per launch (one
# step, or two with the two-step kernel), and the kernel sources they cover
_MARCH = ("step_march.hip", "march_common.h", "step.hip", "lbw_internal.h")
_MARCH2 = ("step_march2.hip", "march_common.h", "lbw_internal.h")
TRAFFIC = {(1, 1): ("traffic_step_cylinder_128x128x256.txt", _MARCH),
           (2, 1): ("traffic_step_horn_128x128x512.txt", _MARCH),
           (3, 1): ("traffic_step_torus_96x256x512.txt", _MARCH),
           (4, 1): ("traffic_step_general_duct_128x128x128.txt", ("step_general.hip", "lbw_internal.h")),
           (2, 2): ("traffic_step2_horn_128x128x512.txt", _MARCH2),
           (3, 2): ("traffic_step2_torus_96x256x512.txt", _MARCH2)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash(config: int = 1, steps_per_launch: int = 1):
    h = hashlib.sha256()
    for name in TRAFFIC[(config, steps_per_launch)][1]:
        with open(os.path.join(ROOT, "paper_1705_01801_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(config: int = 1, steps_per_launch: int = 1):
    """HBM bytes per launch (of one or two steps) from the committed
    rocprofv3 counter summary of this configuration and kernel, if it was
    taken on the current kernel source."""
    key = (config, steps_per_launch)
    if key not in TRAFFIC:
        return None
    path = os.path.join(ROOT, "profiles", TRAFFIC[key][0])
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash(config, steps_per_launch):
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


# working sets below the 256 MB Infinity Cache are served from it, not HBM
INFINITY_CACHE_BYTES = 256 * 2 ** 20


def time_config(config, steps, warmup, launch="auto", two_step=None):
    """Runs one configuration's full step (probes recorded) after tuning the
    launch shape, timed with HIP events on the stream the library launches
    on; returns the numbers the JSON line reports."""
    import torch

    import paper_1705_01801_amd as lbw
    import workloads as W

    w = W.general_workload() if config == 4 else W.workload(config)
    geom = w["geom"]
    N = W.num_nodes(geom)
    g = lbw.Geometry(geom)
    sim = lbw.Simulation(g, w["P0"], w["probes"], t_max=warmup + steps)
    general = config == 4          # per-node kernel: no launch shapes to tune
    if general:
        tuned_us = float("nan")
    elif launch == "auto":
        tuned_us = sim.autotune(reps=20)
    else:
        g.set_step_config(*(int(v) for v in launch.split(",")))
        tuned_us = float("nan")
    if two_step and not general:
        # a fixed two-steps-per-launch shape (for profiling that kernel)
        g.set_step2_config(*(int(v) for v in two_step.split(",")))
    tile = g.step_config()
    two = g.step2_config() if not general else (0, 0, 0, 0)
    log("bench: %s, %d nodes, warmup %d, steps %d, launch shape %s, two-step %s (tuner %.2f us per step)"
        % (w["name"], N, warmup, steps, tile, two, tuned_us))
    sim.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    sim.probe(0, min(sim.t, sim.t_max))  # raises on a non-finite trace
    ms_per_step = ms / steps
    # algorithmic bytes per node update: 7 populations read and written, plus
    # 9 float coefficients read per node for a geometry given by its metric
    bpn = 92.0 if general else 56.0
    achieved = bpn * N / (ms_per_step / 1e3) / 1e9
    working_set = (2 * 28 + (36 if general else 0)) * N
    out = {"workload": w["name"], "nodes": N, "ms_per_step": round(ms_per_step, 5),
           "mlups": round(N * steps / (ms / 1e3) / 1e6, 1), "achieved_gbs": round(achieved, 1),
           "frac": round(achieved / HBM_PEAK_GBS, 4),
           # HBM bytes per launch of the kernel that ran (two steps per
           # launch with the two-step kernel; achieved_gbs covers the same)
           "traffic": read_traffic(config, 2 if two[0] else 1),
           "residency": "infinity-cache" if working_set <= INFINITY_CACHE_BYTES else "hbm",
           "working_set_bytes": working_set, "probes": int(len(w["probes"])), "c": geom["c"],
           "launch": {"tile_x": tile[0], "tile_y": tile[1], "chunk_z": tile[2], "blocks": tile[3],
                      "graph_block": 32, "steps_per_launch": 2 if two[0] else 1}}
    if two[0]:
        out["launch"]["two_step"] = {"tile_x": two[0], "tile_y": two[1], "chunk_z": two[2], "blocks": two[3]}
    sim.close()
    g.close()
    return out, w


def copy_ceiling(N):
    """A device-to-device copy moving the same 56 B per node (torch copy_)."""
    import torch
    src = torch.empty(7 * N, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    stream = torch.cuda.current_stream()
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(50):
        dst.copy_(src)
    c1.record(stream)
    torch.cuda.synchronize()
    return 56.0 * N / (c0.elapsed_time(c1) / 50 / 1e3) / 1e9


def surrogate_leg(candidates, train):
    """Shape-spectra per second on the same GPU: plain per-shape LBM (the
    first training horns one after another), batched LBM (the training
    ensemble in one launch per step), and surrogate + fallback on
    `candidates` candidate profiles with the whole fallback set simulated
    (batched) and timed; 30000 steps and 10 modes per spectrum."""
    from paper_1705_01801_amd import surrogate_study
    log("bench: surrogate leg, %d training horns, %d candidates" % (train, candidates))
    return surrogate_study.measured_rate(train=train, candidates=candidates, log=log)


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
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--launch", default="auto",
                    help="'auto' (autotune) or TILE_X,TILE_Y,CHUNK_Z,BLOCKS to fix the step kernel's launch shape")
    ap.add_argument("--two-step", default=None,
                    help="TILE_X,TILE_Y,CHUNK_Z,BLOCKS: run two steps per launch with this shape (headline only)")
    ap.add_argument("--config", type=int, default=3, choices=(1, 2, 3, 4),
                    help="3-D workload of the headline: 3 torus 96x256x512 (the largest single-GPU one), "
                         "1 cylinder 128x128x256, 2 horn 128x128x512, 4 duct 128x128x128 given by its metric")
    ap.add_argument("--legs", default="1,2",
                    help="other configurations timed as extra legs (comma list, empty for none)")
    ap.add_argument("--leg-steps", type=int, default=500)
    ap.add_argument("--candidates", type=int, default=10000,
                    help="candidate horn profiles of the surrogate leg (0 skips it)")
    ap.add_argument("--train-horns", type=int, default=512)
    ap.add_argument("--sweep-points", type=int, default=119,
                    help="drive frequencies in the driven-pipe sweep leg (0 skips it)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path (the slab decomposition that "
              "would shard a grid is described in the design notes); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    torch.cuda.set_device(0)
    head, w = time_config(args.config, args.steps, args.warmup, args.launch, args.two_step)
    N = head["nodes"]
    copy_gbs = copy_ceiling(N)
    out = {
        "metric": METRIC, "value": head["mlups"], "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": head["workload"], "nodes": N, "lattice": "D3Q7", "probes": head["probes"],
                   "c": head["c"], "launch": head["launch"], "residency": head["residency"]},
        "roofline": {"bound": "hbm", "achieved": head["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": head["frac"], "traffic": head["traffic"]},
        "copy_ceiling": {"achieved": round(copy_gbs, 1), "unit": "GB/s",
                         "note": "device copy of the same 56 B/node, torch copy_"},
    }
    legs = [int(v) for v in args.legs.split(",") if v.strip() and int(v) != args.config]
    if legs:
        out["legs"] = {}
        for c in legs:
            leg, _ = time_config(c, args.leg_steps, max(args.leg_steps // 10, 10), args.launch)
            out["legs"][leg["workload"]] = {k: leg[k] for k in ("mlups", "ms_per_step", "achieved_gbs", "frac",
                                                                  "residency", "traffic", "launch")}
    if args.candidates > 0:
        out["surrogate"] = surrogate_leg(args.candidates, args.train_horns)
    if args.sweep_points > 0:
        out["sweep"] = sweep_leg(args.sweep_points)
    if not args.no_cpu_baseline:
        log("bench: oracle baseline, %d steps" % args.cpu_steps)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
