"""Batched horn ensemble + surrogate study (prints one JSON report).

1. LBM spectra of the training ensemble (seeded horns R(z) = a + b e^{kz} on
   uneven grids), all horns advanced together by the batched kernel;
2. the same horns' spectra from per-shape runs (a sample), for the plain
   per-shape rate;
3. a 4-member MLP ensemble trained on the batched spectra;
4. inference on the candidate profiles; candidates whose members disagree
   by more than the threshold fall back to the LBM;
5. the LBM as judge: a sample of accepted candidates is simulated to measure
   the surrogate's error, and a sample of the fallback set is simulated to
   measure the fallback cost per spectrum.

Usage: python -m paper_1705_01801_amd.surrogate_study [--train 512] ...
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np


def measured_rate(train: int = 512, candidates: int = 10000, plain: int = 4, judge: int = 64,
                  threshold: float = 0.01, train_steps: int = 10000, log=None) -> dict:
    """Measured shape-spectra rates on one GPU, every spectrum produced by the
    library: the batched LBM on the training ensemble, the per-shape LBM on
    its first horns, and surrogate + fallback on the first `candidates`
    candidate profiles, where the whole fallback set is simulated (batched)
    and timed, not projected.  A sample of accepted candidates is simulated
    too, as the judge of the surrogate's error."""
    import torch

    import workloads as W
    from paper_1705_01801_amd import surrogate as S

    steps, K = W.ENSEMBLE_STEPS, W.ENSEMBLE_MODES
    members = S.with_wave_speeds(W.ensemble(train, stream=0))
    p0s = [W.horn_pulse(m["geom"]) for m in members]
    f_train, t_step, t_modes = S.run_batch(members, p0s, steps, K)
    batched = len(members) / (t_step + t_modes)
    f_plain, t_plain = S.run_plain(members[:plain], p0s[:plain], steps, K)
    same = np.isfinite(f_plain) & np.isfinite(f_train[:plain])
    prof = np.array([m["profile"] for m in members])
    sur = S.Surrogate([W.HORN_RANGES[k] for k in ("a", "b", "k")], members=4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sur.fit(prof, f_train, steps=train_steps)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    cprof, cgrid = W.candidates(candidates)

    def simulate(idx):
        ms = S.with_wave_speeds([W.horn_member(cprof[i], cgrid[i]) for i in idx])
        ps = [W.horn_pulse(m["geom"]) for m in ms]
        f, ts, tm = S.run_batch(ms, ps, steps, K)
        return f, ts + tm

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mean, spread, _ = sur.predict(cprof)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    fallback = np.flatnonzero(spread > threshold)
    t_fb = 0.0
    if len(fallback):
        if log:
            log("surrogate leg: %d of %d candidates fall back to the LBM" % (len(fallback), candidates))
        _, t_fb = simulate(fallback)
    rate = candidates / (t_inf + t_fb)
    acc = np.flatnonzero(spread <= threshold)
    out = {"unit": "spectra/s", "plain": round(plain / t_plain, 3), "batched": round(batched, 3),
           "surrogate_plus_fallback": round(rate, 2), "surrogate_vs_plain": round(rate * t_plain / plain, 1),
           "batched_vs_plain": round(batched * t_plain / plain, 2), "candidates": candidates,
           "fallback": int(len(fallback)), "inference_s": round(t_inf, 4), "fallback_lbm_s": round(t_fb, 2),
           "training_horns": len(members), "training_lbm_s": round(t_step + t_modes, 2),
           "training_s": round(t_train, 2),
           "end_to_end_with_training": round(candidates / (t_step + t_modes + t_train + t_inf + t_fb), 2),
           "plain_horns": plain, "steps": steps, "modes": K,
           "max_rel_diff_plain_vs_batched": float(np.max(np.abs(f_plain[same] / f_train[:plain][same] - 1.0)))
           if same.any() else None}
    if judge and len(acc):
        jidx = np.random.default_rng(7).choice(acc, size=min(judge, len(acc)), replace=False)
        f_judge, _ = simulate(jidx)
        ok = np.isfinite(f_judge) & np.isfinite(mean[jidx])
        err = np.abs(mean[jidx][ok] / f_judge[ok] - 1.0)
        out["judge"] = {"accepted_sampled": len(jidx), "modes": int(ok.sum()),
                        "rel_err_median": float(np.median(err)), "rel_err_max": float(err.max())}
    return out


EXTRA_PEAK_GAP = 0.6


def extra_peak(f: np.ndarray) -> np.ndarray:
    """Rows of spectra (ascending peaks) with two consecutive peaks closer
    than EXTRA_PEAK_GAP times the row's median gap (False where a peak is
    missing)."""
    out = np.zeros(len(f), dtype=bool)
    ok = np.isfinite(f).all(axis=1)
    if ok.any():
        g = np.diff(f[ok], axis=1)
        out[ok] = g.min(axis=1) < EXTRA_PEAK_GAP * np.median(g, axis=1)
    return out


def multi_family(f: np.ndarray, profiles) -> np.ndarray:
    """Rows of ten-peak spectra (physical units) that are not one longitudinal
    family: the second axisymmetric radial family of the bell, from
    j'_{0,2} / (2 pi R(1)), starts below the last peak, or extra_peak()."""
    from scipy.special import jn_zeros
    p = np.asarray(profiles, dtype=np.float64).reshape(-1, 3)
    cut2 = jn_zeros(1, 2)[1] / (2.0 * math.pi * (p[:, 0] + p[:, 1] * np.exp(p[:, 2])))
    return (cut2 < np.nan_to_num(f[:, -1], nan=0.0)) | extra_peak(f)


def census(rule: str = "stated", n: int = 512, steps: int | None = None, growth: float = 2.0, log=None) -> dict:
    """Which horns of the configured profile box and grids the scheme serves:
    classify() of workloads.stated_ensemble(n, rule)."""
    import workloads as W
    return dict(classify(W.stated_ensemble(n, rule), steps, growth, log), rule=rule)


def classify(members, steps: int | None = None, growth: float = 2.0, log=None) -> dict:
    """Every horn simulated by the batched LBM for the configured steps and
    put in the first class that applies:
      unstable      the population 2-norm grows more than `growth`-fold over
                    the run, or turns non-finite;
      unresolved    fewer than ten spectral peaks found, or the first
                    usable spectral frequency, 16 / (nfft c h_ref) in
                    physical units, above 0.25, the lowest resonance of a
                    closed-open tube of unit length (flare only raises it):
                    the run is too short in physical time to see the
                    fundamental;
      multi-family  the ten peaks are not one longitudinal family: the
                    second axisymmetric radial family of the bell, which
                    starts at j'_{0,2} / (2 pi R(1)) in physical units, lies
                    below the tenth peak (the probes sit on the nodal circle
                    of the first radial family only), or two consecutive
                    peaks lie closer than EXTRA_PEAK_GAP times the median
                    gap (the longitudinal ladder is evenly spaced, about 0.5
                    apart, so a closer pair holds a peak of another family);
      usable        the rest.
    Returns the class counts and the per-horn figures."""
    import torch
    from scipy.special import jn_zeros

    import workloads as W
    from paper_1705_01801_amd import Batch, Geometry
    from paper_1705_01801_amd import surrogate as S

    steps = steps or W.ENSEMBLE_STEPS
    K = W.ENSEMBLE_MODES
    members = S.with_wave_speeds(members)
    n = len(members)
    geoms = [m["geom"] for m in members]
    prof = np.array([m["profile"] for m in members])
    grid = np.array([g["n"][:3] for g in geoms], dtype=np.int64)
    mrr = np.zeros(n)
    for i, g in enumerate(geoms):
        geo = Geometry(g)
        mrr[i] = geo.table()[0].max()           # largest Mhat^rr of the horn
        geo.close()
    b = Batch(geoms, [W.horn_pulse(g) for g in geoms], [m["probes"] for m in members], t_max=steps)
    b.autotune(reps=5)

    def norms():
        return np.array([float(torch.linalg.vector_norm(b.populations(h).double())) for h in range(n)])

    n0 = norms()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        m = min(5000, steps - done)
        b.step(m)
        done += m
        if log:
            torch.cuda.synchronize()
            log("classify %d horns: %d/%d steps, %.1f s" % (n, done, steps, time.perf_counter() - t0))
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    n1 = norms()
    fq, _ = b.modes(K)
    b.close()
    f = S.physical(fq, geoms)
    a, bb, k = prof.T
    R1 = a + bb * np.exp(k)
    ratio = np.where(np.isfinite(n1), n1 / n0, np.inf)
    unstable = ratio > growth
    nfft = 4 * (1 << int(math.ceil(math.log2(steps))))
    f_lo = 16.0 / (nfft * np.array([g["c"] for g in geoms]) * np.array([g["h_ref"] for g in geoms]))
    unresolved = ~unstable & (np.isnan(f).any(axis=1) | (f_lo > 0.25))
    cut2 = jn_zeros(1, 2)[1] / (2.0 * math.pi * R1)
    multi = ~unstable & ~unresolved & multi_family(f, prof)
    usable = ~(unstable | unresolved | multi)
    nodes = int(grid.prod(axis=1).sum())
    counts = {"unstable": int(unstable.sum()), "unresolved": int(unresolved.sum()),
              "multi_family": int(multi.sum()), "usable": int(usable.sum())}
    return {"horns": n, "steps": steps, "nodes": nodes, "seconds": seconds,
            "glups": nodes * steps / seconds / 1e9, "growth_limit": growth, "counts": counts,
            "fractions": {key: v / n for key, v in counts.items()},
            "per_horn": {"profile": prof.tolist(), "grid": grid.tolist(),
                         "c": [g["c"] for g in geoms], "h_ref": [g["h_ref"] for g in geoms],
                         "mhat_rr_max": mrr.tolist(), "norm_ratio": ratio.tolist(), "freq": f.tolist(),
                         "first_usable_frequency": f_lo.tolist(),
                         "bell_radius": R1.tolist(), "bell_slope": (bb * k * np.exp(k)).tolist(),
                         "second_radial_cut_on": cut2.tolist(),
                         "class": np.select([unstable, unresolved, multi], ["unstable", "unresolved", "multi-family"],
                                            "usable").tolist()}}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=512)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--plain", type=int, default=16)
    ap.add_argument("--judge", type=int, default=128)
    ap.add_argument("--no-bootstrap", action="store_true", help="train every member on the whole training set")
    ap.add_argument("--fallback-sample", type=int, default=256)
    ap.add_argument("--candidates", type=int, default=100000)
    ap.add_argument("--threshold", type=float, default=0.01)
    ap.add_argument("--train-steps", type=int, default=10000)
    ap.add_argument("--hidden", type=int, default=256, help="width of the three hidden layers")
    ap.add_argument("--out", default=None)
    ap.add_argument("--save-npz", default=None, help="write training spectra (and traces) here")
    ap.add_argument("--train-only", action="store_true", help="stop after the batched training ensemble")
    ap.add_argument("--box", choices=("narrow", "stated"), default="narrow",
                    help="narrow: the training box HORN_RANGES; stated: the configured box STATED_RANGES, "
                         "candidates outside workloads.served() excluded")
    ap.add_argument("--keep-multi-family", action="store_true",
                    help="with --box stated: train on every training horn, one family or not")
    ap.add_argument("--census", choices=("stated", "stated_short", "isotropic"), default=None,
                    help="classify the horns of the configured profile box and grids instead (see census)")
    args = ap.parse_args(argv)

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import torch

    import workloads as W
    from paper_1705_01801_amd import surrogate as S

    def log(msg):
        print("[study] " + msg, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    if args.census:
        rep = census(args.census, n=args.train, steps=args.steps, log=log)
        log("census (%s): %s" % (args.census, json.dumps(rep["counts"])))
        if args.out:
            with open(args.out, "w") as f:
                f.write(json.dumps(rep) + "\n")
        print(json.dumps({k: v for k, v in rep.items() if k != "per_horn"}), flush=True)
        return
    steps = args.steps or W.ENSEMBLE_STEPS
    K = W.ENSEMBLE_MODES
    rep = {"steps": steps, "modes": K, "threshold": args.threshold, "box": args.box}
    stated = args.box == "stated"
    ranges = W.STATED_RANGES if stated else W.HORN_RANGES

    # 1. batched training ensemble
    members = S.with_wave_speeds(W.served_ensemble(args.train) if stated else W.ensemble(args.train, stream=0))
    p0s = [W.horn_pulse(m["geom"]) for m in members]
    nodes = int(sum(np.prod(m["geom"]["n"]) for m in members))
    log("training ensemble: %d horns, %.1f M nodes" % (len(members), nodes / 1e6))
    f_train, t_step, t_modes, p_train, tr_train = S.run_batch(members, p0s, steps, K, log=log, keep_trace=True)
    if args.save_npz:
        np.savez_compressed(args.save_npz, profiles=np.array([m["profile"] for m in members]),
                            grids=np.array([m["geom"]["n"] for m in members]),
                            c=np.array([m["geom"]["c"] for m in members]),
                            h_ref=np.array([m["geom"]["h_ref"] for m in members]), freq=f_train, power=p_train,
                            trace=tr_train[::2, 1::W.ENSEMBLE_PROBES].astype(np.float32))
    rep["batched"] = {"horns": len(members), "nodes": nodes, "seconds": t_step + t_modes, "step_seconds": t_step,
                      "mode_seconds": t_modes, "spectra_per_s": len(members) / (t_step + t_modes),
                      "glups": nodes * steps / t_step / 1e9}
    log("batched: %.1f s, %.2f spectra/s" % (t_step + t_modes, rep["batched"]["spectra_per_s"]))
    if args.train_only:
        print(json.dumps(rep), flush=True)
        return

    # 2. plain per-shape sample (the first horns of the same ensemble)
    ns = min(args.plain, len(members))
    f_plain, t_plain = S.run_plain(members[:ns], p0s[:ns], steps, K, log=log)
    same = np.isfinite(f_plain) & np.isfinite(f_train[:ns])
    rep["plain"] = {"horns": ns, "seconds": t_plain, "spectra_per_s": ns / t_plain,
                    "max_rel_diff_vs_batched": float(np.nanmax(np.abs(f_plain[same] / f_train[:ns][same] - 1)))
                    if same.any() else None}
    log("plain: %.1f s for %d horns" % (t_plain, ns))

    # 3. surrogate ensemble.  On the configured box, training horns whose
    # peaks are not one family (a peak split where a radial-family mode
    # crosses a longitudinal one) are left out unless --keep-multi-family.
    prof = np.array([m["profile"] for m in members])
    mf = multi_family(f_train, prof)
    rep["training_multi_family"] = int(mf.sum())
    f_fit = f_train
    if stated and not args.keep_multi_family:
        f_fit = np.where(mf[:, None], np.nan, f_train)
        log("training: %d of %d horns left out (not one family)" % (mf.sum(), len(mf)))
    sur = S.Surrogate([ranges[k] for k in ("a", "b", "k")], members=4,
                      widths=(3, args.hidden, args.hidden, args.hidden, K))
    t0 = time.perf_counter()
    losses = sur.fit(prof, f_fit, steps=args.train_steps, log=log, bootstrap=not args.no_bootstrap)
    torch.cuda.synchronize()
    rep["training"] = {"seconds": time.perf_counter() - t0, "final_losses": losses, "widths": sur.widths,
                       "adam_steps": args.train_steps, "bootstrap": not args.no_bootstrap,
                       "valid_targets": int(np.isfinite(f_fit).sum())}

    # 4. inference on candidates (of the configured box: those outside the
    # served region are excluded, neither predicted nor simulated)
    if stated:
        cprof, cgrid = W.stated_candidates(args.candidates)
        keep = W.served(cprof)
        rep["excluded"] = {"candidates": len(cprof), "outside_served": int((~keep).sum()),
                           "fraction": float((~keep).mean()), "rule": "R(1) > %.4f" % W.SERVED_BELL_RADIUS}
        cprof, cgrid = cprof[keep], cgrid[keep]
        log("excluded %d of %d candidates outside the served region" % ((~keep).sum(), len(keep)))
    else:
        cprof, cgrid = W.candidates(args.candidates)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mean, spread, _ = sur.predict(cprof)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    fallback = spread > args.threshold
    rep["inference"] = {"candidates": len(cprof), "seconds": t_inf, "fallback": int(fallback.sum()),
                        "fallback_fraction": float(fallback.mean())}
    log("inference: %.3f s, fallback %d of %d" % (t_inf, fallback.sum(), len(cprof)))

    rng = np.random.default_rng(7)

    def simulate(idx):
        ms = S.with_wave_speeds([W.horn_member(cprof[i], cgrid[i]) for i in idx])
        ps = [W.horn_pulse(m["geom"]) for m in ms]
        f, ts, tm, pw, _ = S.run_batch(ms, ps, steps, K, log=log, keep_trace=True)
        return f, ts + tm, pw

    # 5. judge accepted candidates
    acc = np.flatnonzero(~fallback)
    if len(acc):
        jidx = rng.choice(acc, size=min(args.judge, len(acc)), replace=False)
        f_judge, t_judge, pw_judge = simulate(jidx)
        ok = np.isfinite(f_judge) & np.isfinite(mean[jidx])
        err = np.abs(mean[jidx][ok] / f_judge[ok] - 1.0)
        rep["judge"] = {"sampled": len(jidx), "seconds": t_judge, "modes_compared": int(ok.sum()),
                        "rel_err_median": float(np.median(err)), "rel_err_p95": float(np.quantile(err, 0.95)),
                        "rel_err_max": float(err.max()), "frac_within_1pct": float((err <= 0.01).mean())}
        # accepted candidates with a mode more than 1 % off: what the surrogate
        # predicted against the LBM's modes and their spectral powers
        cand_err = np.where(ok, np.abs(mean[jidx] / np.where(ok, f_judge, 1.0) - 1.0), 0.0).max(axis=1)
        rep["judge"]["outliers"] = [
            {"profile": cprof[jidx[i]].tolist(), "grid": [int(v) for v in cgrid[jidx[i]]],
             "spread": float(spread[jidx[i]]), "predicted": mean[jidx[i]].tolist(), "lbm": f_judge[i].tolist(),
             "lbm_power": pw_judge[i].tolist()} for i in np.flatnonzero(cand_err > 0.01)]
        log("judge: median %.2e p95 %.2e max %.2e" % (np.median(err), np.quantile(err, 0.95), err.max()))

    # 6. fallback cost per spectrum (batched LBM on a sample of the fallback set)
    fb = np.flatnonzero(fallback)
    per_spec = rep["batched"]["seconds"] / rep["batched"]["horns"]
    if len(fb):
        fidx = rng.choice(fb, size=min(args.fallback_sample, len(fb)), replace=False)
        _, t_fb, _ = simulate(fidx)
        per_spec = t_fb / len(fidx)
        rep["fallback_sample"] = {"sampled": len(fidx), "seconds": t_fb, "seconds_per_spectrum": per_spec}
    total = t_inf + len(fb) * per_spec
    rep["surrogate_plus_fallback"] = {
        "seconds_projected": total, "spectra_per_s": len(cprof) / total,
        "note": "inference measured on all candidates; fallback time = fallback count x measured batched "
                "LBM seconds per spectrum on the fallback sample"}
    # end to end: the training ensemble's LBM runs and the training itself
    # are paid once for the whole candidate set
    e2e = rep["batched"]["seconds"] + rep["training"]["seconds"] + total
    rep["end_to_end"] = {"seconds": e2e, "spectra_per_s": len(cprof) / e2e,
                         "speedup_vs_plain": len(cprof) / e2e / rep["plain"]["spectra_per_s"]}
    rep["speedup_vs_plain"] = rep["surrogate_plus_fallback"]["spectra_per_s"] / rep["plain"]["spectra_per_s"]
    rep["batched_speedup_vs_plain"] = rep["batched"]["spectra_per_s"] / rep["plain"]["spectra_per_s"]
    line = json.dumps(rep)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
