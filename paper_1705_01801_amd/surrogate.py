"""Batched horn spectra and the learned surrogate with LBM fallback.

Every numerical step runs in the HIP library: the batched LBM
(``Batch``), the device FFT mode extraction, and the MLP kernels (``MLP``).
This module only orchestrates: it picks wave speeds from the library's
stability bound, converts spectra to physical units, normalises features,
and decides which candidates fall back to the LBM.

Physical units: wave speed 1, lengths in horn lengths (z in [0, 1]); a
frequency of f cycles per step is f / (c h_ref) in these units.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import Batch, Geometry, MLP, Simulation

WIDTHS = (3, 256, 256, 256, 10)


def wave_speed(geom: dict, safety: float = 0.9) -> float:
    """safety x the library's stability bound, rounded down so that c^2 is a
    multiple of 2^-16 (exact in float32)."""
    g = Geometry(dict(geom, c=0.1))
    cmax = g.stability_bound()
    g.close()
    c2 = math.floor((safety * cmax) ** 2 * 65536.0) / 65536.0
    return math.sqrt(c2)


def with_wave_speeds(members):
    out = []
    for m in members:
        geom = dict(m["geom"])
        if geom.get("c") is None:
            geom["c"] = wave_speed(geom)
        out.append(dict(m, geom=geom))
    return out


def physical(freq_steps: np.ndarray, geoms) -> np.ndarray:
    """cycles/step -> physical frequency, per geometry (rows)."""
    scale = np.array([1.0 / (g["c"] * g["h_ref"]) for g in geoms])
    return freq_steps * scale[:, None]


def run_batch(members, p0s, steps: int, k: int, chunk: int = 2000, tune: bool = True, log=None, keep_trace=False):
    """Advances all members together (after timing the batch's launch shapes
    on scratch buffers when tune is set: results are the same for every
    shape); returns (physical frequencies [n, k], seconds of stepping,
    seconds of mode extraction)."""
    import torch
    geoms = [m["geom"] for m in members]
    b = Batch(geoms, p0s, [m["probes"] for m in members], t_max=steps)
    if tune:
        b.autotune(reps=10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        n = min(chunk, steps - done)
        b.step(n)
        done += n
        if log:
            torch.cuda.synchronize()
            log("batch of %d: %d/%d steps, %.1f s" % (len(geoms), done, steps, time.perf_counter() - t0))
    torch.cuda.synchronize()
    t_step = time.perf_counter() - t0
    t1 = time.perf_counter()
    f, pw = b.modes(k)
    t_modes = time.perf_counter() - t1
    trace = b.probe() if keep_trace else None
    b.close()
    if keep_trace:
        return physical(f, geoms), t_step, t_modes, pw, trace
    return physical(f, geoms), t_step, t_modes


def run_plain(members, p0s, steps: int, k: int, log=None):
    """Per-shape baseline: each member stepped alone (graph-captured blocks,
    default launch shape).  Returns (physical frequencies, seconds)."""
    import torch
    out = np.full((len(members), k), np.nan)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, (m, p0) in enumerate(zip(members, p0s)):
        g = Geometry(m["geom"])
        s = Simulation(g, p0, m["probes"], t_max=steps)
        s.step(steps)
        f, _ = s.modes(k)
        out[i] = physical(f[None, :], [m["geom"]])[0]
        s.close()
        g.close()
        if log:
            log("plain %d/%d, %.1f s" % (i + 1, len(members), time.perf_counter() - t0))
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


class Features:
    """Affine map of (a, b, k) to [-1, 1] and of log-frequencies to zero
    mean, unit variance per mode (statistics of the training set)."""

    def __init__(self, ranges, logf: np.ndarray):
        self.lo = np.array([r[0] for r in ranges])
        self.hi = np.array([r[1] for r in ranges])
        self.mu = np.nanmean(logf, axis=0)
        self.sd = np.nanstd(logf, axis=0) + 1e-12

    def x(self, prof):
        return (2.0 * (np.asarray(prof) - self.lo) / (self.hi - self.lo) - 1.0).astype(np.float32)

    def y(self, logf):
        return ((logf - self.mu) / self.sd).astype(np.float32)

    def freq(self, ynorm):
        return np.exp(np.asarray(ynorm, dtype=np.float64) * self.sd + self.mu)


def relative_spread(preds: np.ndarray) -> np.ndarray:
    """Ensemble disagreement per candidate: max over modes of
    (max - min over members) / mean over members; preds [members, n, k]."""
    mean = preds.mean(axis=0)
    return ((preds.max(axis=0) - preds.min(axis=0)) / np.abs(mean)).max(axis=1)


class Surrogate:
    """Ensemble of MLPs trained on LBM spectra (log-frequency targets)."""

    def __init__(self, ranges, members: int = 4, widths=WIDTHS, max_batch: int = 131072, seed: int = 0):
        self.ranges = ranges
        self.widths = list(widths)
        self.nets = [MLP(self.widths, max_batch=max_batch) for _ in range(members)]
        self.seed = seed
        self.feat = None

    def fit(self, prof: np.ndarray, freqs: np.ndarray, steps: int = 4000, lr: float = 1e-3, log=None,
            bootstrap: bool = True):
        """Full-batch Adam on all valid (finite, positive) targets; returns
        the final training loss of each member on the whole set.  With
        bootstrap each member sees its own resample of the training horns
        (Poisson(1) multiplicities as weights), so members also disagree where
        the targets jump between neighbouring horns, not only where the data
        is thin."""
        import torch
        logf = np.where(np.isfinite(freqs) & (freqs > 0), np.log(np.where(freqs > 0, freqs, 1.0)), np.nan)
        self.feat = Features(self.ranges, logf)
        dev = torch.device("cuda", torch.cuda.current_device())
        x = torch.as_tensor(self.feat.x(prof), device=dev)
        wn = np.isfinite(logf).astype(np.float32)
        w = torch.as_tensor(wn, device=dev)
        t = torch.as_tensor(np.nan_to_num(self.feat.y(logf), nan=0.0), device=dev)
        wsum = float(wn.sum())
        losses = []
        for i, net in enumerate(self.nets):
            rng = np.random.default_rng(self.seed + 1000 * i)
            params = []
            for l in range(len(self.widths) - 1):
                lim = 1.0 / math.sqrt(self.widths[l])
                params.append(rng.uniform(-lim, lim, size=self.widths[l] * self.widths[l + 1]))
                params.append(np.zeros(self.widths[l + 1]))
            net.set_params(np.concatenate(params))
            # cosine rate lr (1 + cos(pi s / steps)) / 2 + 1e-5, one captured
            # training step replayed by the library
            if bootstrap:
                mult = rng.poisson(1.0, size=len(wn)).astype(np.float32)
                wb = wn * mult[:, None]
                net.train(x, t, torch.as_tensor(wb, device=dev), steps=steps, lr=lr, lr_floor=1e-5,
                          weight_sum=float(wb.sum()))
            else:
                net.train(x, t, w, steps=steps, lr=lr, lr_floor=1e-5, weight_sum=wsum)
            loss = net.loss_grad(x, t, w, weight_sum=wsum)[0].item()
            losses.append(loss)
            if log:
                log("member %d trained, loss %.3e" % (i, loss))
        return losses

    def predict(self, prof: np.ndarray):
        """(mean frequency [n, k], relative spread [n], member predictions)."""
        x = self.feat.x(prof)
        preds = np.stack([self.feat.freq(net.forward(x).cpu().numpy()) for net in self.nets])
        return preds.mean(axis=0), relative_spread(preds), preds
