"""Resonant-frequency extraction from probe traces (FP64, numpy).

TEST INFRASTRUCTURE ONLY (part of the oracle package).

The paper finds resonances with driven frequency sweeps (Sec. IV.A pipe
spectra, Sec. IV.C torus spectra); for a freely ringing field the same
information is the peak set of the probe signal's power spectrum.  Rule:
  1. per probe: subtract the mean, multiply by a symmetric Hann window
     w[t] = 1/2 - 1/2 cos(2 pi t / (T - 1));
  2. zero-pad to nfft = 4 * (smallest power of two >= T), FFT, power |X_k|^2;
  3. sum the power over probes;
  4. peaks: bins k in [16, nfft/2 - 1] with P[k-1] < P[k] >= P[k+1] and
     P[k] > rel_threshold * max_{k >= 16} P.  The main lobe of the window's
     transform is 2/T cycles per step wide on each side, 8 nfft/(4T) <= 16
     bins: below bin 16 a peak can be the leakage of a slow drift that the
     mean removal leaves (a decaying baseline), not a resonance;
  5. refine each by a parabola through ln P at k-1, k, k+1 (no refinement,
     delta = 0, when P[k-1] or P[k+1] is zero):
     delta = (ln P[k-1] - ln P[k+1]) / (2 (ln P[k-1] - 2 ln P[k] + ln P[k+1])),
     frequency (k + delta) / nfft cycles per step,
     power exp(ln P[k] - (ln P[k-1] - ln P[k+1]) delta / 4);
  6. the k lowest frequencies, ascending (NaN-padded when fewer exist).
"""
from __future__ import annotations

import numpy as np


FIRST_BIN = 16


def nfft_for(T: int) -> int:
    p = 1
    while p < T:
        p *= 2
    return 4 * p


def power_spectrum(trace: np.ndarray) -> np.ndarray:
    trace = np.asarray(trace, dtype=np.float64)
    if trace.ndim == 1:
        trace = trace[:, None]
    T = trace.shape[0]
    nfft = nfft_for(T)
    t = np.arange(T, dtype=np.float64)
    win = 0.5 - 0.5 * np.cos(2.0 * np.pi * t / (T - 1)) if T > 1 else np.ones(1)
    x = (trace - trace.mean(axis=0, keepdims=True)) * win[:, None]
    X = np.fft.rfft(x, n=nfft, axis=0)
    return (X.real ** 2 + X.imag ** 2).sum(axis=1)


def modes(trace: np.ndarray, k: int, rel_threshold: float = 1e-3):
    """Returns (freq[k], power[k]) in cycles per step."""
    P = power_spectrum(trace)
    nfft = 2 * (P.size - 1)
    freq = np.full(k, np.nan)
    powr = np.full(k, np.nan)
    if nfft // 2 <= FIRST_BIN + 1:
        return freq, powr
    pmax = P[FIRST_BIN:].max()
    found = 0
    for b in range(FIRST_BIN, nfft // 2):
        if found == k:
            break
        if P[b - 1] < P[b] and P[b] >= P[b + 1] and P[b] > rel_threshold * pmax:
            l0 = np.log(P[b])
            if P[b - 1] > 0.0 and P[b + 1] > 0.0:
                lm, lp = np.log(P[b - 1]), np.log(P[b + 1])
                den = lm - 2.0 * l0 + lp
                delta = 0.5 * (lm - lp) / den if den != 0.0 else 0.0
            else:
                lm = lp = delta = 0.0
            freq[found] = (b + delta) / nfft
            powr[found] = np.exp(l0 - 0.25 * (lm - lp) * delta)
            found += 1
    return freq, powr
