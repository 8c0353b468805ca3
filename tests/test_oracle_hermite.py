"""Pins for the oracle's Hermite-expansion equilibrium (Sec. II, Cartesian
boxes; CPU only).

The Hermite form uses the fixed lattice weights of D2Q5 / D3Q7
(c_s^2 = 1/(D+1), w = c_s^2 / 2) and adds the second-order term
P (c^2 - c_s^2)(xi^2 - D c_s^2) / (2 c_s^4), with f_0 = P - sum_{i>=1} f_i.
Its second moment is therefore c_eff^2 P with
c_eff^2 = c_s^2 + (c^2 - c_s^2)(1 - D c_s^2) / (2 c_s^2)
(c^2/2 + 1/8 on D3Q7, c^2/2 + 1/6 on D2Q5), not c^2 P.  Pins:

* at c = c_s the extra term vanishes and the Hermite form equals the moment-
  matching equilibrium: runs agree to rounding;
* a box eigenmode oscillates at the closed-form lattice frequency
  cos(omega) = 1 - 2 c_eff^2 sum_d sin^2(k_d / 2) of a wave speed c_eff, and
  not at the one of c (a factor or sign error in the Hermite term, or a wrong
  f_0, moves the frequency);
* the closed box conserves sum f;
* only Cartesian boxes accept the Hermite form.
"""
import math

import numpy as np
import pytest

import oracle


def box(n, walls, c, eq):
    d = len(n)
    return dict(kind="box", dim=d, n=tuple(n), qmin=(0.0,) * d, qmax=tuple(float(v) for v in n),
                bc_lo=tuple(walls), bc_hi=tuple(walls), h_ref=1.0, c=c, damp=1.0, params=(), equilibrium=eq)


def c_eff(c, d):
    cs2 = 1.0 / (d + 1)
    return math.sqrt(cs2 + (c * c - cs2) * (1.0 - d * cs2) / (2.0 * cs2))


def mode(n, walls, mvec):
    fields, ks = [], []
    for a in range(len(n)):
        i = np.arange(n[a]) + 0.5
        k = math.pi * mvec[a] / n[a]
        fields.append(np.cos(k * i) if walls[a] == "bounceback" else np.sin(k * i))
        ks.append(k)
    grids = np.meshgrid(*fields[::-1], indexing="ij")
    P = np.ones_like(grids[0])
    for g in grids:
        P = P * g
    return P.reshape(-1), ks


def fit_residual(trace, omega):
    t = np.arange(trace.shape[0])
    B = np.stack([np.ones_like(t, dtype=float), (-1.0) ** t, np.cos(omega * t), np.sin(omega * t)], axis=1)
    coef, *_ = np.linalg.lstsq(B, trace, rcond=None)
    return np.abs(trace - B @ coef).max() / np.abs(trace).max()


@pytest.mark.parametrize("n,walls", [((10, 8, 6), ("bounceback", "fixed", "bounceback")),
                                     ((14, 9), ("fixed", "bounceback"))])
def test_hermite_equals_moment_matching_at_cs(n, walls):
    d = len(n)
    cs = math.sqrt(1.0 / (d + 1))
    P0 = np.random.default_rng(4).uniform(-1, 1, int(np.prod(n)))
    out = []
    for eq in ("corrected", "hermite"):
        o = oracle.Oracle(box(n, walls, cs, eq))
        f = o.init(P0)
        _, tr = o.run(f, 200, [0, 7])
        out.append((f, tr))
    scale = np.abs(out[0][0]).max()
    assert np.abs(out[0][0] - out[1][0]).max() <= 1e-13 * scale
    assert np.abs(out[0][1] - out[1][1]).max() <= 1e-13 * np.abs(out[0][1]).max()


@pytest.mark.parametrize("n,walls,c,mvec", [((12, 10, 8), ("bounceback", "bounceback", "fixed"), 0.6, (1, 2, 1)),
                                            ((16, 12), ("fixed", "bounceback"), 0.3, (3, 2))])
def test_hermite_box_mode_travels_at_effective_speed(n, walls, c, mvec):
    d = len(n)
    ce = c_eff(c, d)
    assert ce < 1.0 / math.sqrt(d)                          # inside the Cartesian stability bound
    P0, k = mode(n, walls, mvec)
    o = oracle.Oracle(box(n, walls, c, "hermite"))
    f = o.init(P0)
    _, tr = o.run(f, 300, np.random.default_rng(2).integers(0, o.N, size=5))
    s = sum(math.sin(kd / 2) ** 2 for kd in k)
    om_eff = math.acos(1.0 - 2.0 * ce * ce * s)
    om_c = math.acos(1.0 - 2.0 * c * c * s)
    assert fit_residual(tr, om_eff) < 1e-10
    assert fit_residual(tr, om_c) > 1e-3


def test_hermite_closed_box_conserves():
    o = oracle.Oracle(box((9, 7, 6), ("bounceback",) * 3, 0.65, "hermite"))
    f = o.init(1.0 + np.random.default_rng(8).uniform(-1, 1, o.N))
    s0 = f.sum()
    o.run(f, 400, [])
    assert abs(f.sum() - s0) <= 1e-12 * abs(s0)


def test_hermite_only_on_boxes():
    import workloads as W
    with pytest.raises(ValueError):
        oracle.Oracle(dict(W.closed_cylinder(scale=16), equilibrium="hermite"))
    with pytest.raises(ValueError):
        oracle.Oracle(box((4, 4, 4), ("bounceback",) * 3, 0.5, "lattice"))
