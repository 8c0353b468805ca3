"""Host-side logic of the surrogate pipeline (CPU only)."""
import numpy as np

import workloads as W
from paper_1705_01801_amd import surrogate as S


def test_relative_spread():
    preds = np.array([[[1.0, 2.0], [10.0, 10.0]], [[1.02, 2.0], [10.0, 10.5]], [[0.98, 2.0], [10.0, 10.0]]])
    sp = S.relative_spread(preds)
    assert np.allclose(sp, [0.04 / 1.0, 0.5 / (30.5 / 3)])


def test_features_round_trip():
    rng = np.random.default_rng(0)
    prof = W.horn_profiles(50, rng)
    logf = np.log(rng.uniform(0.5, 5, size=(50, 10)))
    logf[3, 7] = np.nan
    f = S.Features([W.HORN_RANGES[k] for k in ("a", "b", "k")], logf)
    x = f.x(prof)
    assert x.min() >= -1 - 1e-6 and x.max() <= 1 + 1e-6
    y = f.y(logf)
    assert np.allclose(np.nanmean(y, axis=0), 0, atol=1e-5)
    back = np.log(f.freq(y))
    ok = np.isfinite(logf)
    assert np.allclose(back[ok], logf[ok], rtol=0, atol=1e-5)


def test_physical_units_and_ensemble_shapes():
    geoms = [dict(c=0.5, h_ref=0.01), dict(c=0.25, h_ref=0.02)]
    f = S.physical(np.array([[0.001], [0.002]]), geoms)
    assert np.allclose(f[:, 0], [0.2, 0.4])
    e = W.ensemble(8)
    for m in e:
        g = m["geom"]
        assert g["c"] is None and g["kind"] == "horn" and len(m["probes"]) == W.ENSEMBLE_PROBES
        nr, nt, nz = g["n"]
        assert nt in W.HORN_GRIDS["nt"] and nz >= min(W.HORN_GRIDS["nz"]) and nz % 16 == 0
        assert nr >= 16 and nr % 8 == 0 and g["h_ref"] == 1.0 / nz
        # no radial link shorter than the lattice unit, and the largest such n_r
        rho = 0.95 * W.shortest_radial_link(m["profile"])
        assert rho / nr >= g["h_ref"] * (1 - 1e-12) and (nr == 16 or rho / (nr + 8) < g["h_ref"])
        assert np.all(m["probes"] < np.prod(g["n"]))


def test_extra_peak_detects_a_second_family():
    from paper_1705_01801_amd import surrogate_study as SS
    ladder = 0.25 + 0.5 * np.arange(10)                       # closed-open tube, unit length
    flared = ladder + np.array([0.05, 0.02, 0.01, 0.005, 0, 0, 0, 0, 0, 0])
    doublet = np.sort(np.concatenate([ladder[:8], [3.76], [4.21]]))   # 3.75, 3.76; 4.21, 4.25 missing
    midway = np.sort(np.concatenate([ladder[:9], [2.0]]))    # one peak halfway between 1.75 and 2.25
    missing = flared.copy()
    missing[9] = np.nan
    got = SS.extra_peak(np.stack([ladder, flared, doublet, midway, missing]))
    assert got.tolist() == [False, False, True, True, False]


def test_served_region_and_stated_draws():
    # R(1) = a + b e^k against the measured bound, below the ceiling set by
    # the second radial family of the bell
    assert abs(W.BELL_RADIUS_CEILING * 2 * np.pi * 4.75 - 7.0155866698) < 1e-9
    assert W.SERVED_BELL_RADIUS < W.BELL_RADIUS_CEILING
    assert W.served([[0.1, 0.01, 2.0]]).tolist() == [0.1 + 0.01 * np.exp(2.0) <= W.SERVED_BELL_RADIUS]
    assert W.served([[0.2, 0.05, 5.0], [0.05, 0.005, 1.0], [0.15, 0.01, 1.7]]).tolist() == [False, True, False]
    prof, grid = W.stated_candidates(2000)
    lo = np.array([W.STATED_RANGES[k][0] for k in "abk"])
    hi = np.array([W.STATED_RANGES[k][1] for k in "abk"])
    assert (prof >= lo).all() and (prof <= hi).all()
    assert set(grid[:, 0]) <= set(W.STATED_GRIDS["nt"]) and set(grid[:, 1]) <= set(W.STATED_GRIDS["nz"])
    assert 0.06 < W.served(prof).mean() < 0.13
    ms = W.served_ensemble(64, stream=1)
    assert len(ms) == 64 and W.served([m["profile"] for m in ms]).all()
    st = W.stated_ensemble(16, "stated")
    iso = W.stated_ensemble(16, "isotropic")
    short = W.stated_ensemble(16, "stated_short")
    for s, i, sh in zip(st, iso, short):
        assert s["profile"] == i["profile"] == sh["profile"] and s["geom"]["n"] == sh["geom"]["n"]
        nr, _, nz = sh["geom"]["n"]
        link = W.shortest_radial_link(sh["profile"]) * 0.95 / nr
        assert sh["geom"]["h_ref"] == min(link, 1.0 / nz) and s["geom"]["h_ref"] == 1.0 / nz
        nr, nt, nz = s["geom"]["n"]
        assert nr in W.STATED_GRIDS["nr"] and nt in W.STATED_GRIDS["nt"] and nz in W.STATED_GRIDS["nz"]
        assert i["geom"]["n"][1] == nt and i["geom"]["n"][2] >= nz
