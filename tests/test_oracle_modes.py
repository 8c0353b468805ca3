"""Oracle pins against analytic eigenfrequencies and the spectrum extractor.

* annulus (2-D polar) and hollow cylinder (3-D) normal modes: the scheme must
  converge at second order (Sec. IV.A convergence study) to the continuum
  frequencies c k, with k from the Bessel cross-product equations of the
  Laplacian on an annulus.  Bounce-back walls are zero-flux walls, so the
  radial condition is dP/dr = 0 (zeros built from J'_m, Y'_m); fixed walls
  give P = 0.  m = 0 modes pin the sqrt(g) factor of the Christoffel force,
  m >= 1 and z-dependent modes pin the sign of the gradient force.
* horn longitudinal modes: for a slowly flaring horn the plane-wave modes
  are the eigenvalues of Webster's horn equation (1/S) d/dz (S dp/dz) +
  (2 pi f)^2 p = 0, S ~ R(z)^2, a one-dimensional problem solved here by
  finite volumes; its own error is of order R'^2.  This pins the horn's
  metric terms (the Mhat^rz gradient force in particular) that no closed
  form of the full problem reaches;
* torus ring mode: a wave once around the major circle (cos theta) has the
  lowest eigenvalue of the cross-section problem
      -d_r(r h d_r psi) - d_phi((h/r) d_phi psi) + (r/h) psi = lam r h psi,
  h = R + r cos(phi), zero flux at both walls (finite volumes, scipy); this
  pins the torus metric (G^theta theta = 1/h^2, the sqrt(g) weighting, the
  phi-dependent forces) that no closed form reaches;
* the frequency extractor recovers known sinusoids;
* the zeros the paper prints for the pipe's wall condition (golden file).
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sparse
import scipy.sparse.linalg as sparse_linalg
from scipy.linalg import eigh_tridiagonal
from scipy.optimize import brentq, minimize_scalar
from scipy.special import jv, jvp, yv, yvp

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def first_root(fun, lo=0.5, hi=40.0, step=0.01):
    x = lo
    f0 = fun(x)
    while x < hi:
        x2 = x + step
        f1 = fun(x2)
        if f0 == 0.0 or f0 * f1 < 0:
            return brentq(fun, x, x2, xtol=1e-14)
        x, f0 = x2, f1
    raise RuntimeError("no root")


def annulus_k(m, a, b, outer):
    if outer == "bounceback":
        fun = lambda k: jvp(m, k * a) * yvp(m, k * b) - jvp(m, k * b) * yvp(m, k * a)
    else:
        fun = lambda k: jvp(m, k * a) * yv(m, k * b) - jv(m, k * b) * yvp(m, k * a)
    return first_root(fun)


def radial_profile(m, k, a, r):
    return jv(m, k * r) * yvp(m, k * a) - yv(m, k * r) * jvp(m, k * a)


def measure_omega(trace, guess):
    """Least-squares frequency of traces assumed to hold one oscillation plus
    the stationary and period-2 components of the scheme."""
    t = np.arange(trace.shape[0])

    def resid(om):
        B = np.stack([np.ones_like(t, dtype=float), (-1.0) ** t, np.cos(om * t), np.sin(om * t)], axis=1)
        coef, *_ = np.linalg.lstsq(B, trace, rcond=None)
        return float(((trace - B @ coef) ** 2).sum())

    res = minimize_scalar(resid, bounds=(0.9 * guess, 1.1 * guess), method="bounded",
                          options={"xatol": 1e-13 * guess})
    return res.x


def bound(o):
    tot = np.zeros(o.N)
    for a in range(o.dim):
        m = o.Mhat[a]
        tot += np.where(m <= 1.0, 4.0, (1.0 + m) ** 2 / np.maximum(m, 1e-300))
    return 2.0 / math.sqrt(tot.max())


def annulus_error(nr, m, outer, a=0.3, b=1.0, periods=8):
    geom = dict(kind="polar2d", dim=2, n=(nr, 3 * nr), qmin=(a, 0.0), qmax=(b, 2 * math.pi),
                bc_lo=("bounceback", "periodic"), bc_hi=(outer, "periodic"), h_ref=(b - a) / nr, c=0.3,
                damp=1.0, params=())
    c = 0.8 * bound(oracle.Oracle(geom))
    geom["c"] = c
    o = oracle.Oracle(geom)
    k = annulus_k(m, a, b, outer)
    r, th = W.node_grid(geom)
    P0 = radial_profile(m, k, a, r) * np.cos(m * th)
    f = o.init(P0)
    om_c = k * c * geom["h_ref"]
    T = int(periods * 2 * math.pi / om_c)
    probes = [i + nr * j for i in (1, nr // 3, nr // 2) for j in (0, 1)]
    _, trace = o.run(f, T, probes)
    om = measure_omega(trace, om_c)
    return om / om_c - 1.0


@pytest.mark.parametrize("m,outer", [(0, "bounceback"), (1, "bounceback"), (2, "bounceback"), (1, "fixed")])
def test_annulus_modes_converge_second_order(m, outer):
    e1 = annulus_error(16, m, outer)
    e2 = annulus_error(32, m, outer)
    e3 = annulus_error(64, m, outer)
    assert abs(e3) < 2e-3, (e1, e2, e3)
    r1, r2 = e1 / e2, e2 / e3
    assert 3.0 < r1 < 5.5 and 3.0 < r2 < 5.5, (e1, e2, e3)


def cylinder_error(nr, m=1, nz_mode=1, a=0.3, b=1.0, L=1.0, periods=6):
    n = (nr, 3 * nr, int(round(nr * 10 / 12)))
    geom = dict(kind="cylinder", dim=3, n=n, qmin=(a, 0.0, 0.0), qmax=(b, 2 * math.pi, L),
                bc_lo=("bounceback", "periodic", "bounceback"), bc_hi=("bounceback", "periodic", "bounceback"),
                h_ref=(b - a) / nr, c=0.3, damp=1.0, params=())
    c = 0.8 * bound(oracle.Oracle(geom))
    geom["c"] = c
    o = oracle.Oracle(geom)
    assert abs(o.Mhat[2]).max() > 0.3  # h_z != h_r: the z gradient force is active
    kr = annulus_k(m, a, b, "bounceback")
    k = math.hypot(kr, nz_mode * math.pi / L)
    r, th, z = W.node_grid(geom)
    P0 = radial_profile(m, kr, a, r) * np.cos(m * th) * np.cos(nz_mode * math.pi * z / L)
    f = o.init(P0)
    om_c = k * c * geom["h_ref"]
    T = int(periods * 2 * math.pi / om_c)
    probes = [i + n[0] * (j + n[1] * kz) for i in (1, nr // 2) for j in (0, 1) for kz in (0, n[2] // 3)]
    _, trace = o.run(f, T, probes)
    return measure_omega(trace, om_c) / om_c - 1.0


def test_hollow_cylinder_mode_with_axial_variation():
    e1 = cylinder_error(12)
    e2 = cylinder_error(24)
    assert abs(e2) < 1e-2 and 3.0 < e1 / e2 < 5.5, (e1, e2)


def test_extractor_recovers_sinusoids():
    rng = np.random.default_rng(11)
    for T in (700, 4000, 20000):
        fs = np.array([0.013, 0.041, 0.097, 0.151])
        t = np.arange(T)
        x = sum(a * np.cos(2 * math.pi * f * t + rng.uniform(0, 6)) for f, a in zip(fs, (1.0, 0.5, 0.8, 0.3)))
        x = np.stack([x + 0.2, 0.5 * x - 1.0], axis=1)
        est, pw = oracle.modes(x, 4)
        nfft = oracle.modes.__globals__["nfft_for"](T)
        assert np.abs(est - fs).max() * nfft < 2e-3
        assert np.all(np.diff(est) > 0)
    # a slowly decaying baseline (time constant 2T) leaks into the window's
    # DC main lobe; no peak is reported there
    T = 30000
    t = np.arange(T)
    x = 0.3 * (np.cos(2 * math.pi * 31 / T * t + 1.0) + np.cos(2 * math.pi * 72 / T * t + 1.0)) + 3.0 * np.exp(-t / (2.0 * T))
    est, _ = oracle.modes(x[:, None], 3)
    assert np.abs(est[:2] * T - (31, 72)).max() < 0.05 and np.isnan(est[2])
    # fewer peaks than requested are NaN-padded
    est, _ = oracle.modes(np.cos(0.3 * np.arange(1000))[:, None], 3)
    assert abs(est[0] - 0.3 / (2 * math.pi)) < 1e-4 and np.isnan(est[1:]).all()


def test_paper_robin_zero_table():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "paper_pipe_robin_zeros.txt")) if not l.startswith("#")]
    printed = [float(v) for _, v in rows]
    fun = lambda x: jv(0, x) - x * jv(1, x)  # (m+1) J_m - x J_{m+1}, m = 0
    zeros = [brentq(fun, lo, lo + 1.5) for lo in (0.5, 3.5, 6.5)]
    assert abs(zeros[0] - printed[0]) < 5e-4 and abs(zeros[1] - printed[1]) < 5e-4
    assert abs(zeros[2] - 7.1558) < 1e-3 and abs(zeros[2] - printed[2]) > 1e-2


def webster_frequencies(a, b, k, open_end, n_modes, cells=20000):
    """Eigenfrequencies (wave speed 1, length 1) of Webster's equation for
    S = (a + b e^{kz})^2: p' = 0 at z = 0; p = 0 (open_end) or p' = 0 at z = 1.
    Cell-centred finite volumes, symmetrised generalised eigenproblem."""
    h = 1.0 / cells
    zc = (np.arange(cells) + 0.5) * h
    zf = np.arange(cells + 1) * h
    Sc = (a + b * np.exp(k * zc)) ** 2
    Sf = (a + b * np.exp(k * zf)) ** 2
    diag = np.zeros(cells)
    diag[:-1] += Sf[1:-1]
    diag[1:] += Sf[1:-1]
    if open_end:
        diag[-1] += 2.0 * Sf[-1]  # p = 0 on the end face (odd ghost)
    off = -Sf[1:-1]
    d = 1.0 / np.sqrt(Sc)
    lam = eigh_tridiagonal(diag * d * d / h ** 2, off * d[:-1] * d[1:] / h ** 2, select="i",
                           select_range=(0, n_modes), eigvals_only=True)
    f = np.sqrt(np.maximum(lam, 0.0)) / (2.0 * math.pi)
    return f[f > 1e-6][:n_modes]


def horn_spectrum(a, b, k, n, bell, steps, n_modes):
    """Axisymmetric horn (one theta node: the metric does not depend on
    theta, so this lattice is exactly the theta-independent part of any
    theta resolution), h_ref = h_z, plane pulse, probes along z."""
    nr, nz = n
    geom = W.trumpet_horn(c=0.1, a=a, b=b, k=k, n=(nr, 1, nz))
    geom["h_ref"] = 1.0 / nz
    geom["bc_hi"] = ("bounceback", "periodic", bell)
    o = oracle.Oracle(geom)
    tot = np.zeros(o.N)
    for ax in range(3):  # frozen-coefficient bound, as in the scheme pins
        m = o.Mhat[ax] + (np.abs(o.Mhat[4]) if ax in (0, 2) else 0.0)
        tot += np.where(m <= 1.0, 4.0, (1.0 + m) ** 2 / np.maximum(m, 1e-300))
    geom["c"] = 0.9 * 2.0 / math.sqrt(tot.max())
    o = oracle.Oracle(geom)
    # well inside the neutral range of the scheme (Mhat^dd below about 0.6)
    assert o.Mhat[0].max() < 0.15 and np.abs(o.Mhat[2]).max() < 1e-12
    z = W.node_grid(geom)[2]
    P0 = np.exp(-0.5 * ((z - 0.1) / 0.05) ** 2)
    i0 = int(round((0.63 - 0.05) / (0.95 / nr) - 0.5))
    probes = ((np.arange(8) + 0.5) * nz / 8).astype(np.int64) * nr + i0
    _, trace = o.run(o.init(P0), steps, probes)
    freq, _ = oracle.modes(trace, n_modes)
    return freq / (geom["c"] * geom["h_ref"])


def test_horn_modes_follow_webster():
    a, b, k = 0.06, 0.012, 2.0  # bell/mouth radius 2.07, bell slope 0.18
    closed = webster_frequencies(a, b, k, open_end=False, n_modes=4)
    # the flare matters at the level checked: a straight pipe has n/2
    assert abs(closed[0] / 0.5 - 1.0) > 0.015
    f = horn_spectrum(a, b, k, (16, 224), "bounceback", 16000, 4)
    err = np.abs(f / closed - 1.0)
    assert err.max() < 2.5e-3, err
    # pressure-release bell: the fundamental converges at first order (the
    # end condition on a flared bell), the other modes to the Webster level
    opened = webster_frequencies(a, b, k, open_end=True, n_modes=5)
    assert opened[0] / 0.25 - 1.0 > 0.2
    e1 = np.abs(horn_spectrum(a, b, k, (8, 112), "fixed", 8000, 5) / opened - 1.0)
    e2 = np.abs(horn_spectrum(a, b, k, (16, 224), "fixed", 16000, 5) / opened - 1.0)
    assert e2[0] < 0.025 and e1[0] / e2[0] > 1.6, (e1, e2)
    assert e2[1:].max() < 7e-3, e2


def torus_ring_frequency(R, rmin, rmax, nr=200, nphi=256):
    """Frequency (wave speed 1) of the cos(theta) mode of a torus of major
    radius R and minor radii [rmin, rmax]: smallest eigenvalue of the
    cross-section problem above, finite volumes on nr x nphi cells."""
    hr, hp = (rmax - rmin) / nr, 2.0 * math.pi / nphi
    r = rmin + (np.arange(nr) + 0.5) * hr
    rf = rmin + np.arange(nr + 1) * hr
    p = (np.arange(nphi) + 0.5) * hp
    idx = lambda i, j: i * nphi + (j % nphi)
    rows, cols, vals = [], [], []
    diag = np.zeros(nr * nphi)
    for i in range(nr):
        for j in range(nphi):
            k = idx(i, j)
            for ii, rface in ((i + 1, rf[i + 1]), (i - 1, rf[i])):
                if 0 <= ii < nr:  # no flux through the walls
                    w = rface * (R + rface * math.cos(p[j])) / hr ** 2
                    diag[k] += w
                    rows.append(k), cols.append(idx(ii, j)), vals.append(-w)
            for jj, pf in ((j + 1, p[j] + hp / 2), (j - 1, p[j] - hp / 2)):
                w = (R + r[i] * math.cos(pf)) / r[i] / hp ** 2
                diag[k] += w
                rows.append(k), cols.append(idx(i, jj)), vals.append(-w)
            diag[k] += r[i] / (R + r[i] * math.cos(p[j]))
    A = sparse.csr_matrix((vals, (rows, cols)), shape=(nr * nphi,) * 2) + sparse.diags(diag)
    rr, pp = np.meshgrid(r, p, indexing="ij")
    B = sparse.diags((rr * (R + rr * np.cos(pp))).ravel())
    lam = sparse_linalg.eigsh(A, k=1, M=B, sigma=0, which="LM", return_eigenvectors=False).min()
    return math.sqrt(lam) / (2.0 * math.pi)


def torus_ring_lbm(n, steps):
    """Oracle on a torus grid whose major-angle links are about one lattice
    unit long (the scheme's dispersion along an axis grows as Mhat -> -1),
    started from P0 = cos(theta); lowest spectral peak in physical units."""
    geom = dict(W.torus(c=0.1), n=n, h_ref=0.95 / n[0])
    o = oracle.Oracle(geom)
    tot = np.zeros(o.N)
    for ax in range(3):
        m = o.Mhat[ax] + (np.abs(o.Mhat[4]) if ax in (0, 2) else 0.0)
        tot += np.where(m <= 1.0, 4.0, (1.0 + m) ** 2 / np.maximum(m, 1e-300))
    geom["c"] = 0.9 * 2.0 / math.sqrt(tot.max())
    o = oracle.Oracle(geom)
    nr, nt, nph = n
    probes = np.array([i0 + nr * (i1 + nt * i2) for i0 in (0, nr // 2) for i1 in (0, nt // 8) for i2 in (0, nph // 2)])
    _, trace = o.run(o.init(np.cos(W.node_grid(geom)[1])), steps, probes)
    freq, _ = oracle.modes(trace, 2)
    return freq[0] / (geom["c"] * geom["h_ref"])


def test_torus_ring_mode_converges():
    R = W.torus()["params"][0]
    ref = torus_ring_frequency(R, 0.05, 1.0)
    assert abs(ref * 2.0 * math.pi * R - 1.0) > 0.01  # the cross-section matters at the level checked
    e1 = torus_ring_lbm((8, 128, 12), 5000) / ref - 1.0
    e2 = torus_ring_lbm((12, 192, 18), 7500) / ref - 1.0
    assert abs(e2) < 6e-3 and abs(e1) > 1.5 * abs(e2), (e1, e2)
