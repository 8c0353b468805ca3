"""Pins for the oracle's free wall (CPU only).

Sec. IV.A imposes a free boundary at the open end of the pipe, and at the
inner radius that excludes the axis, by copying the values of the
neighbouring cell normal to the surface; the conclusions use free walls at
every open end.  Reading taken (oracle and kernels alike): the ghost node one
link beyond the wall is a copy of the boundary node after its collision, so
the population that enters the boundary node x_e through the wall is x_e's
own post-collision population in that direction, f_l(x_e, t+1) = f*_l(x_e),
and the metric stress beyond the wall is x_e's own (an even mirror).  Pins:

* per-step identity: the population that enters x_e through a free wall and
  the one x_e streams to its inner neighbour are the same post-collision
  value, so after every step f_l(x_e) = f_l(x_e + xi_l) exactly, on a
  curvilinear grid (a copy of the opposite population or of the inner
  neighbour breaks it);
* the exact periodic steady state of a line driven at one end and free at
  the other, with the identity metric and with a constant metric stress
  along the line (unequal spacings, Mhat^zz = (h_ref / h_z)^2 - 1): a
  separate 1-D implementation of the step gives the one-step matrix A, and
  the phasor of the state after each imposition solves
  (e^{i w} I - Pi A) X = C b e^{i w}, solved in the frequency domain;
* the closed-form reflection of a lattice plane wave at the free end
  (identity metric).  At frequency w, with z = e^{i w} and
  kappa = c^2 (z + 1) / (z - 1 + 2 c^2), the scheme's moving populations
  admit exactly two plane waves lambda^x, lambda + 1/lambda =
  (z^2 + 2 kappa - 1) / (z kappa) (no evanescent ones), and the free rule
  fixes their ratio, so the pressure wave reflects with
  R = lambda^-2 (z / lambda - 1)(z lambda - kappa) /
      ((z / lambda - kappa)(z lambda - 1)),
  referred to the wall half a link beyond the last node, lambda = e^{-ik}
  the incident wave.  As w -> 0, R -> -(1 - c)/(1 + c): a pressure-release
  end that absorbs part of the wave (a third at c = 1/2 is reflected);
* planted mistakes, compiled into copies of the oracle: an odd metric-stress
  mirror at free walls, a copy of the opposite population, a copy of the
  inner neighbour's population; each fails the steady-state pin;
* finding: at a wall where sqrt(g) falls outward (the pipe's inner radius,
  Sec. IV.A; the torus's inner radius, Sec. IV.C) the copy reading is not
  neutral: on the paper's pipe the radial operator with a free inner wall
  has spectral radius 1.0054 at c = 0.1 (a bounce-back wall: 1 to round-off).
  Scaling the copy by sqrt(g)(ghost) / sqrt(g)(x_e) (copying P and J'
  instead of the populations) removes that growth but makes the flaring
  bell of the benchmark horn grow (tenfold per 1000 steps on its coarse
  grid), where the plain copy is bounded (the ensemble horn check in
  test_oracle_scheme).  No single copy reading runs every free wall of the
  paper stably, so the copy reading stays and the sweeps use reflecting
  inner walls.
"""
import math
import os
import subprocess

import numpy as np
import pytest

import oracle
import workloads as W


# ---------------------------------------------------------------------------
# separate 1-D implementation of the step for the pins
# ---------------------------------------------------------------------------

def line_geom(N, c, hz, D, hi="free"):
    """1 x 1 x N box (x and y periodic single nodes), lattice unit 1, axial
    spacing hz (Mhat^zz = 1 / hz^2 - 1), damped bounce-back at z = 0."""
    return dict(kind="box", dim=3, n=(1, 1, N), qmin=(0.0, 0.0, 0.0), qmax=(1.0, 1.0, N * hz),
                bc_lo=("periodic", "periodic", "bounceback"), bc_hi=("periodic", "periodic", hi),
                h_ref=1.0, c=c, damp=D, params=())


def line_step(f, c, m, D):
    """One step on the line: f[7, N] in the order rest, +x, -x, +y, -y, +z,
    -z; constant metric stress c^2 S m along z (central difference, the
    value beyond either end mirrored evenly); the +z population reflects at
    z = 0 with damping D; the free end z = N - 1 feeds -z with the node's
    own post-collision -z population."""
    c2 = c * c
    S = f.sum(axis=0)
    out = np.empty_like(f)
    out[0] = 2.0 * (1.0 - 3.0 * c2) * S - f[0]
    for p, q in ((1, 2), (3, 4)):
        K = f[p] - f[q]
        out[p] = c2 * S + K - f[p]
        out[q] = c2 * S - K - f[q]
    A = c2 * m * S
    A_up = np.append(A[1:], A[-1])
    A_dn = np.insert(A[:-1], 0, A[0])
    K = f[5] - f[6] - 0.25 * (A_up - A_dn)
    out[5] = c2 * S + K - f[5]
    out[6] = c2 * S - K - f[6]
    g = out.copy()
    g[5, 1:] = out[5, :-1]
    g[6, :-1] = out[6, 1:]
    g[5, 0] = D * out[6, 0]
    g[6, -1] = out[6, -1]
    return g


def steady_phasors(N, c, m, D, omega, C):
    """Phasor X[7, N] of the periodic steady state, pressure source at node 0."""
    n = 7 * N
    A = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        A[:, j] = line_step(e.reshape(7, N), c, m, D).reshape(-1)
    keep = np.ones(n)
    keep[np.arange(7) * N] = 0.0
    b = np.zeros(n)
    b[0] = 1.0 - 3.0 * c * c
    b[np.arange(1, 7) * N] = 0.5 * c * c
    z = np.exp(1j * omega)
    return np.linalg.solve(z * np.eye(n) - keep[:, None] * A, C * b * z).reshape(7, N)


def steady_residual(o, N, c, m, D, omega, T=16000, win=400, C=1.1):
    """Largest deviation of the oracle's late trace from the exact steady
    state, relative to the steady amplitude, over four probes."""
    probes = [1, N // 3, 2 * N // 3, N - 1]
    Z = steady_phasors(N, c, m, D, omega, C)[:, probes].sum(axis=0)
    f = o.init(np.zeros(o.N))
    _, tr = o.run(f, T, probes, sources=[0], amplitude=C, omega=omega)
    t = np.arange(T - win, T)
    steady = np.imag(Z[None, :] * np.exp(1j * omega * t)[:, None])
    return float((np.abs(tr[T - win:] - steady).max(axis=0) / np.abs(Z)).max())


LINE_CASES = [(1.0, 0.05), (1.0, 0.21), (1.25, 0.05), (1.25, 0.17), (0.8, 0.09)]   # (h_z, omega)


@pytest.mark.parametrize("hz,omega", LINE_CASES)
def test_free_end_line_reaches_exact_steady_state(hz, omega):
    N, c, D = 36, 0.5, 0.65
    m = 1.0 / hz ** 2 - 1.0
    o = oracle.Oracle(line_geom(N, c, hz, D))
    assert abs(o.Mhat[2][0] - m) < 1e-12
    # the residual is the slowly fading switch-on transient (measured
    # <= 3.6e-4 of the steady amplitude after 16000 steps)
    assert steady_residual(o, N, c, m, D, omega) <= 1e-3


def plane_wave_reflection(omega, c):
    z = np.exp(1j * omega)
    kap = c * c * (z + 1.0) / (z - 1.0 + 2.0 * c * c)
    roots = np.roots([z * kap, -(z * z + 2.0 * kap - 1.0), z * kap])
    lam = roots[np.argmin(np.angle(roots))]          # e^{-ik}, k > 0: the incident wave
    R = lam ** -2 * (z / lam - 1.0) * (z * lam - kap) / ((z / lam - kap) * (z * lam - 1.0))
    return lam, R


@pytest.mark.parametrize("c,omega", [(0.3, 0.05), (0.3, 0.2), (0.5, 0.05), (0.5, 0.3), (0.55, 0.12)])
def test_free_end_reflects_plane_waves_in_closed_form(c, omega):
    """The oracle's steady state on a driven line splits into an incident and
    a reflected plane wave of the lattice whose ratio at the free end is the
    closed form R(omega)."""
    N, D, T, C = 40, 0.65, 16000, 1.0
    lam, R = plane_wave_reflection(omega, c)
    assert abs(abs(lam) - 1.0) < 1e-12                               # propagating
    o = oracle.Oracle(line_geom(N, c, 1.0, D))
    xs = np.arange(2, N)                                             # nodes off the source
    f = o.init(np.zeros(o.N))
    P = 2 * math.ceil(2 * math.pi / omega)                           # two periods or more
    _, tr = o.run(f, T, xs, sources=[0], amplitude=C, omega=omega)
    # demodulate the late window: S(x, t) = Im(X(x) e^{i w t})
    t = np.arange(T - P, T)
    basis = np.stack([np.sin(omega * t), np.cos(omega * t)], axis=1)
    coef, *_ = np.linalg.lstsq(basis, tr[T - P:], rcond=None)
    X = coef[0] + 1j * coef[1]
    M = np.stack([lam ** xs, lam ** (-xs)], axis=1)
    amp, *_ = np.linalg.lstsq(M, X, rcond=None)
    # two plane waves and nothing else, up to the fading switch-on transient
    # (measured <= 1.7e-5 after 16000 steps)
    assert np.abs(M @ amp - X).max() <= 1e-4 * np.abs(X).max()
    xw = N - 0.5
    R_meas = amp[1] * lam ** (-xw) / (amp[0] * lam ** xw)
    assert abs(R_meas - R) <= 1e-5 * abs(R), (R_meas, R)             # measured <= 3.8e-7
    # low-frequency limit of the closed form: -(1 - c)/(1 + c)
    _, R0 = plane_wave_reflection(1e-4, c)
    assert abs(R0 + (1.0 - c) / (1.0 + c)) < 1e-3


def test_free_wall_feeds_the_inner_neighbours_population():
    """After every step the population entering a free wall node equals what
    that node sent to its inner neighbour (both are its post-collision
    value), on a curvilinear grid (r and z free walls of a horn)."""
    geom = W.trumpet_horn(c=0.3, a=0.08, b=0.01, k=2.0, n=(9, 6, 11))
    geom["bc_lo"] = ("free", "periodic", "bounceback")
    o = oracle.Oracle(geom)
    n0, n1, n2 = o.shape
    f = np.random.default_rng(4).uniform(-1, 1, (o.Q, o.N))
    for _ in range(3):
        o.step(f, 1)
        F = f.reshape(o.Q, n2, n1, n0)
        assert np.array_equal(F[1, :, :, 0], F[1, :, :, 1])              # +e0 enters at r_min
        assert np.array_equal(F[6, n2 - 1, :, :], F[6, n2 - 2, :, :])    # -e2 enters at the bell


# ---------------------------------------------------------------------------
# planted mistakes, compiled into copies of the oracle
# ---------------------------------------------------------------------------

FREE_BRANCH = "f[l * N + n] = fs[l * N + n];"
PLANTS = {
    "odd_stress_mirror": ("Aside[side] = (bc == ORC_FIXED) ? -Ahere : Ahere;",
                          "Aside[side] = (bc == ORC_FIXED || bc == ORC_FREE) ? -Ahere : Ahere;"),
    "opposite_population": (FREE_BRANCH, "f[l * N + n] = fs[orc_opposite(l) * N + n];"),
    "inner_neighbour": (FREE_BRANCH,
                        "{ int bq = 0; int64_t in = orc_neighbour(g, idx, orc_axis_of(l), orc_sign_of(l), &bq);"
                        " f[l * N + n] = fs[l * N + (in >= 0 ? in : n)]; }"),
}


@pytest.fixture(scope="module")
def planted(tmp_path_factory):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "lbw_oracle.c")).read()
    out = {}
    d = tmp_path_factory.mktemp("planted")
    for name, (old, new) in PLANTS.items():
        assert src.count(old) == 1, name
        path = d / ("%s.c" % name)
        path.write_text(src.replace(old, new))
        so = str(d / ("%s.so" % name))
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", so, str(path), "-lm"])
        out[name] = oracle.load_library(so)
    return out


@pytest.mark.parametrize("name", sorted(PLANTS))
def test_planted_free_wall_mistakes_fail_the_steady_state_pin(planted, name):
    N, c, D, hz, omega = 36, 0.5, 0.65, 1.25, 0.17
    m = 1.0 / hz ** 2 - 1.0
    bad = oracle.Oracle(line_geom(N, c, hz, D), lib=planted[name])
    r = steady_residual(bad, N, c, m, D, omega)
    assert not r <= 1e-2, r            # misses the steady state, or diverges (the odd mirror: NaN)


# ---------------------------------------------------------------------------
# finding: the copy reading at an inner radial wall
# ---------------------------------------------------------------------------

def radial_line(lo, c):
    """The paper's pipe reduced to its axisymmetric, z-uniform part: r in
    [1, 25] with 20 cells, one theta and one z node (both periodic), one
    lattice unit per radial cell, outer wall reflecting without loss."""
    return dict(kind="cylinder", dim=3, n=(20, 1, 1), qmin=(1.0, 0.0, 0.0), qmax=(25.0, 2 * math.pi, 1.0),
                bc_lo=(lo, "periodic", "periodic"), bc_hi=("bounceback", "periodic", "periodic"),
                h_ref=1.2, c=c, damp=1.0, params=())


def spectral_radius(geom):
    o = oracle.Oracle(geom)
    n = o.Q * o.N
    A = np.empty((n, n))
    for j in range(n):
        f = np.zeros(n)
        f[j] = 1.0
        f = f.reshape(o.Q, o.N).copy()
        o.step(f, 1)
        A[:, j] = f.reshape(-1)
    return float(np.abs(np.linalg.eigvals(A)).max())


def test_copy_reading_grows_at_an_inner_radial_wall():
    assert spectral_radius(radial_line("bounceback", 0.1)) <= 1.0 + 1e-12
    assert spectral_radius(radial_line("fixed", 0.1)) <= 1.0 + 1e-12
    rho = spectral_radius(radial_line("free", 0.1))
    assert 1.004 < rho < 1.007, rho
