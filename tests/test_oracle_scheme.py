"""Pins for the oracle's time step (CPU only).

* identity metric: with g = I the scheme must be Chopard's Cartesian wave LBM
  (Sec. II, moment-matching equilibrium), written here independently with the
  textbook D3Q7 weights w0 = 1/4, w = 1/8;
* box eigenmodes: on a box with half-way bounce-back (or anti-bounce-back)
  walls a cosine (sine) mode evolves exactly as the periodic plane wave of the
  mirrored lattice, whose one-step amplification has the closed form
      cos(omega) = 1 - (c^2/2) sum_d [4 sin^2(k_d/2) + m_d sin^2(k_d)],
  m_d = Mhat^dd = (h_ref/h_d)^2 - 1; unequal spacings make m_d != 0 and so
  fix the sign and factor of the gradient force;
* invariants: sum_x sqrt(g) P is conserved in closed domains (curvilinear
  continuity equation, Sec. III); damping, free and fixed walls break it;
* linearity and mirror symmetry; stability at the configured c and
  divergence above the bound;
* index maps enumerated by brute force on tiny grids.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def box(n, h, bc_lo, bc_hi, c, damp=1.0, ref_axis=0):
    d = len(n)
    return dict(kind="box", dim=d, n=tuple(n), qmin=(0.0,) * d, qmax=tuple(n[a] * h[a] for a in range(d)),
                bc_lo=tuple(bc_lo), bc_hi=tuple(bc_hi), h_ref=h[ref_axis], c=c, damp=damp, params=())


# ---------------------------------------------------------------------------
# identity metric == Chopard's Cartesian wave LBM
# ---------------------------------------------------------------------------

def chopard_d3q7(P0, c, steps, walls):
    """Chopard-Luthi-Wagen wave LBM (Sec. II moment-matching equilibrium),
    tau = 1/2, D3Q7 with w0 = 1/4, w_i = 1/8, c_s^2 = sum_i w_i xi_x^2 = 1/4.
    P0 has array shape (n2, n1, n0).  walls: 'periodic' or 'bounceback' on
    every face.  Returns populations in the oracle's order and layout."""
    w0, wi, cs2 = 0.25, 0.125, 0.25
    vel = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    P = P0.copy()
    J = [np.zeros_like(P) for _ in range(3)]

    def feq(P, J):
        out = [P + (c * c / cs2) * P * (w0 - 1.0)]
        for v in vel[1:]:
            xiJ = v[0] * J[0] + v[1] * J[1] + v[2] * J[2]
            out.append((wi / cs2) * (c * c * P + xiJ))
        return out

    f = feq(P, J)
    for _ in range(steps):
        P = sum(f)
        J = [sum(fl * v[a] for fl, v in zip(f, vel)) for a in range(3)]
        fe = feq(P, J)
        fs = [2.0 * a - b for a, b in zip(fe, f)]
        new = [fs[0]]
        for l, v in enumerate(vel[1:], start=1):
            ax = [a for a in range(3) if v[a] != 0][0]
            s = v[ax]
            arr_ax = 2 - ax
            moved = np.roll(fs[l], s, axis=arr_ax)
            if walls == "bounceback":
                opp = l + 1 if l % 2 == 1 else l - 1
                idx = [slice(None)] * 3
                idx[arr_ax] = 0 if s > 0 else -1
                moved[tuple(idx)] = fs[opp][tuple(idx)]
            new.append(moved)
        f = new
    return np.stack([fl.reshape(-1) for fl in f])


@pytest.mark.parametrize("walls", ["periodic", "bounceback"])
def test_identity_metric_is_chopard(walls):
    n = (9, 7, 6)
    c = 0.5
    geom = box(n, (1.0, 1.0, 1.0), (walls,) * 3, (walls,) * 3, c)
    rng = np.random.default_rng(5)
    P0 = rng.normal(size=n[::-1])
    o = oracle.Oracle(geom)
    f = o.init(P0.reshape(-1))
    o.step(f, 200)
    ref = chopard_d3q7(P0, c, 200, walls)
    assert np.abs(f - ref).max() <= 1e-12 * np.abs(ref).max()


# ---------------------------------------------------------------------------
# box eigenmodes (closed-form dispersion)
# ---------------------------------------------------------------------------

def omega_closed_form(c, k, m, sign=+1.0):
    s = sum(4.0 * math.sin(kd / 2) ** 2 + sign * md * math.sin(kd) ** 2 for kd, md in zip(k, m))
    return math.acos(1.0 - 0.5 * c * c * s)


def fit_residual(trace, omega):
    """Relative residual of the least-squares fit of each probe trace by
    {1, (-1)^t, cos(omega t), sin(omega t)} (the eigenvalues 1, -1, e^{+-i omega}
    of the one-step map at this wave vector)."""
    t = np.arange(trace.shape[0])
    B = np.stack([np.ones_like(t, dtype=float), (-1.0) ** t, np.cos(omega * t), np.sin(omega * t)], axis=1)
    coef, *_ = np.linalg.lstsq(B, trace, rcond=None)
    return np.abs(trace - B @ coef).max() / np.abs(trace).max()


def mode_field(geom, kind_per_axis, mvec):
    shape = W.shape_of(geom)
    d = len(shape)
    fields = []
    for a in range(d):
        i = np.arange(shape[a]) + 0.5
        k = math.pi * mvec[a] / shape[a]
        fields.append(np.cos(k * i) if kind_per_axis[a] == "cos" else np.sin(k * i))
    grids = np.meshgrid(*fields[::-1], indexing="ij")
    P = np.ones_like(grids[0])
    for g in grids:
        P = P * g
    return P.reshape(-1), [math.pi * mvec[a] / shape[a] for a in range(d)]


@pytest.mark.parametrize("case", [
    # (n, h, walls per axis, mode numbers)
    ((12, 10, 8), (1.0, 0.8, 1.3), ("bounceback", "bounceback", "bounceback"), (1, 2, 1)),
    ((12, 10, 8), (1.0, 1.25, 0.7), ("fixed", "bounceback", "fixed"), (2, 1, 1)),
    ((16, 12), (1.0, 0.6), ("bounceback", "fixed"), (3, 2)),
    ((16, 12), (0.9, 1.0), ("fixed", "fixed"), (1, 1)),
])
def test_box_mode_follows_closed_form_dispersion(case):
    n, h, walls, mvec = case
    d = len(n)
    href = h[0]
    m = [(href / h[a]) ** 2 - 1.0 for a in range(d)]
    # stay inside the stability bound
    B = sum(4.0 if md <= 1 else (1 + md) ** 2 / md for md in m)
    c = 0.8 * 2.0 / math.sqrt(B)
    geom = box(n, h, walls, walls, c)
    kinds = ["cos" if w == "bounceback" else "sin" for w in walls]
    P0, k = mode_field(geom, kinds, mvec)
    o = oracle.Oracle(geom)
    assert np.abs(o.Mhat[:d] - np.array(m)[:, None]).max() < 1e-14
    f = o.init(P0)
    probes = np.random.default_rng(1).integers(0, o.N, size=6)
    _, trace = o.run(f, 300, probes)
    om = omega_closed_form(c, k, m)
    assert fit_residual(trace, om) < 1e-10
    if any(abs(md) > 0.1 for md in m):
        # the printed '+' sign of the gradient term would give another frequency
        om_plus = omega_closed_form(c, k, m, sign=-1.0)
        assert fit_residual(trace, om_plus) > 1e-3


# ---------------------------------------------------------------------------
# invariant, linearity, symmetry
# ---------------------------------------------------------------------------

def small_cylinder(bc_r=("bounceback", "bounceback"), bc_z=("bounceback", "bounceback"), damp=1.0, n=(10, 12, 14)):
    g = W.closed_cylinder(c=0.3)
    g.update(n=n, bc_lo=(bc_r[0], "periodic", bc_z[0]), bc_hi=(bc_r[1], "periodic", bc_z[1]), damp=damp)
    return g


def test_invariant_conserved_in_closed_domain():
    geom = small_cylinder()
    o = oracle.Oracle(geom)
    rng = np.random.default_rng(2)
    f = o.init(1.0 + rng.uniform(-1, 1, o.N))
    I0 = o.invariant(f)
    scale = np.abs(f).sum()
    for _ in range(10):
        o.step(f, 1000)
        assert abs(o.invariant(f) - I0) <= 1e-12 * scale


@pytest.mark.parametrize("variant", ["damped", "free", "fixed"])
def test_invariant_broken_by_open_walls(variant):
    if variant == "damped":
        geom = small_cylinder(damp=0.9)
    elif variant == "free":
        geom = small_cylinder(bc_z=("bounceback", "free"))
    else:
        geom = small_cylinder(bc_r=("bounceback", "fixed"))
    o = oracle.Oracle(geom)
    f = o.init(1.0 + np.random.default_rng(2).uniform(0, 1, o.N))
    I0 = o.invariant(f)
    o.step(f, 200)
    assert abs(o.invariant(f) - I0) > 1e-3 * abs(I0)


def test_collision_keeps_zeroth_moment_and_is_linear():
    geom = W.trumpet_horn(c=0.2, n=(8, 6, 10))
    o = oracle.Oracle(geom)
    rng = np.random.default_rng(3)
    f = rng.normal(size=(o.Q, o.N))
    g = rng.normal(size=(o.Q, o.N))
    a, b = 0.7, -1.3
    h = a * f + b * g
    for x in (f, g, h):
        o.step(x, 5)
    assert np.abs(h - (a * f + b * g)).max() < 1e-12 * np.abs(h).max()


def test_mirror_symmetry_in_theta():
    """theta -> -theta maps the cylinder and horn onto themselves; a
    mirror-symmetric state stays mirror-symmetric."""
    for geom in (small_cylinder(), W.trumpet_horn(c=0.2, n=(8, 12, 10))):
        o = oracle.Oracle(geom)
        n0, n1, n2 = o.shape
        P = np.random.default_rng(4).normal(size=(n2, n1, n0))
        mirror = (-np.arange(n1)) % n1
        P = P + P[:, mirror, :]
        f = o.init(P.reshape(-1))
        o.step(f, 50)
        F = f.reshape(o.Q, n2, n1, n0)
        Fm = F[:, :, mirror, :][[0, 1, 2, 4, 3, 5, 6]]  # theta directions swap under the mirror
        assert np.abs(F - Fm).max() < 1e-12 * np.abs(F).max()


def leapfrog_bound(o):
    tot = np.zeros(o.N)
    for a in range(o.dim):
        m = o.Mhat[a] + (np.abs(o.Mhat[4]) if o.dim == 3 and a in (0, 2) else 0.0)
        tot += np.where(m <= 1.0, 4.0, (1.0 + m) ** 2 / np.maximum(m, 1e-300))
    return 2.0 / math.sqrt(tot.max())


@pytest.mark.parametrize("kind", ["cylinder", "horn", "torus"])
def test_stable_below_bound_unstable_above(kind):
    if kind == "cylinder":
        geom = small_cylinder(n=(12, 16, 10))
    elif kind == "horn":
        geom = W.trumpet_horn(c=0.2, n=(10, 12, 16))
    else:
        geom = dict(W.torus(c=0.1), n=(10, 16, 24))
    cmax = leapfrog_bound(oracle.Oracle(geom))
    rng = np.random.default_rng(6)
    grow = {}
    for fac in (0.9, 1.1):
        g = dict(geom, c=fac * cmax)
        o = oracle.Oracle(g)
        f = rng.normal(size=(o.Q, o.N))
        n0 = np.abs(f).max()
        o.step(f, 3000)
        grow[fac] = np.abs(f).max() / n0
    assert grow[0.9] < 20.0, grow
    assert not np.isfinite(grow[1.1]) or grow[1.1] > 1e6, grow


# ---------------------------------------------------------------------------
# index maps (brute force on tiny grids)
# ---------------------------------------------------------------------------

BC = {"periodic": 0, "bounceback": 1, "free": 2, "fixed": 3}


def brute_maps(geom):
    shape = W.shape_of(geom)
    d = len(shape)
    Q = 2 * d + 1
    N = int(np.prod(shape))
    mask = np.zeros(N, np.uint8)
    pull = np.zeros((Q, N), np.int32)
    for n in range(N):
        idx = []
        r = n
        for a in range(d):
            idx.append(r % shape[a])
            r //= shape[a]
        pull[0, n] = n
        for l in range(1, Q):
            a = (l - 1) // 2
            s = 1 if l % 2 == 1 else -1
            # outgoing link
            j = idx[a] + s
            if not (0 <= j < shape[a]) and geom["bc_lo" if s < 0 else "bc_hi"][a] != "periodic":
                mask[n] |= 1 << (l - 1)
            # incoming link: from idx - xi_l
            src = list(idx)
            src[a] = idx[a] - s
            if 0 <= src[a] < shape[a]:
                pass
            else:
                face = "bc_lo" if s > 0 else "bc_hi"
                code = geom[face][a]
                if code == "periodic":
                    src[a] %= shape[a]
                else:
                    pull[l, n] = -(1 + BC[code])
                    continue
            lin = 0
            for b in reversed(range(d)):
                lin = lin * shape[b] + src[b]
            pull[l, n] = lin
    return mask, pull


@pytest.mark.parametrize("geom", [
    box((3, 4, 5), (1, 1, 1), ("bounceback", "periodic", "free"), ("fixed", "periodic", "bounceback"), 0.3),
    box((4, 3), (1, 1), ("periodic", "fixed"), ("periodic", "bounceback"), 0.3),
    box((1, 3, 2), (1, 1, 1), ("bounceback", "periodic", "periodic"), ("free", "periodic", "periodic"), 0.3),
])
def test_maps_brute_force(geom):
    o = oracle.Oracle(geom)
    mask, pull = o.maps()
    bm, bp = brute_maps(geom)
    assert np.array_equal(mask, bm)
    assert np.array_equal(pull, bp)


def test_maps_explicit_entries():
    geom = box((3, 4, 5), (1, 1, 1), ("bounceback", "periodic", "free"), ("fixed", "periodic", "bounceback"), 0.3)
    o = oracle.Oracle(geom)
    mask, pull = o.maps()
    # node (0,0,0): +e0 arrives through the bounce-back low wall of axis 0
    assert pull[1, 0] == -2
    # node (2,0,0): -e0 arrives through the fixed high wall
    assert pull[2, 2] == -4
    # node (0,0,0): +e1 arrives from (0,3,0) by periodic wrap; -e1 from (0,1,0)
    assert pull[3, 0] == 9 and pull[4, 0] == 3
    # node (0,0,0): +e2 arrives through the free low wall of axis 2
    assert pull[5, 0] == -3
    # node (0,0,4): -e2 arrives through the bounce-back high wall of axis 2
    assert pull[6, 48] == -2
    # outgoing wall crossings at the corner node (2,3,4): +e0 and +e2
    assert mask[59] == (1 << 0) | (1 << 4)


def test_gradient_force_coefficient_threshold():
    """The scheme is only neutrally stable while Mhat^dd stays below about
    0.6 on an axis whose coefficients vary along it: there the two-link-wide
    stencil of the gradient force and the one-link Christoffel force no longer
    pair into a symmetric operator.  A cylinder whose lattice unit is longer
    than its radial link (Mhat^rr = 1.25) grows; the same cylinder with the
    radial link as lattice unit (Mhat^rr = 0) does not."""
    def growth(h_ref_over_hr):
        g = small_cylinder(n=(10, 12, 16))
        hr = (g["qmax"][0] - g["qmin"][0]) / g["n"][0]
        g["h_ref"] = h_ref_over_hr * hr
        g["qmax"] = (g["qmax"][0], g["qmax"][1], 16 * hr)  # h_z = h_r
        g["c"] = 0.5 * leapfrog_bound(oracle.Oracle(g))
        o = oracle.Oracle(g)
        f = np.random.default_rng(9).normal(size=(o.Q, o.N))
        n0 = np.sqrt((f * f).sum())
        o.step(f, 3000)
        return np.sqrt((f * f).sum()) / n0, o.Mhat[0].max()
    g_bad, m_bad = growth(1.5)
    g_ok, m_ok = growth(1.0)
    assert m_bad > 1.0 and g_bad > 1e3
    assert abs(m_ok) < 1e-14 and g_ok < 2.0


def test_ensemble_horn_lattice_unit():
    """Ensemble horns take h_z as lattice unit on a grid whose radial links
    are nowhere shorter than h_z, so Mhat^zz = 0, Mhat^rr <= 0 and
    |Mhat^rz| < 1 (checked with the oracle's tables for a sample of the
    training ensemble).  The same horn with the mouthpiece's radial link as
    unit on a fine axial grid (Mhat^zz > 0.6 along the flare) grows; on its
    ensemble grid it does not.  The runs use one theta node: the metric does
    not depend on theta, so this lattice is exactly the axisymmetric part of
    any theta resolution."""
    for m in W.ensemble(512)[::16]:
        n0, _, n2 = m["geom"]["n"]
        assert m["geom"]["h_ref"] == 1.0 / n2 and n0 % 8 == 0 and n0 >= 16
        o = oracle.Oracle(dict(m["geom"], n=(n0, 1, n2), c=0.1))
        assert np.abs(o.Mhat[2]).max() < 1e-12
        assert o.Mhat[0].max() <= 1e-12 and np.abs(o.Mhat[4]).max() < 1.0

    a, b, k = 0.19, 0.03, 2.0
    hr = 0.95 / 32

    def growth(n, h_ref):
        g = W.trumpet_horn(c=0.1, a=a, b=b, k=k, n=n)
        g["h_ref"] = h_ref
        g["c"] = 0.9 * leapfrog_bound(oracle.Oracle(g))
        o = oracle.Oracle(g)
        f = np.random.default_rng(3).normal(size=(o.Q, o.N))
        n_start = np.sqrt((f * f).sum())
        o.step(f, 6000)
        return np.sqrt((f * f).sum()) / n_start, o

    g_bad, o_bad = growth((32, 1, 224), (a + b) * hr / math.sqrt(1.0 + (b * k) ** 2))
    assert o_bad.Mhat[2].max() > 0.6 and g_bad > 5.0, g_bad
    n_ok = W.horn_grid((a, b, k), 1, 224)
    g_ok, _ = growth(n_ok, 1.0 / n_ok[2])
    assert g_ok < 1.2, g_ok
