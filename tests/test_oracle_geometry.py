"""Pins for the oracle's geometry coefficients (CPU only).

The oracle derives sqrt(g), the inverse metric and the contracted Christoffel
symbols from the coordinate embeddings.  These tests hold them against
(1) the metric tensors and Christoffel symbols the paper prints for the
cylinder, the Bessel horn and the torus (Sec. IV.A-C), with the printed typos
corrected as noted per case, and (2) the identity
Gamma^i_jk g^jk = -(1/sqrt g) d_j (sqrt g g^ij), checked by central
differences on the oracle's own per-node fields.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _lattice(gmat, gam, h, href):
    """Paper-side conversion: metric g_ij and Christoffel Gamma^i_jk at one
    point -> (sqrtg, Mhat in plane order 00,11,22,01,02,12, Gamh)."""
    d = gmat.shape[0]
    G = np.linalg.inv(gmat)
    sg = math.sqrt(np.linalg.det(gmat))
    Gc = np.einsum("ijk,jk->i", gam, G)
    M = href * href * G / np.outer(h, h) - np.eye(d)
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    Mv = np.array([M[i, j] if i < d and j < d else 0.0 for i, j in pairs])
    Gv = np.zeros(3)
    Gv[:d] = href * href * Gc / h
    return sg, Mv, Gv


def _compare(geom, paper_point):
    o = oracle.Oracle(geom)
    d = geom["dim"]
    h = np.array(o.spacing())
    href = geom["h_ref"]
    q = W.node_grid(geom)
    worst = 0.0
    for n in range(o.N):
        gmat, gam = paper_point([qq[n] for qq in q])
        sg, Mv, Gv = _lattice(np.asarray(gmat, float), np.asarray(gam, float), h, href)
        scale_m = max(1.0, np.abs(Mv).max())
        scale_g = max(1.0, np.abs(Gv).max())
        worst = max(worst, abs(o.sqrtg[n] - sg) / sg, np.abs(o.Mhat[:, n] - Mv).max() / scale_m,
                    np.abs(o.Gamh[:, n] - Gv).max() / scale_g)
    return worst


def _cyl_paper(q):
    # Sec. IV.A: g = diag(1, r^2, 1); Gamma^r_thth = -r, Gamma^th_rth = Gamma^th_thr = 1/r
    r = q[0]
    g = np.diag([1.0, r * r, 1.0])
    gam = np.zeros((3, 3, 3))
    gam[0, 1, 1] = -r
    gam[1, 0, 1] = gam[1, 1, 0] = 1.0 / r
    return g, gam


def _polar_paper(q):
    g, gam = _cyl_paper([q[0], q[1], 0.0])
    return g[:2, :2], gam[:2, :2, :2]


def _bessel_horn_paper(lam, zmax, fix_typo=True):
    # Sec. IV.B, Bessel horn metric and Christoffel symbols, Z = Zmax - z.
    # The printed Gamma^th_zth = lambda / Z^2 is a typo for lambda / Z (the
    # log-derivative of the radius Z^-lambda); fix_typo=False keeps the print.
    def point(q):
        r, _, z = q
        Z = zmax - z
        g = np.array([[Z ** (-2 * lam), 0.0, Z ** (-2 * lam - 1) * lam * r],
                      [0.0, Z ** (-2 * lam) * r * r, 0.0],
                      [Z ** (-2 * lam - 1) * lam * r, 0.0, (Z ** (-2 * lam) * lam * lam * r * r + Z * Z) / (Z * Z)]])
        gam = np.zeros((3, 3, 3))
        gam[0, 0, 2] = gam[0, 2, 0] = lam / Z
        gam[0, 2, 2] = r * lam * (lam + 1) / (Z * Z)
        gam[1, 2, 1] = gam[1, 1, 2] = lam / Z if fix_typo else lam / (Z * Z)
        gam[0, 1, 1] = -r
        gam[1, 0, 1] = gam[1, 1, 0] = 1.0 / r
        return g, gam
    return point


def _torus_paper(R, fix_typo=True):
    # Sec. IV.C, torus metric diag(1, (R + r cos phi)^2, r^2) and Christoffel
    # symbols.  Printed Gamma^r_thth = +(R + r cos phi) cos phi has the wrong
    # sign (the centripetal term points inwards); the printed
    # "Gamma_phi^{thth}" is read as Gamma^phi_thth.
    def point(q):
        r, _, f = q
        u = R + r * math.cos(f)
        g = np.diag([1.0, u * u, r * r])
        gam = np.zeros((3, 3, 3))
        gam[0, 1, 1] = (-u if fix_typo else u) * math.cos(f)
        gam[0, 2, 2] = -r
        gam[1, 0, 1] = gam[1, 1, 0] = math.cos(f) / u
        gam[1, 1, 2] = gam[1, 2, 1] = -math.sin(f) * r / u
        gam[2, 0, 2] = gam[2, 2, 0] = 1.0 / r
        gam[2, 1, 1] = u * math.sin(f) / r
        return g, gam
    return point


def _geom(kind, dim, n, qmin, qmax, bc_lo, bc_hi, ref_axis=0, params=()):
    h_ref = (qmax[ref_axis] - qmin[ref_axis]) / n[ref_axis]
    return dict(kind=kind, dim=dim, n=n, qmin=qmin, qmax=qmax, bc_lo=bc_lo, bc_hi=bc_hi, h_ref=h_ref,
                c=0.3, damp=1.0, params=params)


def test_cylinder_matches_printed_metric():
    geom = _geom("cylinder", 3, (6, 5, 4), (0.4, 0.0, 0.0), (2.0, 2 * math.pi, 3.0),
                 ("bounceback", "periodic", "bounceback"), ("bounceback", "periodic", "free"))
    assert _compare(geom, _cyl_paper) < 1e-13


def test_polar_matches_printed_metric():
    geom = _geom("polar2d", 2, (7, 9), (0.05, 0.0), (1.0, 2 * math.pi), ("bounceback", "periodic"),
                 ("fixed", "periodic"))
    assert _compare(geom, _polar_paper) < 1e-13


def test_bessel_horn_matches_printed_metric():
    # the paper's trumpet: lambda = 0.2, r in [2, 150], Zmax = 750 (lattice units)
    geom = _geom("bessel_horn", 3, (5, 4, 7), (2.0, 0.0, 0.0), (150.0, 2 * math.pi, 700.0),
                 ("free", "periodic", "bounceback"), ("bounceback", "periodic", "free"), ref_axis=2,
                 params=(0.2, 750.0))
    assert _compare(geom, _bessel_horn_paper(0.2, 750.0)) < 1e-12
    # the printed Gamma^th_zth enters the contracted Gamma^theta only through
    # g^{z theta} = 0, so the typo does not reach the scheme: the uncorrected
    # table gives the same coefficients.
    assert _compare(geom, _bessel_horn_paper(0.2, 750.0, fix_typo=False)) < 1e-12


def test_torus_matches_printed_metric_with_sign_fix():
    # the paper's torus: R = 640, 5.12 < r < 409.6
    geom = _geom("torus", 3, (5, 6, 7), (5.12, 0.0, 0.0), (409.6, 2 * math.pi, 2 * math.pi),
                 ("free", "periodic", "periodic"), ("bounceback", "periodic", "periodic"), params=(640.0,))
    assert _compare(geom, _torus_paper(640.0)) < 1e-12
    # the printed sign of Gamma^r_thth would change the radial force
    assert _compare(geom, _torus_paper(640.0, fix_typo=False)) > 1e-3


def _fd_identity_error(geom):
    """max over interior nodes of |Gamh^i + (1/sqrtg) sum_j D_j(sqrtg Ghat^ij)|
    with D_j the central difference over one lattice link."""
    o = oracle.Oracle(geom)
    d = geom["dim"]
    shape = o.shape[::-1]  # array order: slowest first
    pairs = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (0, 1): 3, (1, 0): 3, (0, 2): 4, (2, 0): 4, (1, 2): 5, (2, 1): 5}
    sg = o.sqrtg.reshape(shape)
    err = 0.0
    for i in range(d):
        div = np.zeros(shape)
        for j in range(d):
            Ghat = o.Mhat[pairs[(i, j)]].reshape(shape) + (1.0 if i == j else 0.0)
            F = sg * Ghat
            ax = d - 1 - j
            if geom["bc_lo"][j] == "periodic":
                div += 0.5 * (np.roll(F, -1, axis=ax) - np.roll(F, 1, axis=ax))
            else:
                D = np.full(shape, np.nan)
                sl_c = [slice(None)] * d
                sl_p = [slice(None)] * d
                sl_m = [slice(None)] * d
                sl_c[ax] = slice(1, -1)
                sl_p[ax] = slice(2, None)
                sl_m[ax] = slice(0, -2)
                D[tuple(sl_c)] = 0.5 * (F[tuple(sl_p)] - F[tuple(sl_m)])
                div += D
        resid = o.Gamh[i].reshape(shape) + div / sg
        scale = max(1e-3, np.nanmax(np.abs(o.Gamh[i])))
        err = max(err, np.nanmax(np.abs(resid)) / scale)
    return err


@pytest.mark.parametrize("kind", ["horn", "torus", "cylinder"])
def test_christoffel_identity_second_order(kind):
    if kind == "horn":
        mk = lambda n: W.trumpet_horn(c=0.2, n=n)
        e1 = _fd_identity_error(mk((48, 8, 64)))
        e2 = _fd_identity_error(mk((96, 8, 128)))
    elif kind == "torus":
        mk = lambda n: dict(W.torus(c=0.1), n=n)
        e1 = _fd_identity_error(mk((12, 16, 16)))
        e2 = _fd_identity_error(mk((24, 16, 32)))
    else:
        mk = lambda n: dict(W.closed_cylinder(c=0.1), n=n)
        e1 = _fd_identity_error(mk((12, 8, 8)))
        e2 = _fd_identity_error(mk((24, 8, 8)))
    # cylinder: the fields are linear in r, so the differences are exact
    assert e1 < 0.1 and (e2 < e1 / 2.5 or e2 < 1e-12), (e1, e2)


def test_configured_wave_speeds_are_stable():
    """Every configured c is at most 0.9 of the frozen-coefficient bound
    c_max = 2 / sqrt(max_x sum_d B_d) with B_d = 4 for m_d <= 1 and
    (1 + m_d)^2 / m_d otherwise (m_d = Mhat^dd, plus |Mhat^02| on axes 0, 2):
    the largest c for which the per-node leapfrog-type amplification stays on
    the unit circle (see test_oracle_scheme for the dispersion relation)."""
    for idx in range(4):
        geom = W.GEOMETRIES[idx]()
        o = oracle.Oracle(geom)
        tot = np.zeros(o.N)
        for a in range(o.dim):
            m = o.Mhat[a] + (np.abs(o.Mhat[4]) if o.dim == 3 and a in (0, 2) else 0.0)
            tot += np.where(m <= 1.0, 4.0, (1.0 + m) ** 2 / np.maximum(m, 1e-300))
        cmax = 2.0 / math.sqrt(tot.max())
        assert geom["c"] <= 0.9 * cmax + 1e-12, (idx, geom["c"], cmax)
        assert geom["c"] > 0.89 * cmax
