"""Pins for geometries given by their metric (CPU only).

Sec. III: the scheme sees a geometry only through sqrt(g), the inverse metric
and the contracted Christoffel symbols, so any coordinate system can be run
by supplying them per node.  The inputs of the synthetic duct (a stretched,
sheared and bumped embedding, every metric component non-zero and varying
along all three axes) and the oracle's use of them are pinned by:

* the contraction identity Gamma^i = -(1/sqrt(g)) d_j(sqrt(g) G^{ij}),
  checked with central differences of the generated fields, and
  sqrt(g) = det J, G g = I;
* a built-in geometry (a horn) run through the general path with its own
  metric data in physical units gives the built-in run's result;
* the closed duct conserves sum sqrt(g) P (curvilinear continuity equation)
  and stays bounded at its configured wave speed.
"""
import numpy as np
import pytest

import oracle
import workloads as W


def test_duct_inputs_satisfy_christoffel_identity():
    rng = np.random.default_rng(5)
    q = rng.uniform(0.1, 0.9, size=(3, 200))
    v = W.general_at(q)
    sg, G = v[0], np.array([[v[1], v[4], v[5]], [v[4], v[2], v[6]], [v[5], v[6], v[3]]])
    J, _ = W.duct_embedding(q)
    assert np.abs(sg - np.linalg.det(np.moveaxis(J, (0, 1), (-2, -1)))).max() < 1e-13
    g = np.einsum("ai...,aj...->ij...", J, J)
    assert np.abs(np.einsum("ij...,jk...->ik...", G, g) - np.eye(3)[:, :, None]).max() < 1e-12
    for name in ("G01", "G02", "G12"):
        assert np.abs(v[W.GENERAL_PLANES.index(name)]).max() > 1e-3      # non-separable
    d = 1e-5
    div = np.zeros((3, q.shape[1]))
    for j in range(3):
        e = np.zeros((3, 1))
        e[j] = d
        vp, vm = W.general_at(q + e), W.general_at(q - e)
        Gp = np.array([[vp[1], vp[4], vp[5]], [vp[4], vp[2], vp[6]], [vp[5], vp[6], vp[3]]])
        Gm = np.array([[vm[1], vm[4], vm[5]], [vm[4], vm[2], vm[6]], [vm[5], vm[6], vm[3]]])
        div += (vp[0] * Gp[:, j] - vm[0] * Gm[:, j]) / (2 * d)
    assert np.abs(v[7:10] + div / sg).max() < 1e-7


def test_builtin_geometry_through_general_path():
    geom = W.trumpet_horn(c=0.3, a=0.08, b=0.01, k=2.0, n=(10, 8, 14))
    o = oracle.Oracle(geom)
    h = o.spacing()
    href = geom["h_ref"]
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    given = np.zeros((10, o.N))
    given[0] = o.sqrtg
    for m, (i, j) in enumerate(pairs):
        given[1 + m] = (o.Mhat[m] + (1.0 if i == j else 0.0)) * h[i] * h[j] / href ** 2
    for i in range(3):
        given[7 + i] = o.Gamh[i] * h[i] / href ** 2
    og = oracle.Oracle(dict(geom, kind="general", coeffs=given))
    assert np.abs(og.Mhat - o.Mhat).max() < 1e-12 and np.abs(og.Gamh - o.Gamh).max() < 1e-12
    rng = np.random.default_rng(3)
    P0 = rng.uniform(-1, 1, o.N)
    fa, fb = o.init(P0), og.init(P0)
    o.step(fa, 200)
    og.step(fb, 200)
    assert np.abs(fa - fb).max() <= 1e-10 * np.abs(fa).max()


def test_closed_duct_conserves_and_stays_bounded():
    geom = W.general_duct(n=(12, 10, 16))
    o = oracle.Oracle(dict(geom, coeffs=W.general_coefficients(geom)))
    assert np.abs(o.Mhat[3]).max() > 1e-3 and np.abs(o.Mhat[5]).max() > 1e-3   # cross terms 01, 12 in play
    rng = np.random.default_rng(9)
    f = o.init(rng.uniform(-1, 1, o.N))
    I0 = o.invariant(f)
    m0 = np.abs(f).max()
    for _ in range(4):
        o.step(f, 500)
        assert abs(o.invariant(f) - I0) <= 1e-12 * np.abs(f).sum()
    assert np.abs(f).max() < 10 * m0
