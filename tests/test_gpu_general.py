"""GPU: geometries given by their metric (per-node coefficients).

The general step kernel against the FP64 oracle on the non-separable duct
(every metric component non-zero and varying along all axes), the general
path fed a built-in geometry's own metric against that geometry's z-marching
kernel, conservation in the closed duct, sources on per-node sqrt(g), and
the calls a general geometry rejects.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_1705_01801_amd as lbw
import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def duct(n=(12, 10, 16), periodic1=False):
    geom = W.general_duct(n=n)
    if periodic1:  # axis 1 periodic (the lattice problem is valid for any metric)
        geom["bc_lo"] = ("bounceback", "periodic", "bounceback")
        geom["bc_hi"] = ("bounceback", "periodic", "fixed")
    return dict(geom, coeffs=W.general_coefficients(geom))


# tile widths 32 and 64, several axis-0 tiles and partial axis-1 tiles,
# a periodic axis (ring nodes wrap), a fixed wall, chunks of 1 to 32 planes
@pytest.mark.parametrize("n,periodic1,shape", [((12, 10, 16), False, None), ((33, 7, 20), False, None),
                                               ((70, 9, 12), False, (64, 4, 5)), ((20, 12, 17), True, None),
                                               ((40, 11, 9), False, (32, 8, 1)), ((40, 11, 9), True, (64, 4, 32)),
                                               ((70, 19, 12), False, (64, 8, 8))])
def test_general_duct_matches_oracle(n, periodic1, shape):
    geom = duct(n, periodic1)
    N = W.num_nodes(geom)
    say("general duct", n, "periodic axis 1" if periodic1 else "", shape)
    o = oracle.Oracle(geom)
    g = lbw.Geometry(geom)
    if shape:
        g.set_step_config(*shape)
        assert g.step_config()[:3] == shape
    t = g.table()
    assert np.abs(t[0:6] - o.Mhat).max() <= 1e-13 * max(1.0, np.abs(o.Mhat).max())
    assert np.abs(t[6:9] - o.Gamh).max() <= 1e-13 * max(1.0, np.abs(o.Gamh).max())
    assert np.array_equal(t[9], o.sqrtg)
    rng = np.random.default_rng(11)
    P0 = rng.uniform(-1, 1, N)
    probes = rng.integers(0, N, size=5)
    T = 210                                            # graph blocks of 32 plus single launches
    sim = lbw.Simulation(g, P0, probes, t_max=T)
    sim.step(T)
    f = o.init(P0)
    _, tr = o.run(f, T, probes)
    assert rel_l2(sim.populations().double().cpu().numpy(), f) <= 1e-5
    assert np.abs(sim.probe() - tr).max() <= 1e-5 * np.abs(tr).max()


def test_general_path_reproduces_builtin_horn():
    geom = W.trumpet_horn(c=0.3, a=0.08, b=0.01, k=2.0, n=(24, 20, 36))
    g = lbw.Geometry(geom)
    tab = g.table()                                    # per (i0, i2) entry
    n0, n1, n2 = geom["n"]
    h = [(geom["qmax"][a] - geom["qmin"][a]) / geom["n"][a] for a in range(3)]
    href = geom["h_ref"]
    node = np.arange(n0 * n1 * n2)
    e = node % n0 + n0 * (node // (n0 * n1))
    metric = np.zeros((10, node.size))
    metric[0] = tab[7][e]
    for m, (i, j, plane) in enumerate([(0, 0, 0), (1, 1, 1), (2, 2, 2)]):
        metric[1 + m] = (tab[plane][e] + 1.0) * h[i] * h[j] / href ** 2
    metric[5] = tab[3][e] * h[0] * h[2] / href ** 2    # G^02; G^01 = G^12 = 0
    for a in range(3):
        metric[7 + a] = tab[4 + a][e] * h[a] / href ** 2
    gg = lbw.Geometry(dict(geom, kind="general", coeffs=metric))
    rng = np.random.default_rng(4)
    P0 = rng.uniform(-1, 1, node.size)
    a = lbw.Simulation(g, P0, [5, 700], t_max=150)
    b = lbw.Simulation(gg, P0, [5, 700], t_max=150)
    a.step(150)
    b.step(150)
    fa = a.populations().double().cpu().numpy()
    assert rel_l2(b.populations().double().cpu().numpy(), fa) <= 1e-5
    assert np.abs(a.probe() - b.probe()).max() <= 1e-5 * np.abs(a.probe()).max()


def test_general_closed_duct_conserves():
    geom = duct()
    rng = np.random.default_rng(2)
    sim = lbw.Simulation(lbw.Geometry(geom), rng.uniform(0, 1, W.num_nodes(geom)))
    I0 = float(sim.populations().double().sum())
    sim.step(1000)
    I1 = float(sim.populations().double().sum())
    assert abs(I1 - I0) <= 1e-4 * abs(I0)


def test_general_sources_use_per_node_sqrtg():
    geom = duct()
    n0, n1 = geom["n"][0], geom["n"][1]
    src = [3 + n0 * (4 + n1 * 7), 8 + n0 * (2 + n1 * 11)]
    sim = lbw.Simulation(lbw.Geometry(geom), np.zeros(W.num_nodes(geom)), src, t_max=80)
    sim.set_sources(src, 0.9, 0.07)
    sim.step(80)
    assert np.abs(sim.probe() - 0.9 * np.sin(0.07 * np.arange(80))[:, None]).max() <= 2e-6
    o = oracle.Oracle(geom)
    f = o.init(np.zeros(o.N))
    o.run(f, 80, [], sources=src, amplitude=0.9, omega=0.07)
    assert rel_l2(sim.populations().double().cpu().numpy(), f) <= 1e-5


def test_general_rejections():
    geom = duct()
    N = W.num_nodes(geom)
    with pytest.raises(lbw.LbwError):                  # built-in entry point
        lbw.check(lbw.lib().lbw_make_geometry(lbw.ctypes.byref(lbw.to_desc(geom)), None,
                                             lbw.ctypes.byref(lbw.ctypes.c_void_p())))
    bad = np.array(geom["coeffs"])
    bad[0, 5] = 0.0
    with pytest.raises(lbw.LbwError):
        lbw.Geometry(dict(geom, coeffs=bad))
    bad = np.array(geom["coeffs"])
    bad[4, 7] = np.nan
    with pytest.raises(lbw.LbwError):
        lbw.Geometry(dict(geom, coeffs=bad))
    g = lbw.Geometry(geom)
    with pytest.raises(lbw.LbwError):
        g.set_step_config(16, 16, 16)
    with pytest.raises(lbw.LbwError):
        g.set_step_config(32, 8, 16, 64)
    sim = lbw.Simulation(g, np.zeros(N))
    with pytest.raises(lbw.LbwError):
        sim.autotune(reps=2)
    with pytest.raises(lbw.LbwError):
        lbw.Batch([geom], [np.zeros(N)], [[0]], t_max=4)


def test_general_full_size_one_step():
    """The 128^3 duct in the benchmark's launch configuration (the default
    64 x 8 tiles, 16 planes per chunk): after 10 GPU steps, one oracle step
    on the GPU state must match the GPU's next step."""
    w = W.general_workload()
    geom, P0 = w["geom"], w["P0"]
    say("general full size one step", geom["n"])
    g = lbw.Geometry(geom)
    assert g.step_config()[:3] == (64, 8, 16)
    sim = lbw.Simulation(g, P0, w["probes"], t_max=32)
    sim.step(10)
    f = sim.populations().double().cpu().numpy()
    sim.step(1)
    fg = sim.populations().double().cpu().numpy()
    o = oracle.Oracle(geom)
    o.step(f, 1)
    assert np.abs(fg - f).max() <= 2e-6 * np.abs(f).max()
    assert rel_l2(fg, f) <= 1e-6
