"""Host logic of the frequency sweeps (CPU only): the peak finder and the
closed-form resonances the pipe sweep is compared with.

* peaks: on a sampled sum of Lorentzian lines the parabola through the three
  samples around each local maximum lands within a tenth of the sample
  spacing of the true centre, and lines below 2 % of the largest are
  ignored;
* radial_wavenumbers: every returned zeta > 0 is a root of the annulus
  cross-product J_1(zeta a) Y_1(zeta b) - J_1(zeta b) Y_1(zeta a), the list
  is increasing, and as a -> 0 the roots tend to the zeros of J_1(zeta b)
  (the full disk with a reflecting wall), taken from scipy's jn_zeros;
* resonances: c sqrt(zeta^2 + k_z^2) with the closed-open and closed-closed
  axial series, every value below wmax and the plane-wave members
  (zeta = 0) equal to (2n + 1) pi c / (2L) and n pi c / L.
"""
import math

import numpy as np
from scipy.special import j1, jn_zeros, y1

from paper_1705_01801_amd import sweep_study as S


def test_peaks_refine_lorentzian_centres():
    om = np.linspace(0.0, 0.03, 121)
    centres, widths, heights = [0.0043, 0.0121, 0.0188, 0.0257], [4e-4, 6e-4, 5e-4, 7e-4], [1.0, 0.6, 0.3, 0.01]
    amp = sum(h / (1.0 + ((om - c) / w) ** 2) for c, w, h in zip(centres, widths, heights))
    found = S.peaks(om, amp)
    assert len(found) == 3                                  # the 1 % line is ignored
    spacing = om[1] - om[0]
    for c, f in zip(centres[:3], found):
        assert abs(f - c) <= 0.1 * spacing, (c, f)


def test_annulus_radial_wavenumbers():
    a, b = 1.0, 25.0
    roots = S.radial_wavenumbers(a, b, 1.0)
    assert roots[0] == 0.0 and np.all(np.diff(roots) > 0) and len(roots) >= 5
    for z in roots[1:]:
        v = j1(z * a) * y1(z * b) - j1(z * b) * y1(z * a)
        scale = abs(j1(z * a) * y1(z * b)) + abs(j1(z * b) * y1(z * a))
        assert abs(v) <= 1e-9 * scale
    small = S.radial_wavenumbers(1e-3, b, 0.6)[1:]
    disk = jn_zeros(1, len(small)) / b
    assert np.allclose(small, disk, rtol=1e-3)


def test_resonance_series():
    c, L, a, b = 0.1, 100.0, 1.0, 25.0
    wmax = 0.03
    for closed_open in (True, False):
        res = S.resonances(c, L, a, b, wmax, closed_open)
        assert all(0 < w <= wmax for w in res) and res == sorted(res)
        plane = [(2 * n + 1) * math.pi * c / (2 * L) if closed_open else n * math.pi * c / L for n in range(0, 20)]
        plane = [w for w in plane if 0 < w <= wmax]
        for w in plane:
            assert min(abs(r - w) for r in res) <= 1e-15


def test_sweep_source_and_probe_nodes():
    """Node lists of the sweeps land where their docstrings say (CPU)."""
    import workloads as W
    pipe = W.driven_pipe("fixed")
    n0, n1, n2 = pipe["n"]
    ring, plate, probes = W.pipe_ring(pipe), W.pipe_plate(pipe), W.pipe_probes(pipe)
    assert np.array_equal(ring % n0, np.zeros(n1)) and np.all(ring // (n0 * n1) == 0)   # r_min, z = 0
    assert np.array_equal(np.sort(plate), np.arange(n0 * n1))                         # the whole z = 0 plane
    assert np.array_equal(probes // (n0 * n1), [10, 50]) and np.all(probes % n0 == 1)
    tor = W.driven_torus()
    t0, t1, t2 = tor["n"]
    src = W.torus_sources(tor)
    assert src["inner"].size == t1 * t2 and np.all(src["inner"] % t0 == 0)
    small = src["small_ring"]
    assert small.size == t2 and np.all(small % (t0 * t1) == 0)                        # rho_min, theta = 0
    tp = W.torus_probes(tor)
    assert tp[0] % t0 == t0 - 1 and (tp[0] // t0) % t1 == t1 // 2 and tp[0] // (t0 * t1) == 0
    w = W.torus_omegas()
    assert w.size == 499 and abs(w[1] - w[0] - 0.001) < 1e-12
    geom, pt, om = W.point_source_box()
    assert pt == [50 + 100 * 50] and abs(om - 2 * math.pi * 0.5 / 10) < 1e-15
