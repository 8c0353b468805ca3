"""C-ABI checks that need no GPU: the library loads, exports every symbol
declared in include/lbw.h, and rejects invalid descriptors on the host
before touching the device."""
import ctypes
import os
import re

import pytest

import paper_1705_01801_amd as lbw
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "lbw.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbw_[a-z_0-9]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(lbw.SYMBOLS)


def test_library_exports_every_declared_symbol():
    L = lbw.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_desc_struct_layout():
    # int32 x 12 (kind, dim, n[3], bc_lo[3], bc_hi[3], reserved) then 13 doubles
    assert ctypes.sizeof(lbw.GeometryDesc) == 12 * 4 + 13 * 8
    assert lbw.GeometryDesc.h_ref.offset == 48 + 48


def _rc(geom):
    d = lbw.to_desc(geom)
    h = ctypes.c_void_p()
    rc = lbw.lib().lbw_make_geometry(ctypes.byref(d), None, ctypes.byref(h))
    return rc, lbw.lib().lbw_last_error().decode(), h


@pytest.mark.parametrize("mutate,msg", [
    (lambda g: g.update(c=0.0), "c must be"),
    (lambda g: g.update(c=float("nan")), "c must be"),
    (lambda g: g.update(h_ref=-1.0), "h_ref"),
    (lambda g: g.update(damp=1.5), "damping"),
    (lambda g: g.update(n=(0, 8, 8)), "n[0]"),
    (lambda g: g.update(qmin=(0.0, 0.0, 0.0)), "radius"),
    (lambda g: g.update(bc_lo=("bounceback", "periodic", "periodic")), "paired"),
    (lambda g: g.update(dim=2), "dim 3"),
    (lambda g: g.update(n=(4096, 4096, 4096)), "too many nodes"),
])
def test_invalid_descriptor_rejected_on_host(mutate, msg):
    g = W.closed_cylinder(scale=8)
    mutate(g)
    rc, err, h = _rc(g)
    assert rc == -1 and msg in err and not h.value


def test_torus_and_horn_ranges_checked():
    g = W.torus(scale=8)
    g["params"] = (0.5,)
    rc, err, _ = _rc(g)
    assert rc == -1 and "R > rho_max" in err
    g = W.trumpet_horn(scale=8)
    g["params"] = (-1.0, 0.01, 1.0)
    rc, err, _ = _rc(g)
    assert rc == -1 and "horn radius" in err


def test_null_arguments():
    L = lbw.lib()
    assert L.lbw_make_geometry(None, None, None) == -1
    assert L.lbw_step_n(None, 1) == -1
    assert L.lbw_free_state(None) == 0 and L.lbw_free_geometry(None) == 0


def _general_rc(geom, metric):
    d = lbw.to_desc(geom)
    h = ctypes.c_void_p()
    ptr = None if metric is None else metric.ctypes.data
    rc = lbw.lib().lbw_make_geometry_general(ctypes.byref(d), ptr, None, ctypes.byref(h))
    return rc, lbw.lib().lbw_last_error().decode(), h


def test_general_metric_rejected_on_host():
    import numpy as np
    geom = W.general_duct(n=(6, 5, 4))
    metric = W.general_coefficients(geom)
    rc, err, h = _rc(geom)                                  # built-in entry point refuses the kind
    assert rc == -1 and "lbw_make_geometry_general" in err and not h.value
    rc, err, h = _general_rc(dict(geom, kind="box"), metric)
    assert rc == -1 and "LBW_GENERAL" in err and not h.value
    rc, err, h = _general_rc(geom, None)
    assert rc == -1 and "metric is NULL" in err
    bad = metric.copy()
    bad[3, 17] = np.inf
    rc, err, h = _general_rc(geom, bad)
    assert rc == -1 and "non-finite" in err and not h.value
    bad = metric.copy()
    bad[0, 9] = -1.0
    rc, err, h = _general_rc(geom, bad)
    assert rc == -1 and "sqrt(g)" in err and not h.value
    # 36 N bytes of coefficients must stay below 2^31 (rejected before the
    # metric is read, so a small array stands in)
    rc, err, h = _general_rc(dict(geom, n=(1024, 1024, 60)), metric)
    assert rc == -1 and "per-node coefficients" in err and not h.value


def test_source_calls_reject_null():
    L = lbw.lib()
    L.lbw_set_sources.restype = ctypes.c_int
    assert L.lbw_set_sources(None, None, 0, 1.0, 0.1, 0) == -1
    assert L.lbw_amplitude(None, 0, 1, None) == -1
    assert L.lbw_batch_set_sources(None, None, None, None, None, None, 0) == -1
    assert L.lbw_batch_amplitude(None, 0, 1, None) == -1


def test_hermite_equilibrium_checked_on_host():
    cyl = dict(W.closed_cylinder(scale=16), equilibrium="hermite")
    rc, err, h = _rc(cyl)
    assert rc == -1 and "Cartesian boxes only" in err and not h.value
    box = dict(kind="box", dim=3, n=(4, 4, 4), qmin=(0.0, 0.0, 0.0), qmax=(4.0, 4.0, 4.0),
               bc_lo=("bounceback",) * 3, bc_hi=("bounceback",) * 3, h_ref=1.0, c=0.5, damp=1.0, params=())
    d = lbw.to_desc(box)
    d.equilibrium = 2
    hh = ctypes.c_void_p()
    rc = lbw.lib().lbw_make_geometry(ctypes.byref(d), None, ctypes.byref(hh))
    assert rc == -1 and "unknown equilibrium" in lbw.lib().lbw_last_error().decode() and not hh.value
    with pytest.raises(ValueError):
        lbw.to_desc(dict(box, equilibrium="lattice"))
