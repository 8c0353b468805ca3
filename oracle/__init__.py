"""FP64 CPU oracle for the curvilinear wave lattice-Boltzmann scheme.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  The product library never
calls it, and it shares no code with the HIP path.

The numerical work lives in ``lbw_oracle.c`` (plain C, double precision,
whole-grid passes in the paper's order); this module compiles it with gcc,
loads it with ctypes and converts a geometry description (a plain dict, see
``workloads``) into the C struct.  ``modes`` (in ``oracle.modes``) extracts
resonant frequencies from probe traces with numpy's FFT.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .modes import modes  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbw_oracle.c")
_LIB = os.path.join(_HERE, "liblbw_oracle.so")

KINDS = {"box": 0, "polar2d": 1, "cylinder": 2, "horn": 3, "torus": 4, "bessel_horn": 5, "general": 6}
BCS = {"periodic": 0, "bounceback": 1, "free": 2, "fixed": 3}


class _Geom(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("dim", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("bc_lo", ctypes.c_int32 * 3),
        ("bc_hi", ctypes.c_int32 * 3),
        ("hermite", ctypes.c_int32),
        ("qmin", ctypes.c_double * 3),
        ("qmax", ctypes.c_double * 3),
        ("href", ctypes.c_double),
        ("c", ctypes.c_double),
        ("damp", ctypes.c_double),
        ("par", ctypes.c_double * 4),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, one thread)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def load_library(path: str):
    """Loads a compiled copy of the oracle (the default build, or a copy
    a test compiled from an edited source to plant a mistake) and declares
    its entry points."""
    lib = ctypes.CDLL(path)
    _declare(lib)
    return lib


def _load():
    global _lib
    if _lib is None:
        _lib = load_library(build())
    return _lib


def _declare(lib):
    dp = ctypes.POINTER(ctypes.c_double)
    gp = ctypes.POINTER(_Geom)
    lib.orc_coeffs.argtypes = [gp, dp, dp, dp]
    lib.orc_coeffs_given.argtypes = [gp, dp, dp, dp, dp]
    lib.orc_maps.argtypes = [gp, ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_int32)]
    lib.orc_init.argtypes = [gp, dp, dp, dp]
    lib.orc_step.argtypes = [gp, dp, dp, dp, dp, dp]
    lib.orc_run.argtypes = [gp, dp, dp, dp, dp, dp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                            ctypes.c_int, dp]
    lib.orc_run_driven.argtypes = [gp, dp, dp, dp, dp, dp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                                   ctypes.c_int, dp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                                   ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int]
    lib.orc_invariant.argtypes = [gp, dp]
    lib.orc_invariant.restype = ctypes.c_double
    lib.orc_pressure.argtypes = [gp, dp, dp, dp]


def _ptr(a, ctype=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _to_struct(geom: dict) -> _Geom:
    s = _Geom()
    s.kind = KINDS[geom["kind"]]
    s.dim = int(geom["dim"])
    n = list(geom["n"]) + [1] * (3 - len(geom["n"]))
    qmin = list(geom["qmin"]) + [0.0] * (3 - len(geom["qmin"]))
    qmax = list(geom["qmax"]) + [1.0] * (3 - len(geom["qmax"]))
    lo = list(geom["bc_lo"]) + ["periodic"] * (3 - len(geom["bc_lo"]))
    hi = list(geom["bc_hi"]) + ["periodic"] * (3 - len(geom["bc_hi"]))
    for a in range(3):
        s.n[a] = int(n[a])
        s.qmin[a] = float(qmin[a])
        s.qmax[a] = float(qmax[a])
        s.bc_lo[a] = BCS[lo[a]]
        s.bc_hi[a] = BCS[hi[a]]
    eq = geom.get("equilibrium", "corrected")
    if eq not in ("corrected", "hermite") or (eq == "hermite" and geom["kind"] != "box"):
        raise ValueError("equilibrium must be 'corrected', or 'hermite' on a box")
    s.hermite = 1 if eq == "hermite" else 0
    s.href = float(geom["h_ref"])
    s.c = float(geom["c"])
    s.damp = float(geom.get("damp", 1.0))
    par = list(geom.get("params", ())) + [0.0] * 4
    for i in range(4):
        s.par[i] = float(par[i])
    return s


class Oracle:
    """One geometry: per-node FP64 coefficients plus step/run helpers.

    Arrays follow the layout f[l, n] with n = i0 + n0 * (i1 + n1 * i2).
    """

    def __init__(self, geom: dict, lib=None):
        self.geom = dict(geom)
        self._g = _to_struct(geom)
        self.dim = self._g.dim
        self.Q = 2 * self.dim + 1
        self.shape = tuple(int(self._g.n[a]) for a in range(self.dim))
        self.N = int(np.prod(self.shape))
        self.lib = _load() if lib is None else lib
        self.sqrtg = np.zeros(self.N)
        self.Mhat = np.zeros((6, self.N))
        self.Gamh = np.zeros((3, self.N))
        if geom["kind"] == "general":
            # a geometry given by its metric: per-node sqrt(g), G^{ij}, Gamma^i
            given = np.ascontiguousarray(geom["coeffs"], dtype=np.float64).reshape(10, self.N)
            self.lib.orc_coeffs_given(ctypes.byref(self._g), _ptr(given), _ptr(self.sqrtg), _ptr(self.Mhat),
                                      _ptr(self.Gamh))
        else:
            self.lib.orc_coeffs(ctypes.byref(self._g), _ptr(self.sqrtg), _ptr(self.Mhat), _ptr(self.Gamh))
        self._work = None

    # -- index maps ---------------------------------------------------------
    def maps(self):
        mask = np.zeros(self.N, dtype=np.uint8)
        pull = np.zeros((self.Q, self.N), dtype=np.int32)
        self.lib.orc_maps(ctypes.byref(self._g), _ptr(mask, ctypes.c_uint8), _ptr(pull, ctypes.c_int32))
        return mask, pull

    # -- state --------------------------------------------------------------
    def init(self, P0) -> np.ndarray:
        P0 = np.ascontiguousarray(P0, dtype=np.float64).reshape(-1)
        assert P0.size == self.N
        f = np.zeros((self.Q, self.N))
        self.lib.orc_init(ctypes.byref(self._g), _ptr(self.sqrtg), _ptr(P0), _ptr(f))
        return f

    def _workbuf(self):
        if self._work is None:
            self._work = np.zeros((self.Q + 1) * self.N)
        return self._work

    def step(self, f: np.ndarray, n: int = 1) -> np.ndarray:
        """Advances f (Q x N, float64, C-contiguous) in place by n steps."""
        assert f.dtype == np.float64 and f.flags.c_contiguous and f.shape == (self.Q, self.N)
        return self.run(f, n, [])[0]

    def run(self, f: np.ndarray, nsteps: int, probes, sources=None, amplitude: float = 0.0, omega: float = 0.0,
            t0: int = 0, flux_axis=None):
        """Advances f in place from time t0; returns (f, trace[nsteps, n_probes])
        where trace[s] is the pressure at each probe at time t0 + s, before
        that step.  With sources (node indices) the pressure
        amplitude * sin(omega t) is imposed at those nodes at every time t
        before the probes are read (populations at rest at that pressure);
        with flux_axis = a the flux J'_a = amplitude * sin(omega t) is imposed
        instead (the node keeps its S; the oscillating plate)."""
        assert f.dtype == np.float64 and f.flags.c_contiguous and f.shape == (self.Q, self.N)
        probes = np.ascontiguousarray(probes, dtype=np.int64).reshape(-1)
        src = np.ascontiguousarray([] if sources is None else sources, dtype=np.int64).reshape(-1)
        assert src.size == 0 or (src.min() >= 0 and src.max() < self.N)
        trace = np.zeros((max(int(nsteps), 0), probes.size))
        w = self._workbuf()
        self.lib.orc_run_driven(ctypes.byref(self._g), _ptr(self.Mhat), _ptr(self.Gamh), _ptr(self.sqrtg), _ptr(f),
                                _ptr(w), int(nsteps), _ptr(probes, ctypes.c_int64), int(probes.size), _ptr(trace),
                                int(t0), _ptr(src, ctypes.c_int64), int(src.size), float(amplitude), float(omega),
                                0 if flux_axis is None else 1 + int(flux_axis))
        return f, trace

    @staticmethod
    def amplitude(trace: np.ndarray, t0: int, t1: int) -> np.ndarray:
        """Response intensity of a driven run (Sec. IV.A, the pipe sweeps):
        the largest |P| at each probe over trace rows [t0, t1)."""
        return np.abs(np.asarray(trace)[t0:t1]).max(axis=0)

    def invariant(self, f) -> float:
        return float(self.lib.orc_invariant(ctypes.byref(self._g), _ptr(np.ascontiguousarray(f))))

    def pressure(self, f) -> np.ndarray:
        P = np.zeros(self.N)
        self.lib.orc_pressure(ctypes.byref(self._g), _ptr(np.ascontiguousarray(f)), _ptr(self.sqrtg), _ptr(P))
        return P

    # -- derived quantities used by tests -------------------------------------
    def spacing(self):
        return tuple((self.geom["qmax"][a] - self.geom["qmin"][a]) / self.shape[a] for a in range(self.dim))
