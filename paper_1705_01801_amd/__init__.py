"""Python binding of liblbw: the curvilinear wave lattice-Boltzmann step of
Velasco, Munoz and Mendoza (arXiv 1705.01801) on MI355X.

Argument marshalling only: every step of the method runs in the HIP library
(``liblbw.so``, built by ``paper_1705_01801_amd.build``).  PyTorch provides
device memory and the stream.  Importing works without a GPU; creating a
geometry needs the built library and a device, and fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbw.so")

KINDS = {"box": 0, "polar2d": 1, "cylinder": 2, "horn": 3, "torus": 4, "bessel_horn": 5, "general": 6}
BCS = {"periodic": 0, "bounceback": 1, "free": 2, "fixed": 3}
EQUILIBRIA = {"corrected": 0, "hermite": 1}
EXPORT_TABLE_F64, EXPORT_MASK_U8, EXPORT_PULL_I32 = 0, 1, 2
TABLE_PLANES = ("Mhat00", "Mhat11", "Mhat22", "Mhat02", "Gamh0", "Gamh1", "Gamh2", "sqrtg")

# every symbol include/lbw.h declares
SYMBOLS = ("lbw_make_geometry", "lbw_make_geometry_general", "lbw_free_geometry", "lbw_geometry_export", "lbw_stability_bound",
           "lbw_set_step_config", "lbw_get_step_config", "lbw_set_step2_config", "lbw_get_step2_config", "lbw_init",
           "lbw_step_n", "lbw_autotune", "lbw_set_graph_block", "lbw_probe", "lbw_modes", "lbw_modes_noalloc",
           "lbw_state_info",
           "lbw_pressure", "lbw_free_state", "lbw_set_sources", "lbw_amplitude", "lbw_batch_make", "lbw_batch_layout", "lbw_batch_set_step_config",
           "lbw_batch_get_step_config", "lbw_batch_autotune", "lbw_batch_set_graph_block", "lbw_batch_step_n",
           "lbw_batch_info", "lbw_batch_probe", "lbw_batch_modes", "lbw_batch_set_sources",
           "lbw_batch_amplitude", "lbw_batch_free", "lbw_mlp_create",
           "lbw_mlp_param_count", "lbw_mlp_set_params", "lbw_mlp_get_params", "lbw_mlp_forward", "lbw_mlp_loss_grad",
           "lbw_mlp_adam_step", "lbw_mlp_train", "lbw_mlp_free", "lbw_last_error")


class GeometryDesc(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("dim", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("bc_lo", ctypes.c_int32 * 3),
        ("bc_hi", ctypes.c_int32 * 3),
        ("equilibrium", ctypes.c_int32),
        ("qmin", ctypes.c_double * 3),
        ("qmax", ctypes.c_double * 3),
        ("h_ref", ctypes.c_double),
        ("c", ctypes.c_double),
        ("damping", ctypes.c_double),
        ("params", ctypes.c_double * 4),
    ]


class LbwError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("lbw error %d: %s" % (code, msg))
        self.code = code


_lib = None


def _hip_runtimes():
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    paths.add(line.split()[-1])
    except OSError:
        pass
    return paths


def lib():
    """The loaded HIP library; raises if it has not been built.

    torch is imported first so that the library's libamdhip64.so.7
    dependency resolves to the HIP runtime torch already loaded: streams and
    device pointers handed over by torch are only valid in that runtime."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblbw.so is not built (run paper_1705_01801_amd/build.py); "
                               "there is no fallback path")
        import torch  # noqa: F401  (loads torch's HIP runtime)
        L = ctypes.CDLL(LIB_PATH)
        runtimes = _hip_runtimes()
        if len(runtimes) > 1:
            raise RuntimeError("two HIP runtimes loaded in one process: %s" % sorted(runtimes))
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        L.lbw_make_geometry.argtypes = [ctypes.POINTER(GeometryDesc), vp, ctypes.POINTER(vp)]
        L.lbw_free_geometry.argtypes = [vp]
        L.lbw_geometry_export.argtypes = [vp, i32, vp, ctypes.c_size_t]
        L.lbw_stability_bound.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
        ip = ctypes.POINTER(ctypes.c_int)
        L.lbw_make_geometry_general.argtypes = [ctypes.POINTER(GeometryDesc), vp, vp, ctypes.POINTER(vp)]
        L.lbw_set_step_config.argtypes = [vp, i32, i32, i32, i32]
        L.lbw_get_step_config.argtypes = [vp, ip, ip, ip, ip]
        L.lbw_set_step2_config.argtypes = [vp, i32, i32, i32, i32]
        L.lbw_get_step2_config.argtypes = [vp, ip, ip, ip, ip]
        L.lbw_init.argtypes = [vp, vp, vp, vp, ctypes.POINTER(i64), i32, vp, i64, vp, ctypes.POINTER(vp)]
        L.lbw_step_n.argtypes = [vp, i64]
        L.lbw_autotune.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double)]
        L.lbw_set_graph_block.argtypes = [vp, i32]
        L.lbw_probe.argtypes = [vp, vp, i64, i64]
        L.lbw_modes.argtypes = [vp, i32, vp, vp]
        L.lbw_modes_noalloc.argtypes = [vp, i32, vp, vp]
        L.lbw_state_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(vp)]
        L.lbw_pressure.argtypes = [vp, vp]
        L.lbw_free_state.argtypes = [vp]
        L.lbw_set_sources.argtypes = [vp, ctypes.POINTER(i64), i32, ctypes.c_double, ctypes.c_double, i32]
        L.lbw_amplitude.argtypes = [vp, i64, i64, vp]
        L.lbw_batch_make.argtypes = [ctypes.POINTER(GeometryDesc), i32, vp, vp, vp, ctypes.POINTER(i64),
                                     ctypes.POINTER(ctypes.c_int32), vp, i64, vp, ctypes.POINTER(vp)]
        L.lbw_batch_layout.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.lbw_batch_set_step_config.argtypes = [vp, i32, i32, i32]
        L.lbw_batch_get_step_config.argtypes = [vp, ip, ip, ip]
        L.lbw_batch_autotune.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double)]
        L.lbw_batch_set_graph_block.argtypes = [vp, i32]
        L.lbw_batch_step_n.argtypes = [vp, i64]
        L.lbw_batch_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(vp)]
        L.lbw_batch_probe.argtypes = [vp, vp, i64, i64]
        L.lbw_batch_modes.argtypes = [vp, i32, vp, vp]
        L.lbw_batch_free.argtypes = [vp]
        L.lbw_batch_set_sources.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_int32), i32]
        L.lbw_batch_amplitude.argtypes = [vp, i64, i64, vp]
        L.lbw_mlp_create.argtypes = [ctypes.POINTER(ctypes.c_int32), i32, i32, vp, ctypes.POINTER(vp)]
        L.lbw_mlp_param_count.argtypes = [vp, ctypes.POINTER(i64)]
        L.lbw_mlp_set_params.argtypes = [vp, vp]
        L.lbw_mlp_get_params.argtypes = [vp, vp]
        L.lbw_mlp_forward.argtypes = [vp, vp, i32, vp]
        L.lbw_mlp_loss_grad.argtypes = [vp, vp, vp, vp, i32, ctypes.c_float, vp, vp]
        L.lbw_mlp_adam_step.argtypes = [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float]
        L.lbw_mlp_train.argtypes = [vp, vp, vp, vp, i32, ctypes.c_float, i32, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_float, ctypes.c_float, ctypes.c_float, vp]
        L.lbw_mlp_free.argtypes = [vp]
        L.lbw_last_error.restype = ctypes.c_char_p
        for name in SYMBOLS:
            getattr(L, name).restype = ctypes.c_int if name != "lbw_last_error" else ctypes.c_char_p
        _lib = L
    return _lib


def check(rc: int):
    if rc != 0:
        raise LbwError(rc, lib().lbw_last_error().decode())


def to_desc(geom: dict) -> GeometryDesc:
    """Geometry description (plain dict, see ``workloads``) -> C struct."""
    d = GeometryDesc()
    d.kind = KINDS[geom["kind"]]
    d.dim = int(geom["dim"])
    dim = d.dim
    for a in range(3):
        if a < dim:
            d.n[a] = int(geom["n"][a])
            d.qmin[a] = float(geom["qmin"][a])
            d.qmax[a] = float(geom["qmax"][a])
            d.bc_lo[a] = BCS[geom["bc_lo"][a]]
            d.bc_hi[a] = BCS[geom["bc_hi"][a]]
        else:
            d.n[a], d.qmin[a], d.qmax[a] = 1, 0.0, 1.0
    eq = geom.get("equilibrium", "corrected")
    if eq not in EQUILIBRIA:
        raise ValueError("equilibrium must be one of %s" % sorted(EQUILIBRIA))
    d.equilibrium = EQUILIBRIA[eq]
    d.h_ref = float(geom["h_ref"])
    d.c = float(geom["c"])
    d.damping = float(geom.get("damp", 1.0))
    par = list(geom.get("params", ())) + [0.0] * 4
    for i in range(4):
        d.params[i] = float(par[i])
    return d


def _stream_ptr(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Geometry:
    """Device coefficient tables of one coordinate system and grid."""

    def __init__(self, geom: dict, stream=None):
        self.geom = dict(geom)
        self.dim = int(geom["dim"])
        self.Q = 2 * self.dim + 1
        self.shape = tuple(int(v) for v in geom["n"][: self.dim])
        self.N = int(np.prod(self.shape))
        self.general = geom["kind"] == "general"
        self.E = self.N if self.general else self.shape[0] * (self.shape[2] if self.dim == 3 else 1)
        self._desc = to_desc(geom)
        self._stream = stream
        h = ctypes.c_void_p()
        if self.general:
            # a geometry given by its metric: 10 planes of N doubles (sqrt(g),
            # G^{ij} 00 11 22 01 02 12, Gamma^i 0 1 2)
            metric = np.ascontiguousarray(geom["coeffs"], dtype=np.float64).reshape(10, self.N)
            check(lib().lbw_make_geometry_general(ctypes.byref(self._desc), metric.ctypes.data, _stream_ptr(stream),
                                                  ctypes.byref(h)))
        else:
            check(lib().lbw_make_geometry(ctypes.byref(self._desc), _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h

    def table(self) -> np.ndarray:
        out = np.zeros((10 if self.general else 8, self.E))
        check(lib().lbw_geometry_export(self.handle, EXPORT_TABLE_F64, out.ctypes.data, out.nbytes))
        return out

    def maps(self):
        mask = np.zeros(self.N, np.uint8)
        pull = np.zeros((self.Q, self.N), np.int32)
        check(lib().lbw_geometry_export(self.handle, EXPORT_MASK_U8, mask.ctypes.data, mask.nbytes))
        check(lib().lbw_geometry_export(self.handle, EXPORT_PULL_I32, pull.ctypes.data, pull.nbytes))
        return mask, pull

    def stability_bound(self) -> float:
        v = ctypes.c_double()
        check(lib().lbw_stability_bound(self.handle, ctypes.byref(v)))
        return v.value

    def set_step_config(self, tile_x: int, tile_y: int, chunk_z: int, blocks: int = 0):
        check(lib().lbw_set_step_config(self.handle, int(tile_x), int(tile_y), int(chunk_z), int(blocks)))

    def step_config(self):
        """(tile_x, tile_y, chunk_z, blocks) of the 3-D step kernel."""
        v = [ctypes.c_int() for _ in range(4)]
        check(lib().lbw_get_step_config(self.handle, *(ctypes.byref(x) for x in v)))
        return tuple(x.value for x in v)

    def set_step2_config(self, tile_x: int, tile_y: int = 0, chunk_z: int = 16, blocks: int = 0):
        """Two time steps per launch with this shape (tile_x 96 with tile_y
        6, or 128 with 4); tile_x = 0 turns it off."""
        check(lib().lbw_set_step2_config(self.handle, int(tile_x), int(tile_y), int(chunk_z), int(blocks)))

    def step2_config(self):
        """(tile_x, tile_y, chunk_z, blocks) of the two-step launches, zeros when off."""
        v = [ctypes.c_int() for _ in range(4)]
        check(lib().lbw_get_step2_config(self.handle, *(ctypes.byref(x) for x in v)))
        return tuple(x.value for x in v)

    def close(self):
        if getattr(self, "handle", None):
            lib().lbw_free_geometry(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Simulation:
    """A wave field on a geometry: caller-owned populations (two float32
    buffers, Q x N), an FP64 probe trace, and the step/probe/modes calls."""

    def __init__(self, geometry: Geometry, P0, probes=(), t_max: int = 0, stream=None):
        import torch
        self.geometry = geometry
        dev = torch.device("cuda", torch.cuda.current_device())
        P0 = torch.as_tensor(P0, dtype=torch.float64).reshape(-1).to(dev).contiguous()
        if P0.numel() != geometry.N:
            raise ValueError("P0 has %d values, geometry has %d nodes" % (P0.numel(), geometry.N))
        self._P0 = P0
        self.f = [torch.empty((geometry.Q, geometry.N), dtype=torch.float32, device=dev) for _ in range(2)]
        probes = np.ascontiguousarray(np.asarray(probes, dtype=np.int64).reshape(-1))
        self.n_probes = int(probes.size)
        self.t_max = int(t_max) if self.n_probes else 0
        self.trace = torch.zeros((max(self.t_max, 1), max(self.n_probes, 1)), dtype=torch.float64, device=dev)
        self._stream = stream
        h = ctypes.c_void_p()
        pp = probes.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if self.n_probes else None
        check(lib().lbw_init(geometry.handle, P0.data_ptr(), self.f[0].data_ptr(), self.f[1].data_ptr(), pp,
                             self.n_probes, self.trace.data_ptr() if self.n_probes else None, self.t_max,
                             _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h

    def step(self, n: int = 1):
        check(lib().lbw_step_n(self.handle, int(n)))

    def autotune(self, reps: int = 20) -> float:
        """Times the step kernel's launch shapes on this state (unchanged by
        the timing) and keeps the fastest; returns microseconds per step."""
        us = ctypes.c_double()
        check(lib().lbw_autotune(self.handle, int(reps), ctypes.byref(us)))
        return us.value

    def set_graph_block(self, steps: int):
        check(lib().lbw_set_graph_block(self.handle, int(steps)))

    @property
    def t(self) -> int:
        t = ctypes.c_int64()
        check(lib().lbw_state_info(self.handle, ctypes.byref(t), None))
        return t.value

    def populations(self):
        """The torch tensor (Q x N, float32) holding the current state."""
        p = ctypes.c_void_p()
        check(lib().lbw_state_info(self.handle, None, ctypes.byref(p)))
        return self.f[0] if p.value == self.f[0].data_ptr() else self.f[1]

    def probe(self, t0: int = 0, t1: int | None = None) -> np.ndarray:
        rows = min(self.t, self.t_max)
        t1 = rows if t1 is None else t1
        out = np.zeros((max(t1 - t0, 0), self.n_probes))
        if out.size == 0:
            return out
        check(lib().lbw_probe(self.handle, out.ctypes.data, int(t0), int(t1)))
        return out

    def modes(self, k: int):
        freq = np.zeros(k)
        power = np.zeros(k)
        check(lib().lbw_modes(self.handle, int(k), freq.ctypes.data, power.ctypes.data))
        return freq, power

    def modes_noalloc(self, k: int, freq, power):
        """lbw_modes into caller-owned device tensors (k float64 each) through
        the library's fixed work space; queued, not waited for."""
        check(lib().lbw_modes_noalloc(self.handle, int(k), freq.data_ptr(), power.data_ptr()))

    def set_sources(self, nodes, amplitude: float, omega: float, flux_axis=None):
        """Drives the pressure amplitude * sin(omega t) at the given nodes
        from the next step on (an empty list removes the sources); with
        flux_axis = a, the flux J'_a = amplitude * sin(omega t) instead (the
        oscillating plate)."""
        nodes = np.ascontiguousarray(np.asarray(nodes, dtype=np.int64).reshape(-1))
        kind = 0 if flux_axis is None else 1 + int(flux_axis)
        check(lib().lbw_set_sources(self.handle, nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    int(nodes.size), float(amplitude), float(omega), kind))

    def amplitude(self, t0: int, t1: int) -> np.ndarray:
        """Largest |P| of each probe over recorded rows [t0, t1)."""
        out = np.zeros(self.n_probes)
        check(lib().lbw_amplitude(self.handle, int(t0), int(t1), out.ctypes.data))
        return out

    def pressure(self):
        import torch
        out = torch.empty(self.geometry.N, dtype=torch.float64, device=self.f[0].device)
        check(lib().lbw_pressure(self.handle, out.data_ptr()))
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib().lbw_free_state(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many D3Q7 geometries advanced by one launch per step.

    geoms: list of geometry descriptions; P0s: list of initial pressure
    arrays; probes: list of per-geometry node-index lists; t_max: trace rows.
    Populations live in two caller-side float32 tensors of 7 * sum(N)
    values; geometry h's block starts at 7 * node_offsets[h]."""

    def __init__(self, geoms, P0s, probes, t_max: int, stream=None):
        import torch
        n = len(geoms)
        assert n == len(P0s) == len(probes) and n > 0
        self.geoms = [dict(g) for g in geoms]
        self.n = n
        descs = (GeometryDesc * n)(*[to_desc(g) for g in geoms])
        dev = torch.device("cuda", torch.cuda.current_device())
        sizes = [int(np.prod(g["n"][:3])) for g in geoms]
        self.node_offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        total = int(self.node_offsets[-1])
        p0 = torch.cat([torch.as_tensor(np.asarray(p, dtype=np.float64).reshape(-1)) for p in P0s]).to(dev)
        if p0.numel() != total:
            raise ValueError("P0 sizes do not match the grids")
        self._P0 = p0
        self.f = [torch.empty(7 * total, dtype=torch.float32, device=dev) for _ in range(2)]
        counts = np.array([len(p) for p in probes], dtype=np.int32)
        flat = np.ascontiguousarray(np.concatenate([np.asarray(p, dtype=np.int64).reshape(-1) for p in probes])
                                    if counts.sum() else np.zeros(0, np.int64))
        self.probe_offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
        self.P = int(counts.sum())
        self.t_max = int(t_max) if self.P else 0
        self.trace = torch.zeros((max(self.t_max, 1), max(self.P, 1)), dtype=torch.float64, device=dev)
        h = ctypes.c_void_p()
        check(lib().lbw_batch_make(descs, n, p0.data_ptr(), self.f[0].data_ptr(), self.f[1].data_ptr(),
                                   flat.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if self.P else None,
                                   counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   self.trace.data_ptr() if self.P else None, self.t_max, _stream_ptr(stream),
                                   ctypes.byref(h)))
        self.handle = h

    def step(self, n: int = 1):
        check(lib().lbw_batch_step_n(self.handle, int(n)))

    def set_step_config(self, tile_x: int, chunk_z: int, blocks: int = 0):
        check(lib().lbw_batch_set_step_config(self.handle, int(tile_x), int(chunk_z), int(blocks)))

    def step_config(self):
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(lib().lbw_batch_get_step_config(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def autotune(self, reps: int = 10) -> float:
        """Times the batch's launch shapes on scratch buffers (state, step
        count and trace unchanged) and keeps the fastest; returns
        microseconds per step."""
        us = ctypes.c_double()
        check(lib().lbw_batch_autotune(self.handle, int(reps), ctypes.byref(us)))
        return us.value

    def set_graph_block(self, steps: int):
        check(lib().lbw_batch_set_graph_block(self.handle, int(steps)))

    @property
    def t(self) -> int:
        t = ctypes.c_int64()
        check(lib().lbw_batch_info(self.handle, ctypes.byref(t), None))
        return t.value

    def populations(self, h: int):
        """Current populations of geometry h as a (7, N_h) view."""
        p = ctypes.c_void_p()
        check(lib().lbw_batch_info(self.handle, None, ctypes.byref(p)))
        f = self.f[0] if p.value == self.f[0].data_ptr() else self.f[1]
        a, b = int(self.node_offsets[h]), int(self.node_offsets[h + 1])
        return f[7 * a: 7 * b].view(7, b - a)

    def probe(self, t0: int = 0, t1: int | None = None) -> np.ndarray:
        rows = min(self.t, self.t_max)
        t1 = rows if t1 is None else t1
        out = np.zeros((max(t1 - t0, 0), self.P))
        if out.size == 0:
            return out
        check(lib().lbw_batch_probe(self.handle, out.ctypes.data, int(t0), int(t1)))
        return out

    def set_sources(self, nodes, geom, amplitude, omega, flux_axis=None):
        """Source i drives amplitude[i] * sin(omega[i] t) at node nodes[i]
        of geometry geom[i] (scalars broadcast); empty lists remove them.
        The drive is a pressure, or with flux_axis[i] = a >= 0 the flux
        J'_a (a negative entry keeps that source a pressure)."""
        nodes = np.ascontiguousarray(np.asarray(nodes, dtype=np.int64).reshape(-1))
        n = nodes.size
        geom = np.ascontiguousarray(np.broadcast_to(np.asarray(geom, dtype=np.int32), (n,)))
        amp = np.ascontiguousarray(np.broadcast_to(np.asarray(amplitude, dtype=np.float64), (n,)))
        om = np.ascontiguousarray(np.broadcast_to(np.asarray(omega, dtype=np.float64), (n,)))
        kp = None
        if flux_axis is not None:
            ax = np.broadcast_to(np.asarray(flux_axis, dtype=np.int64), (n,))
            kind = np.ascontiguousarray(np.where(ax < 0, 0, ax + 1).astype(np.int32))
            kp = kind.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        check(lib().lbw_batch_set_sources(self.handle, nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                          geom.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                          amp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          om.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), kp, int(n)))

    def amplitude(self, t0: int, t1: int) -> np.ndarray:
        """Largest |P| of every probe (global order) over rows [t0, t1)."""
        out = np.zeros(self.P)
        check(lib().lbw_batch_amplitude(self.handle, int(t0), int(t1), out.ctypes.data))
        return out

    def modes(self, k: int):
        freq = np.zeros((self.n, k))
        power = np.zeros((self.n, k))
        check(lib().lbw_batch_modes(self.handle, int(k), freq.ctypes.data, power.ctypes.data))
        return freq, power

    def close(self):
        if getattr(self, "handle", None):
            lib().lbw_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MLP:
    """Surrogate network on the device (BF16 weights/activations, FP32
    accumulation and master weights, Adam)."""

    def __init__(self, widths, max_batch: int, stream=None):
        import torch
        self.widths = [int(v) for v in widths]
        arr = (ctypes.c_int32 * len(self.widths))(*self.widths)
        h = ctypes.c_void_p()
        check(lib().lbw_mlp_create(arr, len(self.widths) - 1, int(max_batch), _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h
        n = ctypes.c_int64()
        check(lib().lbw_mlp_param_count(self.handle, ctypes.byref(n)))
        self.n_params = n.value
        self.max_batch = int(max_batch)
        self._dev = torch.device("cuda", torch.cuda.current_device())

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
        assert p.size == self.n_params
        check(lib().lbw_mlp_set_params(self.handle, p.ctypes.data))

    def get_params(self) -> np.ndarray:
        p = np.zeros(self.n_params, dtype=np.float32)
        check(lib().lbw_mlp_get_params(self.handle, p.ctypes.data))
        return p

    def forward(self, x):
        import torch
        x = torch.as_tensor(x, dtype=torch.float32, device=self._dev).contiguous()
        B = x.shape[0]
        y = torch.empty((B, self.widths[-1]), dtype=torch.float32, device=self._dev)
        for s in range(0, B, self.max_batch):
            e = min(B, s + self.max_batch)
            check(lib().lbw_mlp_forward(self.handle, x[s:e].data_ptr(), e - s, y[s:e].data_ptr()))
        return y

    def loss_grad(self, x, t, w=None, want_grad=False, weight_sum=None):
        import torch
        x = torch.as_tensor(x, dtype=torch.float32, device=self._dev).contiguous()
        t = torch.as_tensor(t, dtype=torch.float32, device=self._dev).contiguous()
        w = None if w is None else torch.as_tensor(w, dtype=torch.float32, device=self._dev).contiguous()
        if weight_sum is None:
            weight_sum = t.numel() if w is None else w.sum().item()
        wsum = float(weight_sum)
        loss = torch.zeros(1, dtype=torch.float32, device=self._dev)
        grad = torch.zeros(self.n_params, dtype=torch.float32, device=self._dev) if want_grad else None
        check(lib().lbw_mlp_loss_grad(self.handle, x.data_ptr(), t.data_ptr(), None if w is None else w.data_ptr(),
                                      x.shape[0], wsum, loss.data_ptr(), None if grad is None else grad.data_ptr()))
        return loss, grad

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        check(lib().lbw_mlp_adam_step(self.handle, float(lr), float(beta1), float(beta2), float(eps)))

    def train(self, x, t, w=None, steps=1000, lr=1e-3, lr_floor=1e-5, weight_sum=None, beta1=0.9, beta2=0.999,
              eps=1e-8) -> float:
        """steps graph-replayed training steps with the cosine learning rate
        lr (1 + cos(pi s / steps)) / 2 + lr_floor; returns the last loss."""
        import torch
        B = int(x.shape[0])
        if weight_sum is None:
            weight_sum = float(w.sum().item()) if w is not None else float(t.numel())
        loss = torch.zeros(1, dtype=torch.float32, device=x.device)
        check(lib().lbw_mlp_train(self.handle, x.data_ptr(), t.data_ptr(), None if w is None else w.data_ptr(), B,
                                  float(weight_sum), int(steps), float(lr), float(lr_floor), float(beta1),
                                  float(beta2), float(eps), loss.data_ptr()))
        return float(loss.item())

    def close(self):
        if getattr(self, "handle", None):
            lib().lbw_mlp_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
