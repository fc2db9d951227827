"""ctypes binding of libcountpairs (include/countpairs.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Point sets are torch tensors on the GPU (their data pointers are
handed to the library as device pointers); edges and outputs are host numpy
arrays.  The library must be built (python -m paper_1911_08275_amd.build);
importing this module without it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcountpairs.so")

CP_F64, CP_F32 = 0, 1
CP_PREC_FP64, CP_PREC_FP32_RECHECK = 0, 1
CP_ORDERED, CP_UNIQUE = 0, 1
CP_OK = 0
ERR_NAMES = {-1: "CP_ERR_INVALID_ARG", -2: "CP_ERR_OUT_OF_BOX", -3: "CP_ERR_NONFINITE",
             -4: "CP_ERR_NOMEM", -5: "CP_ERR_DEVICE", -6: "CP_ERR_INTERNAL"}

EXPORTS = [
    "cp_default_options", "countpairs_xi", "countpairs_wp", "countpairs_cross",
    "countpairs_cross_wp", "countpairs_xi_noalloc", "countpairs_workspace_size",
    "countpairs_strerror",
    "countpairs_last_error", "countpairs_last_stats", "cp_plan_create", "cp_plan_execute",
    "cp_plan_results", "cp_plan_stats", "cp_plan_destroy", "cp_rr_periodic_xi",
    "cp_rr_periodic_wp", "cp_xi_natural", "cp_wp_integrate",
]


class cp_points(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("z", ctypes.c_void_p), ("w", ctypes.c_void_p), ("dtype", ctypes.c_int)]


class cp_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("periodic", ctypes.c_int),
                ("boxsize", ctypes.c_double), ("refine", ctypes.c_int * 3),
                ("need_ravg", ctypes.c_int), ("count_mode", ctypes.c_int),
                ("stream", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t), ("no_prune", ctypes.c_int)]


class cp_stats(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_uint64), ("rechecks", ctypes.c_uint64),
                ("cell_pairs", ctypes.c_uint64), ("cell_pairs_pruned", ctypes.c_uint64),
                ("tiles", ctypes.c_uint64), ("grid", ctypes.c_int * 3),
                ("refine", ctypes.c_int * 3), ("ms_grid", ctypes.c_float),
                ("ms_pairs", ctypes.c_float), ("ms_total", ctypes.c_float),
                ("precision", ctypes.c_int), ("tuned", ctypes.c_int),
                ("chunk_pct", ctypes.c_int), ("waves", ctypes.c_int)]

    def todict(self) -> dict:
        return dict(candidates=int(self.candidates), rechecks=int(self.rechecks),
                    cell_pairs=int(self.cell_pairs), cell_pairs_pruned=int(self.cell_pairs_pruned),
                    tiles=int(self.tiles), grid=list(self.grid), refine=list(self.refine),
                    ms_grid=float(self.ms_grid), ms_pairs=float(self.ms_pairs),
                    ms_total=float(self.ms_total),
                    precision={CP_PREC_FP64: "fp64",
                               CP_PREC_FP32_RECHECK: "fp32"}.get(int(self.precision), "?"),
                    tuned={0: "given", 1: "tuned", 2: "cached", 3: "default"}.get(int(self.tuned), "?"),
                    chunk_pct=int(self.chunk_pct), waves=int(self.waves))


class CountpairsError(RuntimeError):
    def __init__(self, code: int, detail: str):
        super().__init__(f"{ERR_NAMES.get(code, code)}: {detail}")
        self.code = code
        self.detail = detail


_lib = None


def lib() -> ctypes.CDLL:
    """Load libcountpairs.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run python -m paper_1911_08275_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P, D, U = ctypes.POINTER, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint64)
        pp, po = P(cp_points), P(cp_options)
        L.cp_default_options.argtypes = [po]
        L.cp_default_options.restype = None
        L.countpairs_xi.argtypes = [pp, D, ctypes.c_int, po, U, D, D]
        L.countpairs_wp.argtypes = [pp, D, ctypes.c_int, ctypes.c_double, ctypes.c_int, po, U, D, D]
        L.countpairs_xi_noalloc.argtypes = [pp, D, ctypes.c_int, po, U, D, D]
        L.countpairs_cross.argtypes = [pp, pp, D, ctypes.c_int, po, U, D, D]
        L.countpairs_cross_wp.argtypes = [pp, pp, D, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                          po, U, D, D]
        for f in ("countpairs_xi", "countpairs_wp", "countpairs_cross", "countpairs_cross_wp",
                  "countpairs_xi_noalloc"):
            getattr(L, f).restype = ctypes.c_int
        L.countpairs_workspace_size.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, D,
                                                ctypes.c_int, ctypes.c_double, ctypes.c_int, po]
        L.countpairs_workspace_size.restype = ctypes.c_size_t
        L.countpairs_strerror.argtypes = [ctypes.c_int]
        L.countpairs_strerror.restype = ctypes.c_char_p
        L.countpairs_last_error.argtypes = []
        L.countpairs_last_error.restype = ctypes.c_char_p
        L.countpairs_last_stats.argtypes = [P(cp_stats)]
        L.countpairs_last_stats.restype = ctypes.c_int
        L.cp_plan_create.argtypes = [pp, ctypes.c_int, D, ctypes.c_int, D, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_int, po, P(ctypes.c_void_p)]
        L.cp_plan_create.restype = ctypes.c_int
        L.cp_plan_execute.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.cp_plan_execute.restype = ctypes.c_int
        L.cp_plan_results.argtypes = [ctypes.c_void_p, U, U]
        L.cp_plan_results.restype = ctypes.c_int
        L.cp_plan_stats.argtypes = [ctypes.c_void_p, P(cp_stats), P(cp_stats)]
        L.cp_plan_stats.restype = ctypes.c_int
        L.cp_plan_destroy.argtypes = [ctypes.c_void_p]
        L.cp_plan_destroy.restype = ctypes.c_int
        L.cp_rr_periodic_xi.argtypes = [ctypes.c_int64, ctypes.c_double, D, ctypes.c_int,
                                        ctypes.c_int, D]
        L.cp_rr_periodic_wp.argtypes = [ctypes.c_int64, ctypes.c_double, D, ctypes.c_int,
                                        ctypes.c_double, ctypes.c_int, ctypes.c_int, D]
        L.cp_xi_natural.argtypes = [U, ctypes.c_double, D, ctypes.c_double, ctypes.c_int, D]
        L.cp_wp_integrate.argtypes = [D, ctypes.c_int, ctypes.c_int, ctypes.c_double, D]
        for f in ("cp_rr_periodic_xi", "cp_rr_periodic_wp", "cp_xi_natural", "cp_wp_integrate"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != CP_OK:
        raise CountpairsError(rc, lib().countpairs_last_error().decode(errors="replace"))


@dataclass
class DevicePoints:
    """A point set resident on the GPU (torch tensors kept alive here)."""
    x: object
    y: object
    z: object
    w: object = None

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def struct(self) -> cp_points:
        """The C-ABI view of the point set, validated once per set of tensors
        (re-validated whenever a tensor, its storage or its length changes)."""
        key = (self.x.data_ptr(), self.y.data_ptr(), self.z.data_ptr(),
               None if self.w is None else self.w.data_ptr(),
               self.x.shape, self.y.shape, self.z.shape,
               None if self.w is None else self.w.shape, self.x.dtype)
        c = self.__dict__.get("_struct")
        if c is not None and c[0] == key:
            return c[1]
        import torch
        dt = self.x.dtype
        if dt == torch.float64:
            code = CP_F64
        elif dt == torch.float32:
            code = CP_F32
        else:
            raise TypeError("coordinates must be float32 or float64")
        for t in (self.x, self.y, self.z):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous() or t.dim() != 1:
                raise ValueError("x, y, z must be contiguous 1-D GPU tensors of one dtype")
            if t.shape[0] != self.x.shape[0]:
                raise ValueError("x, y, z lengths differ")
        w = 0
        if self.w is not None:
            if self.w.dtype != torch.float64 or not self.w.is_cuda or not self.w.is_contiguous():
                raise ValueError("w must be a contiguous float64 GPU tensor")
            if self.w.dim() != 1 or self.w.shape[0] != self.x.shape[0]:
                raise ValueError("w must be 1-D with one weight per point")
            w = self.w.data_ptr()
        st = cp_points(self.n, self.x.data_ptr(), self.y.data_ptr(), self.z.data_ptr(), w, code)
        self.__dict__["_struct"] = (key, st)
        return st


def to_device(cat, device="cuda", weights: bool = True) -> DevicePoints:
    """Copy a synth.Catalog (numpy) to the GPU, keeping its dtype."""
    import torch
    t = [torch.from_numpy(np.ascontiguousarray(v)).to(device) for v in (cat.x, cat.y, cat.z)]
    w = None
    if weights and getattr(cat, "w", None) is not None:
        w = torch.from_numpy(np.ascontiguousarray(cat.w, dtype=np.float64)).to(device)
    return DevicePoints(t[0], t[1], t[2], w)


_DEFAULT_OPTIONS = None
_PREC = None
_MODES = None


def _current_stream() -> int:
    """torch's current HIP stream of the current device (0: the null stream)."""
    import torch
    try:
        return int(torch._C._cuda_getCurrentRawStream(torch.cuda.current_device()))
    except Exception:
        try:
            return int(torch.cuda.current_stream().cuda_stream)
        except Exception:
            return 0


def options(precision: str = "fp32", periodic: bool = False, boxsize: float = 0.0,
            refine: Optional[Sequence[int]] = None, need_ravg: bool = False,
            count_mode: str = "ordered", stream=None, workspace=None,
            no_prune: bool = False) -> cp_options:
    global _DEFAULT_OPTIONS, _PREC, _MODES
    if _DEFAULT_OPTIONS is None:
        d = cp_options()
        lib().cp_default_options(ctypes.byref(d))
        _DEFAULT_OPTIONS = bytes(d)
        _PREC = {"fp32": CP_PREC_FP32_RECHECK, "fp64": CP_PREC_FP64}
        _MODES = {"ordered": CP_ORDERED, "unique": CP_UNIQUE}
    o = cp_options.from_buffer_copy(_DEFAULT_OPTIONS)
    o.precision = _PREC[precision]
    o.periodic = 1 if periodic else 0
    o.boxsize = float(boxsize)
    if refine is not None and refine != "auto":
        # None or "auto": refine 0, the library tunes the launch settings
        o.refine[0], o.refine[1], o.refine[2] = int(refine[0]), int(refine[1]), int(refine[2])
    o.need_ravg = 1 if need_ravg else 0
    o.count_mode = _MODES[count_mode]
    o.no_prune = 1 if no_prune else 0
    if workspace is not None:
        # a caller-owned device buffer (e.g. a torch uint8 tensor)
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    o.stream = int(getattr(stream, "cuda_stream", stream)) if stream is not None else _current_stream()
    return o


@dataclass
class Counts:
    npairs: np.ndarray
    wsum: Optional[np.ndarray]
    ravg: Optional[np.ndarray]
    stats: dict


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _up(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def last_stats() -> dict:
    s = cp_stats()
    _check(lib().countpairs_last_stats(ctypes.byref(s)))
    return s.todict()


def _outputs(nout, need):
    n = np.zeros(nout, dtype=np.uint64)
    ws = np.zeros(nout, dtype=np.float64) if need else None
    ra = np.zeros(nout, dtype=np.float64) if need else None
    return n, ws, ra


def countpairs_xi(d: DevicePoints, edges, **opt) -> Counts:
    e = np.ascontiguousarray(edges, dtype=np.float64)
    o = options(**opt)
    n, ws, ra = _outputs(e.size - 1, o.need_ravg)
    pts = d.struct()
    _check(lib().countpairs_xi(ctypes.byref(pts), _dp(e), e.size, ctypes.byref(o), _up(n),
                               _dp(ws) if ws is not None else None,
                               _dp(ra) if ra is not None else None))
    return Counts(n, ws, ra, last_stats())


def countpairs_xi_noalloc(d: DevicePoints, edges, **opt) -> Counts:
    """countpairs_xi on the library's static device scratch (no allocation)."""
    e = np.ascontiguousarray(edges, dtype=np.float64)
    o = options(**opt)
    n, ws, ra = _outputs(e.size - 1, o.need_ravg)
    pts = d.struct()
    _check(lib().countpairs_xi_noalloc(ctypes.byref(pts), _dp(e), e.size, ctypes.byref(o),
                                       _up(n), _dp(ws) if ws is not None else None,
                                       _dp(ra) if ra is not None else None))
    return Counts(n, ws, ra, last_stats())


def countpairs_wp(d: DevicePoints, rp_edges, pimax: float, npibins: int, **opt) -> Counts:
    e = np.ascontiguousarray(rp_edges, dtype=np.float64)
    o = options(**opt)
    n, ws, ra = _outputs((e.size - 1) * npibins, o.need_ravg)
    pts = d.struct()
    _check(lib().countpairs_wp(ctypes.byref(pts), _dp(e), e.size, float(pimax), int(npibins),
                               ctypes.byref(o), _up(n), _dp(ws) if ws is not None else None,
                               _dp(ra) if ra is not None else None))
    shp = (e.size - 1, npibins)
    return Counts(n.reshape(shp), None if ws is None else ws.reshape(shp),
                  None if ra is None else ra.reshape(shp), last_stats())


def countpairs_cross(d1: DevicePoints, d2: DevicePoints, edges, **opt) -> Counts:
    e = np.ascontiguousarray(edges, dtype=np.float64)
    o = options(**opt)
    n, ws, ra = _outputs(e.size - 1, o.need_ravg)
    p1, p2 = d1.struct(), d2.struct()
    _check(lib().countpairs_cross(ctypes.byref(p1), ctypes.byref(p2), _dp(e), e.size,
                                  ctypes.byref(o), _up(n), _dp(ws) if ws is not None else None,
                                  _dp(ra) if ra is not None else None))
    return Counts(n, ws, ra, last_stats())


def countpairs_cross_wp(d1: DevicePoints, d2: DevicePoints, rp_edges, pimax: float,
                        npibins: int, **opt) -> Counts:
    e = np.ascontiguousarray(rp_edges, dtype=np.float64)
    o = options(**opt)
    n, ws, ra = _outputs((e.size - 1) * npibins, o.need_ravg)
    p1, p2 = d1.struct(), d2.struct()
    _check(lib().countpairs_cross_wp(ctypes.byref(p1), ctypes.byref(p2), _dp(e), e.size,
                                     float(pimax), int(npibins), ctypes.byref(o), _up(n),
                                     _dp(ws) if ws is not None else None,
                                     _dp(ra) if ra is not None else None))
    shp = (e.size - 1, npibins)
    return Counts(n.reshape(shp), None if ws is None else ws.reshape(shp),
                  None if ra is None else ra.reshape(shp), last_stats())


class Plan:
    """Batched plan over many catalogues (cp_plan_* in the C ABI)."""

    def __init__(self, mocks: Sequence[DevicePoints], xi_edges=None, wp_edges=None,
                 pimax: float = 0.0, npibins: int = 1, **opt):
        self.mocks = list(mocks)
        self._pts = (cp_points * len(self.mocks))(*[m.struct() for m in self.mocks])
        self.xi_edges = None if xi_edges is None else np.ascontiguousarray(xi_edges, np.float64)
        self.wp_edges = None if wp_edges is None else np.ascontiguousarray(wp_edges, np.float64)
        self.npibins = int(npibins)
        self._opt = options(**opt)
        h = ctypes.c_void_p()
        _check(lib().cp_plan_create(
            self._pts, len(self.mocks),
            _dp(self.xi_edges) if self.xi_edges is not None else None,
            0 if self.xi_edges is None else self.xi_edges.size,
            _dp(self.wp_edges) if self.wp_edges is not None else None,
            0 if self.wp_edges is None else self.wp_edges.size,
            float(pimax), self.npibins, ctypes.byref(self._opt), ctypes.byref(h)))
        self.handle = h

    def execute(self, stream=None):
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        _check(lib().cp_plan_execute(self.handle, ctypes.c_void_p(int(stream))))

    def results(self):
        nm = len(self.mocks)
        xi = wp = None
        if self.xi_edges is not None:
            xi = np.zeros((nm, self.xi_edges.size - 1), dtype=np.uint64)
        if self.wp_edges is not None:
            wp = np.zeros((nm, self.wp_edges.size - 1, self.npibins), dtype=np.uint64)
        _check(lib().cp_plan_results(self.handle, _up(xi) if xi is not None else None,
                                     _up(wp) if wp is not None else None))
        return xi, wp

    def stats(self):
        a, b = cp_stats(), cp_stats()
        _check(lib().cp_plan_stats(self.handle, ctypes.byref(a), ctypes.byref(b)))
        return a.todict(), b.todict()

    def close(self):
        if getattr(self, "handle", None):
            lib().cp_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_size(kind: str, n1: int, n2: int, edges, pimax: float = 0.0, npibins: int = 1,
                   **opt) -> int:
    """Bytes of device scratch a call needs at most (countpairs_workspace_size)."""
    e = np.ascontiguousarray(edges, dtype=np.float64)
    o = options(**opt)
    k = {"xi": 0, "wp": 1, "cross": 2, "cross_wp": 3}[kind]
    return int(lib().countpairs_workspace_size(k, int(n1), int(n2), _dp(e), e.size, float(pimax),
                                                int(npibins), ctypes.byref(o)))


# ------------------------------------------------------------- estimators
# Host functions of the library (Section 1): analytic random pairs of a
# periodic cube, the natural estimator and the w_p line-of-sight sum.

def _mode(count_mode: str) -> int:
    return {"ordered": CP_ORDERED, "unique": CP_UNIQUE}[count_mode]


def cp_rr_periodic_xi(n: int, boxsize: float, edges, count_mode: str = "ordered") -> np.ndarray:
    e = np.ascontiguousarray(edges, dtype=np.float64)
    rr = np.zeros(max(1, e.size - 1), dtype=np.float64)
    _check(lib().cp_rr_periodic_xi(int(n), float(boxsize), _dp(e), e.size, _mode(count_mode),
                                   _dp(rr)))
    return rr


def cp_rr_periodic_wp(n: int, boxsize: float, rp_edges, pimax: float, npibins: int,
                      count_mode: str = "ordered") -> np.ndarray:
    e = np.ascontiguousarray(rp_edges, dtype=np.float64)
    rr = np.zeros((max(1, e.size - 1), max(1, int(npibins))), dtype=np.float64)
    _check(lib().cp_rr_periodic_wp(int(n), float(boxsize), _dp(e), e.size, float(pimax),
                                   int(npibins), _mode(count_mode), _dp(rr)))
    return rr


def cp_xi_natural(dd, rr, dd_norm: float = 1.0, rr_norm: float = 1.0) -> np.ndarray:
    d = np.ascontiguousarray(dd, dtype=np.uint64).ravel()
    r = np.ascontiguousarray(rr, dtype=np.float64).ravel()
    if d.size != r.size:
        raise ValueError("dd and rr differ in size")
    xi = np.zeros(d.size, dtype=np.float64)
    _check(lib().cp_xi_natural(_up(d), float(dd_norm), _dp(r), float(rr_norm), d.size, _dp(xi)))
    return xi.reshape(np.shape(dd))


def cp_wp_integrate(xi2d, pimax: float) -> np.ndarray:
    x = np.ascontiguousarray(xi2d, dtype=np.float64)
    if x.ndim != 2:
        raise ValueError("xi2d must be (rp bins, pi bins)")
    wp = np.zeros(x.shape[0], dtype=np.float64)
    _check(lib().cp_wp_integrate(_dp(x), x.shape[0], x.shape[1], float(pimax), _dp(wp)))
    return wp
