"""CPU FP64 oracle for gridded pair counting.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does, and it
shares no code with the HIP library.

`count()` wraps the C oracle (oracle.c) and returns plain numpy results.  See
oracle.c for the definition it implements (the naive loop of Code 1 over the
separations of Section 1.1, optionally enumerated through the chaining mesh of
Section 1.2) and for every reading of the paper it takes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

XI, WP = 0, 1
ERRORS = {0: "ok", -1: "invalid argument", -2: "point outside the periodic box",
          -3: "non-finite input", -4: "out of memory"}


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (binary64, no contraction, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        lib = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_count.argtypes = [
            ctypes.c_int, ctypes.c_int,
            ctypes.c_int64, dp, dp, dp, dp,
            ctypes.c_int64, dp, dp, dp, dp,
            ctypes.c_int, ctypes.c_double,
            dp, ctypes.c_int, ctypes.c_double, ctypes.c_int,
            ctypes.c_int, ctypes.c_int,
            ctypes.POINTER(ctypes.c_uint64), dp, dp]
        lib.oracle_count.restype = ctypes.c_int
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


@dataclass
class Result:
    npairs: np.ndarray          # uint64, shape (nbins,) or (nbins, npibins)
    wsum: np.ndarray            # float64, sum of w_i w_j per bin
    wrsum: np.ndarray           # float64, sum of w_i w_j * separation per bin

    @property
    def ravg(self) -> np.ndarray:
        """Weighted mean separation per bin (0 where the bin is empty)."""
        out = np.zeros_like(self.wsum)
        nz = self.npairs > 0
        out[nz] = self.wrsum[nz] / self.wsum[nz]
        return out


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code}: {ERRORS.get(code, 'unknown')}")
        self.code = code


def _arr(v):
    if v is None:
        return None, None
    a = np.ascontiguousarray(np.asarray(v, dtype=np.float64))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def count(mode: int, x1, y1, z1, w1=None, x2=None, y2=None, z2=None, w2=None, *,
          edges, periodic: bool, box: float = 0.0, pimax: float = 0.0,
          npibins: int = 1, grid: bool = True, nthreads: int = 0) -> Result:
    """Ordered pair counts.  Auto-count when x2 is None (pairs i != j), cross
    otherwise.  Inputs may be float32 or float64 (float32 promotes exactly)."""
    lib = _load()
    auto = x2 is None
    keep = []
    a1 = [_arr(v) for v in (x1, y1, z1, w1)]
    keep += a1
    n1 = int(a1[0][0].shape[0])
    if auto:
        a2 = [(None, None)] * 4
        n2 = 0
    else:
        a2 = [_arr(v) for v in (x2, y2, z2, w2)]
        keep += a2
        n2 = int(a2[0][0].shape[0])
    e, ep = _arr(edges)
    nbins = e.shape[0] - 1
    npi = npibins if mode == WP else 1
    cnt = np.zeros(nbins * npi, dtype=np.uint64)
    ws = np.zeros(nbins * npi, dtype=np.float64)
    wr = np.zeros(nbins * npi, dtype=np.float64)
    rc = lib.oracle_count(
        mode, 1 if auto else 0,
        n1, a1[0][1], a1[1][1], a1[2][1], a1[3][1],
        n2, a2[0][1], a2[1][1], a2[2][1], a2[3][1],
        1 if periodic else 0, float(box),
        ep, int(e.shape[0]), float(pimax), int(npibins),
        1 if grid else 0, int(nthreads),
        cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
        ws.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        wr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    del keep
    if rc != 0:
        raise OracleError(rc)
    shape = (nbins, npi) if mode == WP else (nbins,)
    return Result(cnt.reshape(shape), ws.reshape(shape), wr.reshape(shape))


def xi(cat, edges, periodic=True, box=0.0, other=None, **kw) -> Result:
    """xi(r) counts of a Catalog (auto) or of cat against `other` (cross)."""
    if other is None:
        return count(XI, cat.x, cat.y, cat.z, cat.w, edges=edges, periodic=periodic,
                     box=box, **kw)
    return count(XI, cat.x, cat.y, cat.z, cat.w, other.x, other.y, other.z, other.w,
                 edges=edges, periodic=periodic, box=box, **kw)


def wp(cat, edges, pimax, npibins, periodic=True, box=0.0, other=None, **kw) -> Result:
    """xi(rp, pi) counts (line of sight z)."""
    if other is None:
        return count(WP, cat.x, cat.y, cat.z, cat.w, edges=edges, periodic=periodic,
                     box=box, pimax=pimax, npibins=npibins, **kw)
    return count(WP, cat.x, cat.y, cat.z, cat.w, other.x, other.y, other.z, other.w,
                 edges=edges, periodic=periodic, box=box, pimax=pimax,
                 npibins=npibins, **kw)
