"""C-ABI checks that need no GPU: the library loads, exports every function
include/countpairs.h declares, and rejects bad arguments before any device
work."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "countpairs.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(\w+)\s*\(", text, flags=re.M)
    return sorted({n for n in names if n not in ("if", "defined")})


@pytest.fixture(scope="module")
def native():
    from paper_1911_08275_amd import native
    native.lib()
    return native


def test_library_exports_header(native):
    names = _declared_functions()
    assert len(names) >= 14
    missing = [n for n in names if not hasattr(native.lib(), n)]
    assert not missing, missing
    assert sorted(native.EXPORTS) == names


def test_struct_layouts(native):
    # cp_points: int64 n, 4 pointers, int dtype (padded)
    assert ctypes.sizeof(native.cp_points) == 48
    assert native.cp_options.stream.offset == 40
    assert native.cp_options.no_prune.offset == 64
    assert ctypes.sizeof(native.cp_options) == 72


def test_struct_layouts_match_header(native, tmp_path):
    """sizeof and field offsets of the C structs, compiled from the header
    with gcc, equal the ctypes mirrors of the binding."""
    import subprocess
    fields = {"cp_points": ["n", "x", "w", "dtype"],
              "cp_options": ["precision", "boxsize", "refine", "stream", "workspace_bytes",
                             "no_prune"],
              "cp_stats": ["candidates", "tiles", "grid", "refine", "ms_grid", "ms_total",
                           "precision", "tuned", "chunk_pct", "waves"]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "countpairs.h"',
             'int main(void) {']
    for st, fs in fields.items():
        lines.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = dict(l.split() for l in subprocess.check_output([str(exe)]).decode().splitlines())
    for st, fs in fields.items():
        cls = getattr(native, st)
        assert int(out[st]) == ctypes.sizeof(cls), st
        for f in fs:
            assert int(out[f"{st}.{f}"]) == getattr(cls, f).offset, (st, f)


def test_rejects_bad_prune_flag(native):
    o = native.options()
    o.no_prune = 2
    p = native.cp_points(4, 0x1000, 0x2000, 0x3000, 0, native.CP_F64)
    e = np.asarray((0.1, 1.0, 2.0), dtype=np.float64)
    out = np.zeros(2, dtype=np.uint64)
    rc = native.lib().countpairs_xi(ctypes.byref(p), native._dp(e), e.size, ctypes.byref(o),
                                    native._up(out), None, None)
    assert rc == -1   # CP_ERR_INVALID_ARG
    assert "no_prune" in native.lib().countpairs_last_error().decode()


def _call_xi(native, n=4, edges=(0.1, 1.0, 2.0), **kw):
    o = native.options(**kw)
    p = native.cp_points(n, 0x1000, 0x2000, 0x3000, 0, native.CP_F64)
    e = np.asarray(edges, dtype=np.float64)
    out = np.zeros(max(1, e.size - 1), dtype=np.uint64)
    rc = native.lib().countpairs_xi(ctypes.byref(p), native._dp(e), e.size, ctypes.byref(o),
                                    native._up(out), None, None)
    return rc, native.lib().countpairs_last_error().decode()


@pytest.mark.parametrize("edges", [(1.0,), (1.0, 1.0), (2.0, 1.0), (-1.0, 1.0),
                                   (0.0, float("nan")), (0.0, float("inf"))])
def test_rejects_bad_edges(native, edges):
    rc, msg = _call_xi(native, edges=edges)
    assert rc == -1 and msg


def test_rejects_bad_options(native):
    assert _call_xi(native, periodic=True, boxsize=0.0)[0] == -1
    assert _call_xi(native, periodic=True, boxsize=float("nan"))[0] == -1
    assert _call_xi(native, n=-1)[0] == -1
    o = native.options()
    o.precision = 7
    p = native.cp_points(4, 0x1000, 0x2000, 0x3000, 0, native.CP_F64)
    e = np.array([0.1, 1.0])
    out = np.zeros(1, dtype=np.uint64)
    assert native.lib().countpairs_xi(ctypes.byref(p), native._dp(e), 2, ctypes.byref(o),
                                      native._up(out), None, None) == -1
    p.dtype = 5
    o.precision = 0
    assert native.lib().countpairs_xi(ctypes.byref(p), native._dp(e), 2, ctypes.byref(o),
                                      native._up(out), None, None) == -1
    # need_ravg without outputs
    o.need_ravg = 1
    p.dtype = 0
    assert native.lib().countpairs_xi(ctypes.byref(p), native._dp(e), 2, ctypes.byref(o),
                                      native._up(out), None, None) == -1


def test_rejects_bad_wp_args(native):
    o = native.options()
    p = native.cp_points(4, 0x1000, 0x2000, 0x3000, 0, native.CP_F64)
    e = np.array([0.1, 1.0, 2.0])
    out = np.zeros(2 * 3, dtype=np.uint64)
    for pimax, npi in ((0.0, 3), (-1.0, 3), (10.0, 0), (10.0, 100000)):
        rc = native.lib().countpairs_wp(ctypes.byref(p), native._dp(e), 3, pimax, npi,
                                        ctypes.byref(o), native._up(out), None, None)
        assert rc == -1


def test_too_many_bins(native):
    rc, _ = _call_xi(native, edges=np.linspace(0.0, 10.0, 80))
    assert rc == -1


def test_strerror(native):
    for c in range(-6, 1):
        assert native.lib().countpairs_strerror(c)
    assert native.lib().countpairs_strerror(-99) == b"unknown error"


def test_workspace_size_monotone(native):
    e = np.array([0.1, 1.0, 25.0])
    o = native.options()
    f = native.lib().countpairs_workspace_size
    a = f(0, 1000, 0, native._dp(e), 3, 0.0, 1, ctypes.byref(o))
    b = f(0, 100000, 0, native._dp(e), 3, 0.0, 1, ctypes.byref(o))
    c = f(2, 100000, 100000, native._dp(e), 3, 0.0, 1, ctypes.byref(o))
    assert 0 < a < b < c


def test_plan_rejects(native):
    o = native.options(periodic=False)
    p = (native.cp_points * 1)(native.cp_points(4, 0x1000, 0x2000, 0x3000, 0, native.CP_F64))
    e = np.array([0.1, 1.0])
    h = ctypes.c_void_p()
    rc = native.lib().cp_plan_create(p, 1, native._dp(e), 2, None, 0, 0.0, 1, ctypes.byref(o),
                                     ctypes.byref(h))
    assert rc == -1  # plans need a periodic box
    o = native.options(periodic=True, boxsize=10.0)
    rc = native.lib().cp_plan_create(p, 0, native._dp(e), 2, None, 0, 0.0, 1, ctypes.byref(o),
                                     ctypes.byref(h))
    assert rc == -1
    assert native.lib().cp_plan_destroy(None) == 0
