"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU, no
GPU): the library's host side (argument validation, binning tables and the
binary32 error bound, grid geometry, queue-item split, estimators, tuning
cache) built with -Xarch_host -fsanitize=... so no device code is
instrumented, and the oracle built with gcc.  Each driver must run clean:
-fno-sanitize-recover turns any UBSan report into a failure, ASan aborts on
any memory error."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1911_08275_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd, r.stdout[-3000:], r.stderr[-3000:])
    return r


@pytest.mark.slow
def test_host_library_sanitized(tmp_path):
    host = []
    for f in SAN:
        host += ["-Xarch_host", f]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics",
             "-Wno-unused-result"] + host
    objs = []
    srcs = [os.path.join(HERE, "host_checks.hip")] + [
        os.path.join(CSRC, s) for s in ("grid_kernels.hip", "pair_kernels.hip", "estimators.cpp",
                                        "tune_cache.cpp")]
    procs = []
    for s in srcs:
        o = str(tmp_path / (os.path.basename(s) + ".o"))
        objs.append(o)
        procs.append(subprocess.Popen([HIPCC] + flags + ["-c", s, "-o", o],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
    for p, s in zip(procs, srcs):
        out = p.communicate()[0].decode(errors="replace")
        assert p.returncode == 0, (s, out[-3000:])
    exe = str(tmp_path / "host_checks")
    _run([HIPCC, "--offload-arch=gfx950"] + host + objs + ["-o", exe])
    r = _run([exe, str(tmp_path)], env=ENV, timeout=300)
    assert "host checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


def test_oracle_sanitized(tmp_path):
    exe = str(tmp_path / "oracle_checks")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off"] + SAN +
         [os.path.join(HERE, "oracle_checks.c"), "-o", exe, "-lm"])
    r = _run([exe], env=dict(ENV, OMP_NUM_THREADS="2"), timeout=300)
    assert "oracle checks passed" in r.stdout
    assert "runtime error" not in r.stderr
