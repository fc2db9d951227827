"""Checks on the gfx950 assembly of our own pair kernels (no GPU needed).

- The binary64 separation that decides a bin must follow the reference
  operation sequence without fused multiply-add: the unweighted xi kernels
  (binary64, and binary32 with its binary64 recheck) contain no v_fma_f64.
  (The weighted kernels use FMA on purpose, only for the separation fed to
  the square root of the weighted mean, never for a bin decision.)
- Packed binary32 arithmetic stays off: no v_pk_{fma,mul,add}_f32 anywhere.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1911_08275_amd", "csrc", "pair_kernels.hip")


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not shutil.which("/opt/rocm/bin/hipcc") and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    from paper_1911_08275_amd import build
    out = tmp_path_factory.mktemp("isa") / "pk.s"
    flags = [f for f in build.FLAGS if f not in ("-shared", "-fPIC")]
    cmd = [build.HIPCC] + flags + ["--cuda-device-only", "-S", SRC, "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    return out.read_text()


def _kernel(asm, mangled):
    m = re.search(r"^" + re.escape(mangled) + r":[^\n]*\n(.*?)s_endpgm", asm, flags=re.S | re.M)
    assert m, mangled
    return m.group(1)


@pytest.mark.parametrize("prec", [0, 1])
def test_unweighted_xi_has_no_fma_f64(asm, prec):
    body = _kernel(asm, f"_ZN2cp7k_pairsILi0ELi{prec}ELi0EEEvNS_10PairParamsE")
    assert "v_fma_f64" not in body and "v_fmac_f64" not in body
    # the binary64 reference path is really there (subtract, square, sum)
    assert "v_mul_f64" in body and "v_add_f64" in body


def test_no_packed_fp32(asm):
    assert not re.search(r"v_pk_(fma|mul|add)_f32", asm)


def test_binary32_filter_uses_fma(asm):
    body = _kernel(asm, "_ZN2cp7k_pairsILi0ELi1ELi0EEEvNS_10PairParamsE")
    assert "v_fma_f32" in body or "v_fmac_f32" in body
