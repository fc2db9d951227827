"""The benchmark's command-line contract and its committed counter summaries
(no GPU needed)."""
import glob
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


TRAFFIC = sorted(os.path.basename(p) for p in glob.glob(
    os.path.join(ROOT, "profiles", "k_pairs_xi_weighted_1e6_traffic*.md")))


def test_traffic_summary_exists():
    assert TRAFFIC


@pytest.mark.parametrize("name", TRAFFIC)
def test_traffic_summaries_parse(name):
    """Each traffic summary carries the fields bench.py reads: the kernel
    source hash, the refine factors and the per-launch byte counts."""
    text = open(os.path.join(ROOT, "profiles", name)).read()
    vals = {}
    for line in text.splitlines():
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    assert re.fullmatch(r"[0-9a-f]{64}", vals["pair_kernels.hip sha256"])
    assert re.fullmatch(r"\d+,\d+,\d+", vals["refine"])
    assert int(vals["fetch bytes per launch"]) > 0
    assert int(vals["write bytes per launch"]) > 0
    assert "rocprofv3 --pmc FETCH_SIZE" in text and "rocprofv3 --pmc WRITE_SIZE" in text
