"""The benchmark's own bookkeeping, on the CPU: the algorithmic byte counts
behind the roofline line follow the formulas they state, a run on more than
one GPU is refused with a message, and the committed rocprofv3 summaries
that the bench line cites belong to the library's current sources."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_forward_bytes_follow_the_stated_count():
    # the forward sweep: 24 bytes per combinational input, 18 per
    # combinational cell, 16 per start point and per endpoint
    N, M, D, E, n_start, n_comb, S = 1000, 900, 7, 40, 100, 800, 2500
    P = M + S
    info = (N, P, M, D, E, n_start, n_comb, S)
    counts = {"paths": 10, "path_pins": 200, "pairs": 30, "touched": 50}
    b = bench.algo_bytes(info, counts)
    A = S - E
    PI = n_start - E
    assert b["forward"] == 24 * A + 18 * n_comb + 16 * (E + E + PI)
    assert b["netpass"] == 28 * S + 28 * M
    assert b["backward"] == 28 * S + 16 * M
    assert b["wa"] == 16 * P + 4 * M + 8 * N
    # the design's own additions are reported apart, never in the roofline
    ov = bench.design_overhead(info, 8)
    assert ov["forward"] == n_comb * (8 * 8 + 64 + 4) + 4 * A


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("name", ["kernel_stats_2m_cells.md", "hbm_traffic_2m_cells.md"])
def test_profiles_belong_to_the_current_sources(name):
    text = open(os.path.join(ROOT, "profiles", name)).read()
    assert f"Source digest: {bench.source_digest()}" in text
    # and they carry the command that made them, which runs committed files
    assert "rocprofv3" in text and "bench.py" in text
