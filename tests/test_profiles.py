"""The committed rocprofv3 summaries (CPU): the HBM traffic summary the bench reads must have been taken
on the library's current code, and every summary must give the command that made it."""
import glob
import os

import bench


def test_traffic_summary_matches_current_sources():
    path = os.path.join(bench.ROOT, "profiles", "sweep_tvs2000_traffic.md")
    t = bench.read_traffic(path, "tvs2000", 0)
    assert t is not None, "profiles/sweep_tvs2000_traffic.md was taken on other library sources: re-profile"
    assert 1e9 < t < 1e10  # bytes per sweep launch of the 2000 x 2000 step


def test_summaries_name_their_commands():
    files = sorted(glob.glob(os.path.join(bench.ROOT, "profiles", "*.md")))
    assert files
    for f in files:
        text = open(f).read()
        assert "rocprofv3" in text and "bench.py" in text, f
