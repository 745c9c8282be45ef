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


def test_summaries_from_other_sources_are_ignored(tmp_path):
    """A summary whose recorded source hash, workload or flags differ from the current ones is not read."""
    for name, reader in (("sweep_tvs2000_traffic.md", bench.read_traffic),
                         ("tvs2000_counters.md", bench.read_counters)):
        text = open(os.path.join(bench.ROOT, "profiles", name)).read()
        assert reader(os.path.join(bench.ROOT, "profiles", name), "tvs2000", 0) is not None
        digest = bench.kernel_source_digest()
        other = tmp_path / name
        other.write_text(text.replace(digest, "0" * len(digest)))
        assert reader(str(other), "tvs2000", 0) is None
        assert reader(os.path.join(bench.ROOT, "profiles", name), "tvs8000", 0) is None
        assert reader(os.path.join(bench.ROOT, "profiles", name), "tvs2000", 64) is None
