"""Batches of independent tiles (tvs_batch_*): the persistent fused relocate + sweep and the
batched back-projection, replayed from a captured graph, against the plain per-tile path and
the oracle (marked `gpu`)."""
import math
import sys

import numpy as np
import pytest

from synth import fractal_dem

pytestmark = pytest.mark.gpu
P_DEFAULT, P_F32 = 65, 33


def note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tvs():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2003_02200_amd as t

    t.lib()
    return t


# (rows, cols, spacing, obs_height, max_dist): uneven sizes, a 1-cell tile, a long strip, an
# unbounded distance and a distance shorter than one cell
TILES = [(40, 53, 10.0, 1.5, 530.0), (1, 1, 5.0, 2.0, 100.0), (97, 12, 10.0, 20.0, math.inf),
         (64, 64, 7.5, 1.5, 480.0), (23, 140, 10.0, 3.0, 1400.0), (130, 77, 10.0, 30.0, 1300.0),
         (16, 16, 10.0, 1.5, 4.0)]


def _make(tiles, seed=0):
    import torch

    dems, host = [], []
    for x, (H, W, dx, h0, R) in enumerate(tiles):
        d = fractal_dem(max(H, W), 100 + seed + x, 0.6, 900.0)[:H, :W].copy()
        host.append(d)
        dems.append(torch.from_numpy(d).cuda())
    return host, dems


def _outs(tiles, fill):
    import torch

    return [torch.full((H, W), fill, dtype=torch.float64, device="cuda") for (H, W, *_r) in tiles]


@pytest.mark.parametrize("flags,prec", [(0, P_DEFAULT), (0x40, P_F32)])
def test_batch_equals_per_tile_and_oracle(tvs, orc, flags, prec):
    import torch

    n = 24
    host, dems = _make(TILES)
    outs_b = _outs(TILES, 7.0)  # stale values: the first chunk must overwrite them
    outs_t = _outs(TILES, -1.0)
    tl_b = [(dems[x], outs_b[x], *TILES[x][2:]) for x in range(len(TILES))]
    tl_t = [(dems[x], outs_t[x], *TILES[x][2:]) for x in range(len(TILES))]
    note(f"batch create flags={flags}")
    b = tvs.Batch(tl_b, n, flags=flags)
    tvs.total_viewshed_tiles(tl_t, n, flags=flags)
    torch.cuda.synchronize()
    want = [o.cpu().numpy() for o in outs_t]
    for x, (H, W, dx, h0, R) in enumerate(TILES):
        np.testing.assert_allclose(want[x], orc.total(host[x], dx, h0, n, R, prec=prec), rtol=1e-12, atol=0)
    # replays of the captured pass, with eager work and synchronisation between them
    for rep in range(3):
        note(f"batch replay {rep} flags={flags}")
        b.run()
        torch.cuda.synchronize()
        for x in range(len(TILES)):
            np.testing.assert_allclose(outs_b[x].cpu().numpy(), want[x], rtol=1e-13, atol=0, err_msg=f"tile {x}")
        for o in outs_b:
            o.fill_(3.0)
        torch.cuda.synchronize()
    inf = b.info()
    # tables and counters, the tiles transposed (n >= 2), per chunk one sweep per bucket of tiles and
    # one back-projection
    assert inf.tiles == len(TILES) and inf.chunks >= 1 and inf.buckets >= 1
    assert inf.kernel_launches == 2 + len(TILES) + inf.chunks * (inf.buckets + 1)
    bks = b.buckets()
    assert sum(bk["tiles"] for bk in bks) == len(TILES)
    nrows = sum(tvs.sector_shape(H, W, n, k)[0] for (H, W, *_r) in TILES for k in range(n))
    assert sum(bk["items"] for bk in bks) == nrows
    assert [bk["side_class"] for bk in bks] == sorted((bk["side_class"] for bk in bks), reverse=True)
    ev = sum(tvs.los_evals(H, W, dx, n, R)[0] for (H, W, dx, h0, R) in TILES)
    assert inf.los_evals == ev
    b.close()


def test_batch_counts_and_chunking(tvs, monkeypatch):
    """A scratch budget small enough to force several chunks; evaluation counts equal the sum of
    the single-tile counts (the same early exit row by row)."""
    import torch

    monkeypatch.setenv("TVS_SCRATCH_MB", "1")
    n = 30
    host, dems = _make(TILES, seed=5)
    outs = _outs(TILES, 0.0)
    tl = [(dems[x], outs[x], *TILES[x][2:]) for x in range(len(TILES))]
    note("batch with forced chunking and counting")
    b = tvs.Batch(tl, n, flags=tvs.FLAG_COUNT_EVALS)
    b.run()
    torch.cuda.synchronize()
    inf = b.info()
    assert inf.chunks > 1
    done = 0
    for x, (H, W, dx, h0, R) in enumerate(TILES):
        ref, st = tvs.total_viewshed(dems[x], dx, h0, n, R, flags=tvs.FLAG_COUNT_EVALS, stats=True)
        torch.cuda.synchronize()
        np.testing.assert_allclose(outs[x].cpu().numpy(), ref.cpu().numpy(), rtol=1e-13, atol=0)
        done += st.sweep_evals_done
    assert inf.sweep_evals_done == done
    b.run()  # a second pass counts again from zero
    torch.cuda.synchronize()
    assert b.info().sweep_evals_done == done
    b.close()


def test_batch_compact_layout(tvs, monkeypatch):
    """Batches with compacted skewed buffers (TVS_FLAG_COMPACT) give the plain batch's maps bit
    for bit, with one chunk and with many."""
    import torch

    n = 30
    host, dems = _make(TILES, seed=9)
    outs_p = _outs(TILES, 0.0)
    outs_c = _outs(TILES, 0.0)
    tl_p = [(dems[x], outs_p[x], *TILES[x][2:]) for x in range(len(TILES))]
    tl_c = [(dems[x], outs_c[x], *TILES[x][2:]) for x in range(len(TILES))]
    for budget in (None, "1"):
        if budget:
            monkeypatch.setenv("TVS_SCRATCH_MB", budget)
        note(f"batch compact budget={budget}")
        bp = tvs.Batch(tl_p, n)
        bc = tvs.Batch(tl_c, n, flags=tvs.FLAG_COMPACT)
        bp.run()
        bc.run()
        torch.cuda.synchronize()
        assert bc.info().chunks <= bp.info().chunks
        for x in range(len(TILES)):
            assert torch.equal(outs_p[x], outs_c[x]), f"tile {x}"
        bp.close()
        bc.close()


def test_batch_autotune(tvs):
    import torch

    n = 12
    host, dems = _make(TILES[:4], seed=9)
    outs = _outs(TILES[:4], 0.0)
    tl = [(dems[x], outs[x], *TILES[x][2:]) for x in range(4)]
    note("batch autotune")
    b = tvs.Batch(tl, n, flags=tvs.FLAG_AUTOTUNE)
    inf = b.info()
    assert inf.tuned == 1 and inf.tune_ms > 0 and inf.waves_per_group in (2, 4, 8)
    b.run()
    torch.cuda.synchronize()
    for x in range(4):
        H, W, dx, h0, R = TILES[x]
        ref = tvs.total_viewshed(dems[x], dx, h0, n, R)
        torch.cuda.synchronize()
        np.testing.assert_allclose(outs[x].cpu().numpy(), ref.cpu().numpy(), rtol=1e-13, atol=0)
    bks = b.buckets()
    assert all(bk["tuned"] == 1 and bk["waves_per_group"] in (2, 4, 8) and bk["groups_per_cu"] in (0, 1, 2, 4, 8, 16)
               for bk in bks)
    # the shapes are remembered per size class
    b2 = tvs.Batch(tl, n)
    assert b2.info().tuned == 1
    assert [(x["waves_per_group"], x["groups_per_cu"]) for x in b2.buckets()] == \
        [(x["waves_per_group"], x["groups_per_cu"]) for x in bks]
    b.close()
    b2.close()


def test_batch_long_lines_of_sight(tvs):
    """Tiles whose lines of sight reach up to 2000 steps: the batch and each tile alone take the
    sliding maxima with the deeper range table; maps equal the full walk's, counts equal the
    single-tile counts."""
    import torch

    n = 8
    tiles = [(3, 2100, 10.0, 1.5, 20000.0), (4, 2050, 10.0, 5.0, 19500.0), (2, 1000, 10.0, 1.5, 9000.0)]
    rng = np.random.default_rng(43)
    dems = [torch.from_numpy((800.0 + rng.normal(0.0, 3.0, (H, W)).cumsum(axis=1)).astype(np.float32)).cuda()
            for (H, W, *_r) in tiles]
    outs = _outs(tiles, 0.0)
    note("batch with lines of sight up to 2000 steps")
    b = tvs.Batch([(dems[x], outs[x], *tiles[x][2:]) for x in range(len(tiles))], n, flags=tvs.FLAG_COUNT_EVALS)
    b.run()
    torch.cuda.synchronize()
    done = 0
    for x, (H, W, dx, h0, R) in enumerate(tiles):
        ref, st = tvs.total_viewshed(dems[x], dx, h0, n, R, flags=tvs.FLAG_COUNT_EVALS, stats=True)
        full = tvs.total_viewshed(dems[x], dx, h0, n, R, flags=tvs.FLAG_NO_PRUNE)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(ref.cpu().numpy(), full.cpu().numpy())
        np.testing.assert_allclose(outs[x].cpu().numpy(), ref.cpu().numpy(), rtol=1e-13, atol=0)
        assert 0 < st.sweep_evals_done < st.los_evals
        done += st.sweep_evals_done
    assert b.info().sweep_evals_done == done
    b.close()


_TUNE_SCRIPT = r"""
import json, sys
sys.path.insert(0, sys.argv[1])
import torch
import paper_2003_02200_amd as tvs
from synth import fractal_dem
torch.cuda.set_device(0)
tiles = [(300, 280, 10.0, 1.5, 3000.0), (70, 90, 10.0, 5.0, 900.0)]
dems = [torch.from_numpy(fractal_dem(max(H, W), 60 + x, 0.6, 900.0)[:H, :W].copy()).cuda()
        for x, (H, W, *_r) in enumerate(tiles)]
outs = [torch.zeros(d.shape, dtype=torch.float64, device="cuda") for d in dems]
flags = tvs.FLAG_AUTOTUNE if sys.argv[2] == "tune" else 0
b = tvs.Batch([(dems[x], outs[x], *tiles[x][2:]) for x in range(2)], 12, flags=flags)
b.run()
m = tvs.total_viewshed(dems[0], 10.0, 1.5, 12, 3000.0, flags=flags)
torch.cuda.synchronize()
print(json.dumps({"buckets": b.buckets(), "sum": float(outs[0].sum()), "single": float(m.sum())}))
b.close()
"""


def test_tuned_shapes_persist_across_processes(tvs, tmp_path):
    """Shapes timed in one process (batch buckets and the single-grid sweep) are written to the tune
    cache with the device and library build, and a fresh process on the same build starts with them;
    maps are the same with any shape."""
    import json
    import os
    import subprocess

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, TVS_TUNE_CACHE=str(tmp_path / "tune.txt"))
    note("tune cache: timing process")
    a = subprocess.run([sys.executable, "-c", _TUNE_SCRIPT, root, "tune"], env=env, capture_output=True, text=True,
                       timeout=180)
    assert a.returncode == 0, a.stderr[-2000:]
    ra = json.loads(a.stdout.strip().splitlines()[-1])
    lines = (tmp_path / "tune.txt").read_text().splitlines()
    assert len(lines) >= len(ra["buckets"]) + 1  # every bucket, and the single-grid sweep (kind 1)
    assert {ln.split()[2] for ln in lines} == {"0", "1"}
    note("tune cache: fresh process")
    b = subprocess.run([sys.executable, "-c", _TUNE_SCRIPT, root, "reuse"], env=env, capture_output=True, text=True,
                       timeout=180)
    assert b.returncode == 0, b.stderr[-2000:]
    rb = json.loads(b.stdout.strip().splitlines()[-1])
    assert all(x["tuned"] == 1 for x in rb["buckets"])
    assert [(x["waves_per_group"], x["groups_per_cu"]) for x in rb["buckets"]] == \
        [(x["waves_per_group"], x["groups_per_cu"]) for x in ra["buckets"]]
    assert ra["sum"] == rb["sum"] and ra["single"] == rb["single"]
