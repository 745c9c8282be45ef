"""GPU parity of libtvs against the CPU oracle (run on an MI355X; marked `gpu`).

Bar (from the method's arithmetic):
* per-sector skewed viewshed (integer ring sums U and clipped-ring counts e): bit-exact against
  the oracle taking the same decisions in the same precision -- double with the slope as the
  difference times the double reciprocal for the default path (oracle prec=65), the double
  quotient for TVS_FLAG_SLOPE_F64 or TVS_FLAG_SLOPE_EXACT (prec=64), and the paper's float
  kernels for TVS_FLAG_SLOPE_F32 (difference times float reciprocal, prec=33; with
  TVS_FLAG_SLOPE_EXACT the correctly rounded float quotient, prec=32);
* total viewshed map: equal to that oracle up to double summation order (rtol 1e-12);
* against the all-double oracle: per-cell relative error <= 1e-4 on cells without a horizon
  flip, horizon flips (POV-sector pairs whose U or e differ) <= 1e-5 of all pairs.
"""
import math
import sys

import numpy as np
import pytest

from synth import cone, flat, fractal_dem, plane, workload_dem, WORKLOADS

pytestmark = pytest.mark.gpu
INF = math.inf
P_DEFAULT, P_DOUBLE, P_F32, P_F32_EXACT = 65, 64, 33, 32
# (flags, oracle precision) of every decision mode: default, double quotient, float, float quotient
F64, EXACT, F32 = 0x1, 0x8, 0x40
MODES = [(0, P_DEFAULT), (F64, P_DOUBLE), (F32, P_F32), (F32 | EXACT, P_F32_EXACT)]


def note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tvs():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2003_02200_amd as t

    t.lib()  # raises if the HIP library is missing: no fallback
    return t


def packed(o):
    v = o["U"].astype(np.uint32) | (o["e"].astype(np.uint32) << np.uint32(30))
    v[o["valid"] == 0] = np.uint32(0xFFFFFFFF)
    return v


def _int_dem(H, W, seed, hi=12):
    rng = np.random.default_rng(seed)
    return np.round(rng.uniform(0, hi, (H, W))).astype(np.float32)


SHAPES = [
    # (H, W, n, R, terrain)
    (1, 1, 3, INF, "fractal"),
    (1, 9, 4, INF, "int"),
    (9, 1, 4, 25.0, "int"),
    (2, 2, 8, INF, "fractal"),
    (37, 53, 7, INF, "fractal"),
    (37, 53, 7, 123.4, "int"),
    (53, 37, 12, 530.0, "fractal"),
    (70, 130, 3, 5.0, "fractal"),      # rho < 1: no target in range
    (64, 64, 2, INF, "flat"),
    (17, 300, 8, INF, "fractal"),      # long rows: many segments and 32-step blocks
    (300, 17, 9, 2000.0, "int"),
    (130, 70, 180, 700.0, "fractal"),
    (45, 45, 4, 300.0, "plane"),
    (9, 6000, 3, 2000.0, "fractal"),   # rows long enough for 16 waves per sweep workgroup
    (3000, 9, 4, 1500.0, "int"),       # 8 waves per workgroup on the transposed axes
]


def _dem(H, W, kind, seed=3):
    if kind == "fractal":
        return fractal_dem(max(H, W), seed, 0.6, 400.0)[:H, :W].copy()
    if kind == "int":
        return _int_dem(H, W, seed)
    if kind == "flat":
        return flat(H, W, 17.0)
    return plane(H, W, 0.75, -0.5, 300.0)


def _sectors(n):
    return list(range(n)) if n <= 16 else sorted(set(list(range(0, n, 7)) + [n // 4, n // 2, 3 * n // 4, n - 1]))


@pytest.mark.parametrize("H,W,n,R,kind", SHAPES)
def test_sector_rays_bitexact_default(tvs, orc, H, W, n, R, kind):
    dem = _dem(H, W, kind)
    for k in _sectors(n):
        note(f"sector_rays default H={H} W={W} n={n} R={R} k={k} kind={kind}")
        g = tvs.debug_sector_rays(dem, 10.0, 1.5, n, R, k)
        o = orc.sector_V(dem, 10.0, 1.5, n, R, k, prec=P_DEFAULT)
        assert g.shape == o["U"].shape
        bad = np.argwhere(g != packed(o))
        assert bad.size == 0, f"k={k}: {len(bad)} samples differ, first {bad[:3].tolist()}"


@pytest.mark.parametrize("H,W,n,R,kind", SHAPES)
def test_sector_rays_bitexact_float(tvs, orc, H, W, n, R, kind):
    """TVS_FLAG_SLOPE_F32 (the paper's float kernels) against the oracle's float mode."""
    dem = _dem(H, W, kind, seed=4)
    for k in _sectors(n):
        note(f"sector_rays float H={H} W={W} n={n} R={R} k={k} kind={kind}")
        g = tvs.debug_sector_rays(dem, 10.0, 1.5, n, R, k, flags=F32)
        o = orc.sector_V(dem, 10.0, 1.5, n, R, k, prec=P_F32)
        assert np.array_equal(g, packed(o)), f"k={k}"


@pytest.mark.parametrize("H,W,n,R,kind", SHAPES[::2])
def test_sector_rays_bitexact_float_quotient(tvs, orc, H, W, n, R, kind):
    """TVS_FLAG_SLOPE_F32 | TVS_FLAG_SLOPE_EXACT (correctly rounded float quotient) against the
    oracle's float division mode."""
    dem = _dem(H, W, kind, seed=6)
    for k in _sectors(n):
        note(f"sector_rays float quotient H={H} W={W} n={n} R={R} k={k} kind={kind}")
        g = tvs.debug_sector_rays(dem, 10.0, 1.5, n, R, k, flags=F32 | EXACT)
        o = orc.sector_V(dem, 10.0, 1.5, n, R, k, prec=P_F32_EXACT)
        assert np.array_equal(g, packed(o)), f"k={k}"


@pytest.mark.parametrize("h0", [0.0, -0.0, 1.5, -2.0])
def test_sector_rays_signed_zeros_and_ties(tvs, orc, h0):
    """Grids of +0/-0 and small integers with h0 = 0 give many exactly equal slopes (hidden under
    the strict comparison) and zero slopes of both signs: the sweep's sign-bit tests must agree
    with the oracle's comparisons bit for bit."""
    rng = np.random.default_rng(99)
    H, W = 41, 150
    dem = np.round(rng.uniform(-2, 3, (H, W))).astype(np.float32)
    dem[rng.uniform(size=(H, W)) < 0.5] = 0.0
    dem = np.where(rng.uniform(size=(H, W)) < 0.5, np.float32(-0.0) * np.abs(dem), dem).astype(np.float32)
    for n, R in ((8, INF), (12, 400.0)):
        for k in range(n):
            note(f"signed zeros h0={h0} n={n} R={R} k={k}")
            for flags, prec in MODES:
                g = tvs.debug_sector_rays(dem, 10.0, h0, n, R, k, flags=flags)
                o = orc.sector_V(dem, 10.0, h0, n, R, k, prec=prec)
                assert np.array_equal(g, packed(o)), f"n={n} k={k} flags={flags}"


@pytest.mark.parametrize("H,W,n,R,kind", SHAPES[::2])
def test_sector_rays_bitexact_double(tvs, orc, H, W, n, R, kind):
    dem = _dem(H, W, kind, seed=5)
    for k in _sectors(n):
        note(f"sector_rays double H={H} W={W} n={n} R={R} k={k} kind={kind}")
        g = tvs.debug_sector_rays(dem, 10.0, 1.5, n, R, k, flags=F64)
        o = orc.sector_V(dem, 10.0, 1.5, n, R, k, prec=P_DOUBLE)
        assert np.array_equal(g, packed(o)), f"k={k}"
        assert np.array_equal(tvs.debug_sector_rays(dem, 10.0, 1.5, n, R, k, flags=EXACT), g)


@pytest.mark.parametrize("H,W,n,R,kind", SHAPES[1::2])
def test_sector_rays_relocation_kernel(tvs, orc, H, W, n, R, kind):
    """TVS_FLAG_RELOCATE: the relocation kernel writes skwDEM and the sweep reads it; the same ring
    sums as the oracle (and as the default sweep, which gathers its rows from the grid)."""
    dem = _dem(H, W, kind, seed=9)
    for k in _sectors(n):
        for flags, prec in MODES[::2]:
            note(f"sector_rays relocate H={H} W={W} n={n} R={R} k={k} flags={flags}")
            g = tvs.debug_sector_rays(dem, 10.0, 1.5, n, R, k, flags=tvs.FLAG_RELOCATE | flags)
            o = orc.sector_V(dem, 10.0, 1.5, n, R, k, prec=prec)
            assert np.array_equal(g, packed(o)), f"k={k} flags={flags}"


@pytest.mark.parametrize("H,W,n,R,kind", SHAPES[1::3])
def test_sector_rays_prefix_max_variant(tvs, orc, H, W, n, R, kind):
    """The lane-per-target sweep (wavefront prefix-max horizon) gives the same integers."""
    dem = _dem(H, W, kind, seed=8)
    for k in _sectors(n)[:6]:
        for flags, prec in MODES:
            note(f"sector_rays scan H={H} W={W} n={n} R={R} k={k} flags={flags}")
            g = tvs.debug_sector_rays(dem, 10.0, 1.5, n, R, k, flags=tvs.FLAG_SWEEP_SCAN | flags)
            o = orc.sector_V(dem, 10.0, 1.5, n, R, k, prec=prec)
            assert np.array_equal(g, packed(o)), f"k={k} flags={flags}"


def _walled(H, W, seed):
    """Low noisy ground with a few tall walls and towers: lines of sight that pass a wall see
    nothing more, so the sweep's early exit fires in the middle of rows."""
    rng = np.random.default_rng(seed)
    dem = rng.uniform(0, 6, (H, W)).astype(np.float32)
    for _ in range(4):
        c = int(rng.integers(0, W))
        dem[:, c:c + 2] += np.float32(rng.uniform(200, 900))
    for _ in range(6):
        i, j = int(rng.integers(0, H)), int(rng.integers(0, W))
        dem[max(0, i - 3):i + 3, max(0, j - 3):j + 3] += np.float32(rng.uniform(300, 2000))
    return dem


EXIT_CASES = [
    # (H, W, n, R, terrain): long rows so that exits land in blocks, before the tail and at K
    (40, 400, 6, INF, "walled"),
    (400, 40, 6, 1500.0, "walled"),
    (90, 333, 10, 777.0, "fractal"),
    (64, 700, 3, 3205.0, "walled"),
    (257, 257, 24, 2570.0, "fractal"),
]


def _exit_dem(H, W, kind, seed):
    if kind == "walled":
        return _walled(H, W, seed)
    return fractal_dem(max(H, W), seed, 0.7, 2500.0)[:H, :W].copy()


@pytest.mark.parametrize("H,W,n,R,kind", EXIT_CASES)
def test_early_exit_equals_full_walk(tvs, orc, H, W, n, R, kind):
    """The sweep's early exit changes no ring sum: pruned and full walks agree bit for bit with
    each other and with the oracle, in every decision mode, for observers above and below
    ground."""
    dem = _exit_dem(H, W, kind, seed=H + W)
    for h0 in (1.5, -3.0, 40.0):
        for k in range(n):
            note(f"early exit H={H} W={W} n={n} R={R} kind={kind} h0={h0} k={k}")
            for flags, prec in MODES:
                g = tvs.debug_sector_rays(dem, 10.0, h0, n, R, k, flags=flags)
                full = tvs.debug_sector_rays(dem, 10.0, h0, n, R, k, flags=flags | tvs.FLAG_NO_PRUNE)
                assert np.array_equal(g, full), f"k={k} flags={flags}: pruned and full walks differ"
                o = orc.sector_V(dem, 10.0, h0, n, R, k, prec=prec)
                assert np.array_equal(g, packed(o)), f"k={k} flags={flags}"


# Rows long enough to take the sweep's other bound paths: an unbounded distance on 4000-sample rows
# (ranges beyond the range table's 64 blocks fall back to the row-end maxima), and rows of 18000
# doubles or 32767 floats, whose LDS leaves no room for the range table: with bounded lines of sight
# they are swept in pieces (each piece's reach with its own tables), unbounded ones stream through LDS
# windows (and, without the bounds, are swept whole). Two sectors keep the skewed arrays small
# (tan s' = 0).
# unbounded steps (the block-pair skip test, exit ranges past the table: the accumulated maxima);
# 1900 steps (the most the sliding maxima take with the 6-level table: exit ranges up to 61 blocks);
# 1950 and 3800 steps (the 7-level table: exit ranges up to 63 and 122 blocks); rows beyond the
# table's LDS in pieces and streamed; float rows with the 7-level table, and beyond the table's LDS
LONG_ROWS = [(5, 4000, INF, 0, P_DEFAULT), (5, 4000, 19000.0, 0, P_DEFAULT), (5, 4000, 19500.0, 0, P_DEFAULT),
             (5, 4000, 38000.0, 0, P_DEFAULT), (2, 18000, 2500.0, 0, P_DEFAULT), (2, 18000, INF, 0, P_DEFAULT),
             (5, 4000, 19500.0, F32, P_F32), (3, 32767, 3000.0, F32, P_F32), (3, 32767, INF, F32, P_F32)]


@pytest.mark.parametrize("H,W,R,flags,prec", LONG_ROWS)
def test_long_rows_bound_paths(tvs, orc, H, W, R, flags, prec):
    # random-walk profiles (a fractal square of side W would take gigabytes)
    dem = (1000.0 + np.random.default_rng(41).normal(0.0, 4.0, (H, W)).cumsum(axis=1)).astype(np.float32)
    for k in range(2):
        note(f"long rows H={H} W={W} R={R} flags={flags} k={k}")
        g = tvs.debug_sector_rays(dem, 10.0, 1.5, 2, R, k, flags=flags)
        full = tvs.debug_sector_rays(dem, 10.0, 1.5, 2, R, k, flags=flags | tvs.FLAG_NO_PRUNE)
        assert np.array_equal(g, full), f"k={k}: pruned and full walks differ"
        o = orc.sector_V(dem, 10.0, 1.5, 2, R, k, prec=prec)
        bad = np.argwhere(g != packed(o))
        assert bad.size == 0, f"k={k}: {len(bad)} samples differ, first {bad[:3].tolist()}"
    _, st = tvs.total_viewshed(dem, 10.0, 1.5, 2, R, flags=flags | tvs.FLAG_COUNT_EVALS, stats=True)
    assert 0 < st.sweep_evals_done <= st.los_evals


LONG_DOUBLE = [
    # (H, W, n, R, sector whose skewed rows are the long ones): double rows of 25000 and 32767 samples,
    # beyond what one workgroup's LDS holds; unbounded and bounded lines of sight
    (2, 25000, 4, INF, 0),
    (2, 25000, 4, 50000.0, 0),
    (25000, 2, 4, INF, 2),  # the long rows in the transposed frame (the 90 deg axis)
    (3, 32767, 4, INF, 0),
    (3, 32767, 4, 30000.0, 0),
    # a skinny grid: only the axis sector along the long side streams; the skewed rows of the others
    # (22.5 and 45 deg: at most 43 and 19 samples) take the single-window sweep, sized by their bound
    (16, 32767, 8, 20000.0, 0),
]


@pytest.mark.parametrize("H,W,n,R,k", LONG_DOUBLE)
def test_double_rows_beyond_lds_streamed(tvs, orc, H, W, n, R, k):
    """Rows longer than the LDS are swept in pieces: with bounded lines of sight each piece's reach is
    loaded whole and swept like a short row; unbounded ones stream their targets through LDS windows,
    each lane's horizon and ring sums carried from window to window. The ring sums of the long sector
    bit for bit against the oracle (default and quotient decisions, rows gathered from the grid or read
    from skwDEM), and the whole map against the oracle."""
    long_side = max(H, W)
    prof = (1000.0 + np.random.default_rng(43).normal(0.0, 4.0, (min(H, W), long_side)).cumsum(axis=1))
    dem = np.ascontiguousarray((prof if W >= H else prof.T).astype(np.float32))
    for flags, prec in ((0, P_DEFAULT), (F64, P_DOUBLE), (0x200, P_DEFAULT)):
        note(f"long double rows H={H} W={W} n={n} R={R} k={k} flags={flags}")
        g = tvs.debug_sector_rays(dem, 10.0, 1.5, n, R, k, flags=flags)
        o = orc.sector_V(dem, 10.0, 1.5, n, R, k, prec=prec)
        bad = np.argwhere(g != packed(o))
        assert bad.size == 0, f"flags={flags}: {len(bad)} samples differ, first {bad[:3].tolist()}"
    note(f"long double rows H={H} W={W} n={n} R={R}: total")
    g, st = tvs.total_viewshed(dem, 10.0, 1.5, n, R, flags=tvs.FLAG_COUNT_EVALS, stats=True)
    np.testing.assert_allclose(g, orc.total(dem, 10.0, 1.5, n, R, prec=P_DEFAULT), rtol=1e-12, atol=0)
    # the streamed pieces skip blocks and stop early like the single-window sweep; without the bounds
    # they walk every target in range, to the same map
    gf, sf = tvs.total_viewshed(dem, 10.0, 1.5, n, R, flags=tvs.FLAG_COUNT_EVALS | tvs.FLAG_NO_PRUNE, stats=True)
    np.testing.assert_array_equal(g, gf)
    assert sf.sweep_evals_done == sf.los_evals
    assert 0 < st.sweep_evals_done < st.los_evals
    # the chunk's long sector streams and its short ones take the single-window sweep, also when both
    # read skwDEM rows in the compacted layout: the same map
    gr = tvs.total_viewshed(dem, 10.0, 1.5, n, R, flags=tvs.FLAG_RELOCATE | tvs.FLAG_COMPACT)
    np.testing.assert_array_equal(g, gr)
    print(f"long rows H={H} W={W} R={R}: {st.sweep_evals_done / st.los_evals:.3f} of the evaluations carried out",
          flush=True)


@pytest.mark.parametrize("bad", [float("nan"), float("inf"), -float("inf"), 1e-30, -2e-25])
def test_device_grid_checked_on_device(tvs, bad):
    """Entry points that take device grids check the elevations on the device: a non-finite value, or a
    nonzero one below 2^-60 m, turns the whole map into NaN (the status cannot report it); the same grid
    without that cell gives a finite map."""
    import torch

    dem = fractal_dem(70, 3, 0.6, 400.0)[:50, :70].copy()
    good = torch.from_numpy(dem).cuda()
    dem[17, 33] = np.float32(bad)
    d = torch.from_numpy(dem).cuda()
    note(f"device grid check bad={bad}")
    ok = tvs.total_viewshed(good, 10.0, 1.5, 8, 300.0)
    assert bool(torch.isfinite(ok).all())
    for out in (tvs.total_viewshed(d, 10.0, 1.5, 8, 300.0), tvs.total_viewshed_noalloc(d, 10.0, 1.5, 8, 300.0)):
        torch.cuda.synchronize()
        assert bool(torch.isnan(out).all())
    o = torch.zeros((50, 70), dtype=torch.float64, device="cuda")
    tvs.total_viewshed_tiles([(d, o, 10.0, 1.5, 300.0)], 8)
    torch.cuda.synchronize()
    assert bool(torch.isnan(o).all())
    # the host entry point rejects the same grid before any work
    with pytest.raises(tvs.TvsError) as ei:
        tvs.total_viewshed(dem, 10.0, 1.5, 8, 300.0)
    assert ei.value.status == -1


@pytest.mark.parametrize("H,W,n,R,kind", EXIT_CASES[:3])
def test_evaluation_counts(tvs, H, W, n, R, kind):
    """The sweep's own count of evaluations: the closed form without the early exit (and for the
    lane-per-target variant), fewer with it; the maps are identical."""
    dem = _exit_dem(H, W, kind, seed=7)
    ev, _ = tvs.los_evals(H, W, 10.0, n, R)
    note(f"evaluation counts H={H} W={W} n={n} R={R}")
    full, st_full = tvs.total_viewshed(dem, 10.0, 1.5, n, R, flags=tvs.FLAG_NO_PRUNE | tvs.FLAG_COUNT_EVALS,
                                       stats=True)
    assert st_full.sweep_evals_done == ev == st_full.los_evals
    _, st_scan = tvs.total_viewshed(dem, 10.0, 1.5, n, R, flags=tvs.FLAG_SWEEP_SCAN | tvs.FLAG_COUNT_EVALS,
                                    stats=True)
    assert st_scan.sweep_evals_done == ev
    pr, st = tvs.total_viewshed(dem, 10.0, 1.5, n, R, flags=tvs.FLAG_COUNT_EVALS, stats=True)
    assert 0 < st.sweep_evals_done < ev
    np.testing.assert_array_equal(pr, full)
    print(f"{kind} {H}x{W}: evaluations carried out {st.sweep_evals_done / ev:.3f} of {ev}", flush=True)


@pytest.mark.parametrize("H,W,n,R,kind", SHAPES)
def test_total_small(tvs, orc, H, W, n, R, kind):
    dem = _dem(H, W, kind, seed=11)
    for flags, prec in MODES:
        note(f"total H={H} W={W} n={n} R={R} kind={kind} flags={flags}")
        g = tvs.total_viewshed(dem, 10.0, 1.5, n, R, flags=flags)
        np.testing.assert_allclose(g, orc.total(dem, 10.0, 1.5, n, R, prec=prec), rtol=1e-12, atol=0)


@pytest.mark.parametrize("H,W,n,R,kind", SHAPES)
def test_total_compact_layout(tvs, orc, H, W, n, R, kind):
    """The compacted skewed layout (TVS_FLAG_COMPACT: skewed row t in row t mod (Hx + 1)) moves
    rows, not results: maps bit-identical to the plain layout in the default and float modes and
    for the lane-per-target sweep, equal to the oracle, in no more scratch. The wide and tall
    shapes wrap the rows many times over."""
    dem = _dem(H, W, kind, seed=13)
    plain0 = None
    for flags, prec in (MODES[0], MODES[2]):
        note(f"compact H={H} W={W} n={n} R={R} kind={kind} flags={flags}")
        plain, st_p = tvs.total_viewshed(dem, 10.0, 1.5, n, R, flags=flags, stats=True)
        comp, st_c = tvs.total_viewshed(dem, 10.0, 1.5, n, R, flags=flags | tvs.FLAG_COMPACT, stats=True)
        assert np.array_equal(plain, comp), f"flags={flags}"
        assert st_c.scratch_bytes <= st_p.scratch_bytes and st_c.chunks <= st_p.chunks
        # the relocation kernel and skwDEM (plain and compacted) give the gathering sweep's map
        for extra in (tvs.FLAG_RELOCATE, tvs.FLAG_RELOCATE | tvs.FLAG_COMPACT):
            assert np.array_equal(tvs.total_viewshed(dem, 10.0, 1.5, n, R, flags=flags | extra), plain), extra
        np.testing.assert_allclose(comp, orc.total(dem, 10.0, 1.5, n, R, prec=prec), rtol=1e-12, atol=0)
        plain0 = plain if plain0 is None else plain0
    scan = tvs.total_viewshed(dem, 10.0, 1.5, n, R, flags=tvs.FLAG_SWEEP_SCAN | tvs.FLAG_COMPACT)
    assert np.array_equal(scan, plain0)


def test_compact_layout_many_chunks(tvs, monkeypatch):
    """A 1 MB scratch budget splits the sectors into many chunks; the compacted layout fits more
    sectors in each and the map stays bit-identical."""
    dem = _dem(130, 70, "fractal", seed=17)
    ref = tvs.total_viewshed(dem, 10.0, 1.5, 180, 700.0)
    monkeypatch.setenv("TVS_SCRATCH_MB", "1")
    note("compact 130x70 n=180 with a 1 MB scratch budget")
    plain, st_p = tvs.total_viewshed(dem, 10.0, 1.5, 180, 700.0, stats=True)
    comp, st_c = tvs.total_viewshed(dem, 10.0, 1.5, 180, 700.0, flags=tvs.FLAG_COMPACT, stats=True)
    assert st_p.chunks > 10 and st_c.chunks < st_p.chunks
    assert np.array_equal(plain, ref) and np.array_equal(comp, ref)


@pytest.mark.parametrize("n", [72, 73, 144])
def test_total_full_chunks(tvs, orc, n):
    """Sector counts at the chunk capacity (72 sectors in the kernel arguments: the last entries and
    the pointers after them lie past 4 KB of arguments) and just beyond it, against the oracle."""
    dem = _dem(41, 37, "fractal", seed=23)
    for flags, prec in (MODES[0], MODES[2]):
        note(f"full chunks n={n} flags={flags}")
        g, st = tvs.total_viewshed(dem, 10.0, 1.5, n, 333.0, flags=flags, stats=True)
        assert st.chunks == (n + 71) // 72
        np.testing.assert_allclose(g, orc.total(dem, 10.0, 1.5, n, 333.0, prec=prec), rtol=1e-12, atol=0)


def test_flat_full_disc_on_gpu(tvs):
    """P1 through the GPU: interior cells of flat ground get pi R^2."""
    H = W = 90
    R = 300.0
    note("flat full disc 90x90 n=45")
    g = tvs.total_viewshed(flat(H, W, 5.0), 10.0, 1.5, 45, R)
    m = int(math.ceil(R / 10.0)) + 2
    np.testing.assert_allclose(g[m:-m, m:-m], math.pi * R * R, rtol=1e-12)
    assert np.all(g <= math.pi * R * R * (1 + 1e-12))


def test_kahan_float_accumulation(tvs, orc):
    dem = fractal_dem(64, 21, 0.6, 900.0)
    note("kahan32 64x64 n=60")
    g = tvs.total_viewshed(dem, 10.0, 1.5, 60, 500.0, flags=tvs.FLAG_ACC_KAHAN32)
    o = orc.total(dem, 10.0, 1.5, 60, 500.0, prec=P_DEFAULT)
    np.testing.assert_allclose(g, o, rtol=2e-6)
    g = tvs.total_viewshed(dem, 10.0, 1.5, 60, 500.0, flags=tvs.FLAG_ACC_KAHAN32 | F32)
    np.testing.assert_allclose(g, orc.total(dem, 10.0, 1.5, 60, 500.0, prec=P_F32), rtol=2e-6)


def test_async_torch_stream_and_stats(tvs):
    import torch

    dem = fractal_dem(96, 2, 0.6, 800.0)[:80].copy()
    note("async on a side stream with stats 80x96 n=30")
    host = tvs.total_viewshed(dem, 10.0, 1.5, 30, 400.0)
    s = torch.cuda.Stream()
    d = torch.from_numpy(dem).cuda()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        out, st = tvs.total_viewshed(d, 10.0, 1.5, 30, 400.0, stream=s, stats=True)
    s.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), host)
    ev, pairs = tvs.los_evals(80, 96, 10.0, 30, 400.0)
    assert st.los_evals == ev and st.pov_sector_pairs == pairs
    assert st.sweep_launches == st.chunks and st.sweep_ms > 0


@pytest.mark.parametrize("H,W,n,R,pov", [(37, 53, 7, INF, (5, 9)), (64, 64, 180, 500.0, (0, 0)),
                                         (64, 64, 180, 500.0, (63, 17)), (1, 1, 3, INF, (0, 0)),
                                         (200, 90, 24, 1500.0, (100, 45)), (50, 50, 4, INF, (10, 40))])
def test_singular(tvs, orc, H, W, n, R, pov):
    dem = fractal_dem(max(H, W), 17, 0.6, 600.0)[:H, :W].copy()
    i0, j0 = pov
    note(f"singular H={H} W={W} n={n} R={R} pov={pov}")
    for flags, prec in MODES + [(EXACT, P_DOUBLE)]:
        area, rays = tvs.singular_viewshed(dem, 10.0, 1.5, n, R, i0, j0, flags=flags, rays=True)
        o = orc.singular(dem, 10.0, 1.5, n, R, i0, j0, prec=prec)
        want = o["U"].astype(np.uint32) | (o["e"].astype(np.uint32) << np.uint32(30))
        assert np.array_equal(rays, want), flags
        assert area == pytest.approx(o["area"], rel=1e-12)


def test_singular_cone_shadow(tvs):
    """P12 through the GPU ray scan: the 45 deg line of sight to a cone apex 50 cells away."""
    dem = cone(81, 81, 60, 60, 30.0, 8.0)
    note("singular cone")
    _, rays = tvs.singular_viewshed(dem, 10.0, 1.5, 4, INF, 10, 10, rays=True)
    assert rays[2] == 51 ** 2


def _flip_stats(tvs, orc, dem, dx, h0, n, R, sectors, flags=0):
    flips = pairs = 0
    for k in sectors:
        g = tvs.debug_sector_rays(dem, dx, h0, n, R, k, flags=flags)
        o = orc.sector_V(dem, dx, h0, n, R, k, prec=64)
        p = packed(o)
        v = o["valid"].astype(bool)
        assert np.array_equal(g == 0xFFFFFFFF, ~v)
        pairs += int(v.sum())
        flips += int(np.sum(g[v] != p[v]))
    return flips, pairs


def test_workload_128_full_map(tvs, orc):
    """The 128 x 128, 180-sector workload: whole map against both oracle precisions."""
    w = WORKLOADS["tvs128"]
    dem = workload_dem("tvs128")
    args = (w["spacing"], w["obs_height"], w["n_sectors"], w["max_dist"])
    note("workload tvs128 total")
    g = tvs.total_viewshed(dem, *args)
    np.testing.assert_allclose(g, orc.total(dem, *args, prec=P_DEFAULT), rtol=1e-12)
    o64 = orc.total(dem, *args, prec=64)
    for name, flags in (("default", 0), ("float", F32)):
        note(f"workload tvs128 flips {name}")
        m = g if flags == 0 else tvs.total_viewshed(dem, *args, flags=flags)
        flips, pairs = _flip_stats(tvs, orc, dem, *args, range(w["n_sectors"]), flags=flags)
        rel = np.abs(m - o64) / o64
        print(f"tvs128 {name}: pairs={pairs} flips={flips} rate={flips / pairs:.3g} max_rel={rel.max():.3g} "
              f"cells>1e-4={int((rel > 1e-4).sum())}", flush=True)
        assert flips / pairs <= 1e-5
        # cells off by more than rounding are exactly the cells fed by a flipped pair: at most 2 per flip
        assert int((rel > 1e-10).sum()) <= 2 * flips
        assert np.median(rel) < 1e-12


def test_workload_2000_sampled(tvs, orc):
    """The 2000 x 2000, 180-sector, 10 km workload in the bench's launch configuration: sampled
    cells against the oracle cell by cell, plus properties that hold at any size."""
    import torch

    w = WORKLOADS["tvs2000"]
    dem = workload_dem("tvs2000")
    args = (w["spacing"], w["obs_height"], w["n_sectors"], w["max_dist"])
    note("workload tvs2000 total (device-resident, async)")
    d = torch.from_numpy(dem).cuda()
    out = tvs.total_viewshed(d, *args)
    torch.cuda.synchronize()
    g = out.cpu().numpy()
    note("workload tvs2000 total without the early exit")
    full = tvs.total_viewshed(d, *args, flags=tvs.FLAG_NO_PRUNE)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(full.cpu().numpy(), g)
    del full
    # the exact bounds must keep doing their work: on this workload the sweep carries out 39.5 % of
    # the evaluations with the skip test on sliding maxima, 41.7 % on block pairs (a guard against
    # the sliding maxima, the block skip or the early exit silently switching off)
    _, st = tvs.total_viewshed(d, *args, flags=tvs.FLAG_COUNT_EVALS, stats=True)
    assert st.sweep_evals_done < 0.405 * st.los_evals, st.sweep_evals_done / st.los_evals
    R = w["max_dist"]
    assert np.all(np.isfinite(g)) and np.all(g > 0) and np.all(g <= math.pi * R * R * (1 + 1e-12))
    rng = np.random.default_rng(2000)
    cells = [(0, 0), (0, 1999), (1999, 0), (1999, 1999), (1000, 1000), (999, 3), (3, 1500)]
    cells += [tuple(int(x) for x in rng.integers(0, 2000, 2)) for _ in range(25)]
    worst32 = 0.0
    worst64 = 0.0
    for (i, j) in cells:
        o32 = orc.total(dem, *args, prec=P_DEFAULT, window=(i, j, 1, 1))[0, 0]  # same decisions
        o64 = orc.total(dem, *args, prec=64, window=(i, j, 1, 1))[0, 0]
        worst32 = max(worst32, abs(g[i, j] - o32) / o32)
        worst64 = max(worst64, abs(g[i, j] - o64) / o64)
    print(f"tvs2000 sampled cells={len(cells)} max_rel_vs_same_precision={worst32:.3g} "
          f"max_rel_vs_double_quotient={worst64:.3g}", flush=True)
    assert worst32 <= 1e-12
    assert worst64 <= 1e-4


def _fed_cells(info, ri, j, H, W):
    """Grid cells whose back-projection (Alg. 9) reads the skewed samples (t0 + ri, j) of a sector:
    base-frame cell (t + d_j, j) with weight 1 - r_j and, when r_j > 0, (t + d_j + 1, j) with
    weight r_j, mapped back through the sector's frame transform."""
    d, r = info["d"][j], info["r"][j]
    t = info["t0"] + ri
    p = np.concatenate([t + d, (t + d + 1)[r > 0]])
    q = np.concatenate([j, j[r > 0]])
    keep = (p >= 0) & (p < info["Hx"])
    p, q = p[keep], q[keep]
    kase = info["case"]
    if kase == 0:
        return p, q
    if kase == 1:
        return q, p
    if kase == 2:
        return q, W - 1 - p
    return p, W - 1 - q


def _flip_scan(tvs, orc, d, args, flags_a, flags_b):
    """Horizon flips between two GPU variants over every POV-sector pair (compared on the device),
    and the cells they feed."""
    import torch

    H, W = d.shape
    spacing, h0, n, R = args
    fed = np.zeros((H, W), bool)
    flips = pairs = 0
    for k in range(n):
        a = tvs.debug_sector_rays(d, spacing, h0, n, R, k, flags=flags_a)
        b = tvs.debug_sector_rays(d, spacing, h0, n, R, k, flags=flags_b)
        va = a != -1
        assert torch.equal(va, b != -1), f"k={k}: sample sets differ"
        diff = (a != b) & va
        pairs += int(va.sum())
        nf = int(diff.sum())
        if nf:
            flips += nf
            ij = diff.nonzero().cpu().numpy()
            i, j = _fed_cells(orc.sector_info(H, W, spacing, n, R, k), ij[:, 0], ij[:, 1], H, W)
            fed[i, j] = True
    torch.cuda.synchronize()
    return flips, pairs, fed


def test_workload_8000_sampled(tvs, orc):
    """The 8000 x 8000 grid (the largest grid shape of Table 2) in the bench's launch configuration:
    sampled cells against the oracle taking the same decisions, plus properties that hold at any size."""
    import torch

    w = WORKLOADS["tvs8000"]
    dem = workload_dem("tvs8000")
    args = (w["spacing"], w["obs_height"], w["n_sectors"], w["max_dist"])
    note("workload tvs8000 total (device-resident)")
    out = tvs.total_viewshed(torch.from_numpy(dem).cuda(), *args)
    torch.cuda.synchronize()
    g = out.cpu().numpy()
    del out
    R = w["max_dist"]
    assert np.all(np.isfinite(g)) and np.all(g > 0) and np.all(g <= math.pi * R * R * (1 + 1e-12))
    rng = np.random.default_rng(8000)
    cells = [(0, 0), (0, 7999), (7999, 0), (7999, 7999), (4000, 4000), (7998, 5), (2, 6000)]
    cells += [tuple(int(x) for x in rng.integers(0, 8000, 2)) for _ in range(13)]
    for (i, j) in cells:
        o = orc.total(dem, *args, prec=P_DEFAULT, window=(i, j, 1, 1))[0, 0]
        assert abs(g[i, j] - o) <= 1e-12 * o, (i, j, g[i, j], o)


def test_workload_2000_crop_against_double_oracle(tvs, orc):
    """The 2000 x 2000, 180-sector workload against the double oracle on the 256 x 256 centre crop
    (R23), with horizon flips counted over all 7.2e8 POV-sector pairs against the GPU double
    variant (R22), which itself must equal the oracle on the crop."""
    import torch

    w = WORKLOADS["tvs2000"]
    dem = workload_dem("tvs2000")
    H, W = dem.shape
    args = (w["spacing"], w["obs_height"], w["n_sectors"], w["max_dist"])
    d = torch.from_numpy(dem).cuda()
    note("tvs2000 maps: default, float, double quotient")
    g = tvs.total_viewshed(d, *args).cpu().numpy()
    gx = tvs.total_viewshed(d, *args, flags=F32).cpu().numpy()
    g64 = tvs.total_viewshed(d, *args, flags=F64).cpu().numpy()
    note("tvs2000 flips: default vs double quotient, float vs double quotient")
    flips, pairs, fed = _flip_scan(tvs, orc, d, args, 0, F64)
    flips_x, _, fed_x = _flip_scan(tvs, orc, d, args, F32, F64)
    assert pairs == tvs.los_evals(H, W, w["spacing"], w["n_sectors"], w["max_dist"])[1]
    c = (H - 256) // 2
    note("tvs2000 crop: double oracle on 256 x 256 cells")
    o64 = orc.total(dem, *args, prec=64, window=(c, c, 256, 256))
    sl = (slice(c, c + 256), slice(c, c + 256))
    np.testing.assert_allclose(g64[sl], o64, rtol=1e-12)
    for name, m, fl, fd in (("default", g, flips, fed), ("float", gx, flips_x, fed_x)):
        rel = np.abs(m[sl] - o64) / o64
        clean = ~fd[sl]
        rel_all = np.abs(m - g64) / g64
        print(f"tvs2000 {name}: flips {fl} of {pairs} ({fl / pairs:.2e}); crop max rel {rel.max():.3g}, "
              f"flip-free crop cells max rel {rel[clean].max():.3g}, crop cells fed by flips {int((~clean).sum())}; "
              f"whole map: cells fed by flips {int(fd.sum())}, max rel {rel_all.max():.3g}, "
              f"flip-free max rel {rel_all[~fd].max():.3g}", flush=True)
        # the default meets the bound; the paper's float decision is reported (about 4e-4)
        assert fl / pairs <= (1e-5 if name == "default" else 1e-3)
        if name == "default":
            assert rel.max() <= 1e-4
        assert rel[clean].max() <= 1e-4
        assert rel_all[~fd].max() <= 1e-10


def test_workload_4000_precision_study(tvs, orc):
    """The 4000 x 4000, 5 m, 360-sector workload: float sweep with double accumulation (default),
    with float Kahan accumulation, with the exact float quotient, and the all-double variant; flips
    of each float variant against the double one over every pair, per-cell errors over the whole
    map against the double variant and on the 128 x 128 centre crop against the double oracle."""
    import torch

    w = WORKLOADS["tvs4000"]
    dem = workload_dem("tvs4000")
    H, W = dem.shape
    args = (w["spacing"], w["obs_height"], w["n_sectors"], w["max_dist"])
    d = torch.from_numpy(dem).cuda()
    maps = {}
    for name, fl in (("double quotient", F64), ("default", 0), ("float", F32),
                     ("float, kahan32", F32 | tvs.FLAG_ACC_KAHAN32), ("default, kahan32", tvs.FLAG_ACC_KAHAN32)):
        note(f"tvs4000 map {name}")
        maps[name] = tvs.total_viewshed(d, *args, flags=fl).cpu().numpy()
    note("tvs4000 flips")
    flips, pairs, fed = _flip_scan(tvs, orc, d, args, 0, F64)
    flips_f, _, fed_f = _flip_scan(tvs, orc, d, args, F32, F64)
    c = (H - 128) // 2
    note("tvs4000 crop: double oracle on 128 x 128 cells")
    o64 = orc.total(dem, *args, prec=64, window=(c, c, 128, 128))
    sl = (slice(c, c + 128), slice(c, c + 128))
    g64 = maps["double quotient"]
    np.testing.assert_allclose(g64[sl], o64, rtol=1e-12)
    for name, fd, fl in (("default", fed, flips), ("default, kahan32", fed, flips), ("float", fed_f, flips_f),
                         ("float, kahan32", fed_f, flips_f)):
        m = maps[name]
        rel = np.abs(m - g64) / g64
        relc = np.abs(m[sl] - o64) / o64
        print(f"tvs4000 {name}: flips {fl} of {pairs} ({fl / pairs:.2e}), cells fed by flips {int(fd.sum())}; "
              f"whole map max rel {rel.max():.3g}, flip-free max rel {rel[~fd].max():.3g}, "
              f"p99 rel {np.quantile(rel, 0.99):.3g}; crop vs oracle max rel {relc.max():.3g}", flush=True)
        assert rel[~fd].max() <= (1e-5 if "kahan32" in name else 1e-10)
        assert fl / pairs <= (1e-5 if name.startswith("default") else 1e-2)


@pytest.mark.parametrize("H,W,n,R,pov", [(41, 41, 8, INF, (20, 5)), (64, 80, 36, 300.0, (0, 0)),
                                         (150, 120, 180, 1000.0, (75, 60)), (1, 1, 3, INF, (0, 0)),
                                         (90, 33, 24, 250.0, (89, 32)), (57, 200, 12, INF, (30, 199))])
def test_singular_mask_bitexact(tvs, orc, H, W, n, R, pov):
    """The visibility mask of a singular viewshed equals the oracle's cell by cell, and the area
    equals the plain singular path's."""
    dem = fractal_dem(max(H, W), 23, 0.6, 700.0)[:H, :W].copy()
    note(f"singular mask H={H} W={W} n={n} R={R} pov={pov}")
    area, mask = tvs.singular_mask(dem, 10.0, 1.5, n, R, *pov)
    want = orc.multiple(dem, 10.0, 1.5, n, R, [pov], prec=P_DEFAULT).astype(np.uint8)
    bad = np.argwhere(mask != want)
    assert bad.size == 0, f"{len(bad)} cells differ, first {bad[:5].tolist()}"
    assert area == tvs.singular_viewshed(dem, 10.0, 1.5, n, R, *pov)
    assert area == pytest.approx(orc.singular(dem, 10.0, 1.5, n, R, *pov, prec=P_DEFAULT)["area"], rel=1e-12)


@pytest.mark.parametrize("flags,prec", MODES)
def test_multiple_viewshed_bitexact(tvs, orc, flags, prec):
    dem = fractal_dem(170, 29, 0.6, 900.0)[:150].copy()
    rng = np.random.default_rng(11)
    povs = [(int(rng.integers(0, 150)), int(rng.integers(0, 170))) for _ in range(10)] + [(0, 0), (149, 169)]
    note(f"multiple viewshed flags={flags}")
    cnt, areas = tvs.multiple_viewshed(dem, 10.0, 1.5, 36, 900.0, povs, flags=flags, areas=True)
    want = orc.multiple(dem, 10.0, 1.5, 36, 900.0, povs, prec=prec)
    assert np.array_equal(cnt, want)
    for p, a in zip(povs, areas):
        assert a == pytest.approx(orc.singular(dem, 10.0, 1.5, 36, 900.0, *p, prec=prec)["area"], rel=1e-12)


def test_multiple_viewshed_workload_2000(tvs, orc):
    """Ten random POVs accumulated on the 2000 x 2000 workload (the shape of the paper's GIS
    comparison, Section 5.3): the whole count map against the oracle."""
    import torch

    w = WORKLOADS["tvs2000"]
    dem = workload_dem("tvs2000")
    rng = np.random.default_rng(2020)
    povs = [(int(rng.integers(0, 2000)), int(rng.integers(0, 2000))) for _ in range(10)]
    note("multiple viewshed tvs2000, 10 POVs")
    d = torch.from_numpy(dem).cuda()
    cnt = tvs.multiple_viewshed(d, w["spacing"], w["obs_height"], w["n_sectors"], w["max_dist"], povs)
    torch.cuda.synchronize()
    want = orc.multiple(dem, w["spacing"], w["obs_height"], w["n_sectors"], w["max_dist"], povs, prec=P_DEFAULT)
    got = cnt.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, want)
    print(f"tvs2000 multiple viewshed: {int((want > 0).sum())} cells seen by at least one of 10 POVs", flush=True)
