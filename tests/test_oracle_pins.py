"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names what it pins. The paper prints no per-cell values, so the pins are
hand-derived fixtures (tests/golden), closed forms, brute force, independent plain walks,
symmetries and invariances of the method's definition.
"""
import json
import math
import os

import numpy as np
import pytest

from synth import cone, flat, fractal_dem, plane

GOLD = os.path.join(os.path.dirname(__file__), "golden")
INF = math.inf


def _rand_dem(H, W, seed, lo=0.0, hi=60.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, (H, W)).astype(np.float32)


def _inv_cos2_reduced(k, n):
    """1/cos^2 of the axis angle folded into [0, 45 deg]: 1 + min(|tan a|, |cot a|)^2 (a = k pi / n)."""
    a = k * math.pi / n
    s, c = abs(math.sin(a)), abs(math.cos(a))
    t = min(s, c) / max(s, c)
    return 1.0 + t * t


# ------------------------------------------------------------------ golden fixtures

def test_golden_row5(orc):
    """Hand-derived 1-D example (Alg. 3/8 visibility, Section 3.1 ring areas, clipped last ring)."""
    g = json.load(open(os.path.join(GOLD, "row5.json")))
    dem = np.array(g["dem"], np.float32)
    for case in g["cases"]:
        R = INF if case["max_dist"] == "inf" else float(case["max_dist"])
        tv = orc.total(dem, g["spacing"], g["obs_height"], g["n_sectors"], R)
        np.testing.assert_allclose(tv[0] / (math.pi / 2), case["tvs_over_pi_half"], rtol=1e-13)
        for prec in (32, 33, 65):
            tvp = orc.total(dem, g["spacing"], g["obs_height"], g["n_sectors"], R, prec=prec)
            np.testing.assert_allclose(tvp[0] / (math.pi / 2), case["tvs_over_pi_half"], rtol=1e-13)


def test_golden_grid5(orc):
    """Hand-derived 5x5 example at 0/45/90/135 deg: pins axis orientation, case transforms and 1/cos^2."""
    g = json.load(open(os.path.join(GOLD, "grid5.json")))
    dem = np.array(g["dem"], np.float32)
    for prec in (64, 65, 32, 33):
        tv = orc.total(dem, g["spacing"], g["obs_height"], g["n_sectors"], INF, prec=prec)
        for i, j, v in g["cells_tvs_over_pi"]:
            assert tv[i, j] / math.pi == pytest.approx(v, rel=1e-13)


# ------------------------------------------------------------------ P1/P2: flat terrain

@pytest.mark.parametrize("n", [1, 3, 16, 45])
def test_flat_interior_full_disc(orc, n):
    """P1: on flat ground with h0 > 0 every sample is visible; cells whose lines of sight all
    reach max_dist get exactly the disc area pi R^2."""
    H = W = 60
    dx, R = 10.0, 200.0
    tv = orc.total(flat(H, W, 123.0), dx, 1.5, n, R)
    m = int(math.ceil(R / dx)) + 2
    inner = tv[m:H - m, m:W - m]
    np.testing.assert_allclose(inner, math.pi * R * R, rtol=1e-12)
    # every cell is at most the disc
    assert np.all(tv <= math.pi * R * R * (1 + 1e-12))


def test_flat_unbounded_n1_closed_form(orc):
    """P1, n = 1, unbounded: cell (i, j) of a W-wide flat row sees (W-j)^2 + (j+1)^2 index^2 units."""
    H, W, dx = 3, 17, 10.0
    tv = orc.total(flat(H, W, 5.0), dx, 2.0, 1, INF)
    j = np.arange(W)
    want = (math.pi / 2) * dx * dx * ((W - j) ** 2 + (j + 1) ** 2)
    np.testing.assert_allclose(tv, np.broadcast_to(want, (H, W)), rtol=1e-13)


@pytest.mark.parametrize("n", [2, 7, 12])
def test_flat_zero_height_only_first_ring(orc, n):
    """P2: flat ground seen from h0 = 0: every slope is 0, so only m = 1 beats -inf (strict '>').
    Each direction sums 1 + 3 = 4; interior cells get sum_k 8 (pi/2n) dx^2 / cos^2 s'_k."""
    H = W = 30
    dx, R = 10.0, 100.0
    tv = orc.total(flat(H, W, 50.0), dx, 0.0, n, R)
    want = sum(8.0 * (math.pi / (2 * n)) * dx * dx * _inv_cos2_reduced(k, n) for k in range(n))
    np.testing.assert_allclose(tv[3:-3, 3:-3], want, rtol=1e-12)


@pytest.mark.parametrize("n", [1, 5, 32])
def test_small_radius_any_terrain(orc, n):
    """With max_dist <= spacing no target is ever in range (rho <= 1), so every cell of any terrain
    gets its own rings only: sum_k 2 rho_k^2 scale_k = pi R^2."""
    dem = fractal_dem(24, 7, 0.6, 900.0)
    R = 7.5
    tv = orc.total(dem, 10.0, 1.5, n, R)
    np.testing.assert_allclose(tv, math.pi * R * R, rtol=1e-12)


def _flat_tvs_geometry(H, W, dx, n, R):
    """Flat-ground total viewshed for every cell from geometry alone: all samples are visible,
    so a line of sight with M targets sums min(M+1, rho)^2; M counts the steps whose continuous
    position f = t + (q +- m) tan(s') stays inside (-1, Hx) and the columns; each cell blends the
    skewed samples at f = p + r and f = p - 1 + r with weights 1 - r and r."""
    idx = np.arange(H * W).reshape(H, W)
    out = np.zeros(H * W)
    for k in range(n):
        Xi, sp = _base_frame(idx, k, n)
        T = 0.0 if 4 * k in (0, 2 * n) else (1.0 if 4 * k in (n, 3 * n) else math.tan(sp))
        Hx, Wx = Xi.shape
        rho = R * math.cos(sp) / dx
        scale = (math.pi / (2 * n)) * dx * dx / math.cos(sp) ** 2

        def V(f0, q):
            tot = 0.0
            for delta in (1, -1):
                m = 0
                while True:
                    j = q + delta * (m + 1)
                    f = f0 + delta * (m + 1) * T
                    if not (0 <= j < Wx and -1 < f < Hx and m + 1 < rho):
                        break
                    m += 1
                tot += min(m + 1.0, rho) ** 2
            return tot

        for p in range(Hx):
            for q in range(Wx):
                y = q * T
                r = y - math.floor(y)
                val = (1 - r) * V(p + r, q) + (r * V(p - 1 + r, q) if r > 0 else 0.0)
                out[Xi[p, q]] += scale * val
    return out.reshape(H, W)


@pytest.mark.parametrize("n,R", [(12, 75.0), (9, INF), (20, 42.0)])
def test_flat_every_cell_from_geometry(orc, n, R):
    """P1, whole grid: edges, clipped rows and the two-sample blend of Alg. 9 on flat ground
    match the geometric closed form (pins sample existence in (-1, Hx) and the blend weights)."""
    H, W, dx = 14, 19, 10.0
    tv = orc.total(flat(H, W, 7.0), dx, 1.5, n, R)
    np.testing.assert_allclose(tv, _flat_tvs_geometry(H, W, dx, n, R), rtol=1e-9)


@pytest.mark.parametrize("R", [60.0, 65.0, 10.0])
def test_clipped_ring_split(orc, R):
    """The ring sum splits into whole rings U and e clipped last rings of area rho^2 - K^2,
    K = ceil(rho) - 1: flat interior samples have U = 2 K^2 and e = 2 (ring K is visible both
    ways), so U + e (rho^2 - K^2) = 2 rho^2, also when rho is an integer."""
    dx = 10.0
    rho = R / dx
    K = math.ceil(rho) - 1
    sv = orc.sector_V(flat(5, 40, 3.0), dx, 1.5, 1, R, 0)
    assert sv["K"] == K
    mid = sv["U"][3, 15:25]  # row t = 2, columns far from both ends
    assert np.all(mid == 2 * K * K)
    assert np.all(sv["e"][3, 15:25] == 2)
    dem = fractal_dem(30, 4, 0.6, 200.0)
    for k in (0, 3):
        sv = orc.sector_V(dem, dx, 1.5, 7, R, k)
        v = sv["valid"].astype(bool)
        np.testing.assert_allclose((sv["U"] + sv["e"] * (sv["rho"] ** 2 - sv["K"] ** 2))[v], sv["cv"][v],
                                   rtol=1e-13)


# ------------------------------------------------------------------ P3: tilted plane

@pytest.mark.parametrize("prec", [64, 32, 33])
@pytest.mark.parametrize("n", [7, 12])
def test_tilted_plane_interior_full_disc(orc, n, prec):
    """P3: interpolated samples of a plane lie on the plane, so all are visible. A wrong
    interpolation weight or skew direction makes samples wobble off the line and hides some."""
    H = W = 50
    dx, R = 10.0, 150.0
    dem = plane(H, W, 0.75, -0.5, 300.0)
    tv = orc.total(dem, dx, 1.5, n, R, prec=prec)
    m = int(math.ceil(R / dx)) + 2
    np.testing.assert_allclose(tv[m:H - m, m:W - m], math.pi * R * R, rtol=1e-12)


# ------------------------------------------------------------------ P4: 0 and 90 deg are plain walks

def _plain_walk(z, j0, h, delta, rho):
    cv = min(1.0, rho) ** 2
    mx = -INF
    m = 1
    while 0 <= j0 + delta * m < len(z) and m < rho:
        th = (float(z[j0 + delta * m]) - h) / m
        if th > mx:
            cv += min(m + 1.0, rho) ** 2 - m * m
            mx = th
        m += 1
    return cv


@pytest.mark.parametrize("R", [INF, 45.0, 61.0])
def test_n1_n2_equal_row_and_column_walks(orc, R):
    """P4: the 0 deg axis is a plain walk along grid rows and the 90 deg axis a plain walk
    along grid columns (no skew, no interpolation)."""
    H, W, dx, h0 = 9, 12, 10.0, 1.5
    dem = np.round(_rand_dem(H, W, 3, 0, 40)).astype(np.float32)
    rho = R / dx
    rows = np.zeros((H, W))
    cols = np.zeros((H, W))
    for i in range(H):
        for j in range(W):
            h = float(dem[i, j]) + h0
            rows[i, j] = _plain_walk(dem[i, :], j, h, 1, rho) + _plain_walk(dem[i, :], j, h, -1, rho)
            cols[i, j] = _plain_walk(dem[:, j], i, h, 1, rho) + _plain_walk(dem[:, j], i, h, -1, rho)
    t1 = orc.total(dem, dx, h0, 1, R)
    np.testing.assert_allclose(t1, (math.pi / 2) * dx * dx * rows, rtol=1e-13)
    t2 = orc.total(dem, dx, h0, 2, R)
    np.testing.assert_allclose(t2, (math.pi / 4) * dx * dx * (rows + cols), rtol=1e-13)


# ------------------------------------------------------------------ P5: singular == total at n = 4

@pytest.mark.parametrize("prec", [64, 65, 32, 33])
def test_n4_singular_equals_total(orc, prec):
    """P5: at 0/45/90/135 deg every skew weight is 0, so the two skewed POVs a cell blends
    collapse to the cell itself and the total viewshed equals the singular one exactly."""
    dem = fractal_dem(17, 11, 0.6, 500.0)[:, :13].copy()
    H, W = dem.shape
    tv = orc.total(dem, 10.0, 1.5, 4, INF, prec=prec)
    for i in range(H):
        for j in range(W):
            s = orc.singular(dem, 10.0, 1.5, 4, INF, i, j, prec=prec)
            assert s["area"] == tv[i, j]


def test_singular_close_to_total_on_smooth_terrain(orc):
    """Away from n = 4 the singular line of sight passes through the POV while the total
    viewshed blends the two straddling skewed POVs; on smooth terrain the two stay close."""
    dem = plane(40, 40, 0.5, 0.25, 100.0)
    tv = orc.total(dem, 10.0, 1.5, 24, 120.0, window=(15, 15, 10, 10))
    for a in range(0, 10, 3):
        for b in range(0, 10, 3):
            s = orc.singular(dem, 10.0, 1.5, 24, 120.0, 15 + a, 15 + b)
            assert s["area"] == pytest.approx(tv[a, b], rel=1e-12)


# ------------------------------------------------------------------ P6: brute force per pair

@pytest.mark.parametrize("prec", [64, 65, 32, 33])
def test_running_max_equals_brute_force(orc, prec):
    """P6: 'visible iff the slope beats the running maximum' equals the O(M^2) definition
    'visible iff every earlier slope is strictly smaller', and the ring sum follows from it."""
    rng = np.random.default_rng(5)
    checked = 0
    for trial in range(12):
        H, W = int(rng.integers(1, 15)), int(rng.integers(1, 15))
        dem = np.round(rng.uniform(0, 8, (H, W))).astype(np.float32)  # many exact ties
        n = int(rng.integers(1, 17))
        R = INF if trial % 3 == 0 else float(rng.uniform(5, 150))
        dx, h0 = 10.0, float(rng.choice([0.0, 1.5, 4.0]))
        for k in range(n):
            info = orc.sector_info(H, W, dx, n, R, k)
            sv = orc.sector_V(dem, dx, h0, n, R, k, prec=prec)
            for ti in range(info["nrows"]):
                for q in range(info["Wx"]):
                    if not sv["valid"][ti, q]:
                        continue
                    t = info["t0"] + ti
                    tot = 0.0
                    for delta in (1, -1):
                        r = orc.ray(dem, dx, h0, n, R, k, 0, t, q, delta, prec=prec)
                        th = r["theta"]
                        brute = np.array([np.all(th[:m] < th[m]) for m in range(r["M"])], bool)
                        assert np.array_equal(brute, r["vis"])
                        rho = info["rho"]
                        cv = min(1.0, rho) ** 2 + sum(min(m + 2.0, rho) ** 2 - (m + 1.0) ** 2
                                                      for m in range(r["M"]) if brute[m])
                        assert cv == pytest.approx(r["cv"], rel=1e-14)
                        tot += cv
                        checked += 1
                    assert tot == pytest.approx(sv["cv"][ti, q], rel=1e-14)
    assert checked > 500


# ------------------------------------------------------------------ P7: independent ray geometry

def _base_frame(dem, k, n):
    """Independent construction of the 0..45 deg base frame by the axis direction's octant."""
    if 4 * k <= n:
        return dem, k * math.pi / n
    if 4 * k <= 2 * n:
        return dem.T, math.pi / 2 - k * math.pi / n
    if 4 * k < 3 * n:
        return np.flipud(dem.T), k * math.pi / n - math.pi / 2
    return np.fliplr(dem), math.pi - k * math.pi / n


def _lerp_col(X, f, j):
    Hx = X.shape[0]
    fl = math.floor(f)
    fr = f - fl
    a = float(X[min(max(fl, 0), Hx - 1), j])
    b = float(X[min(max(fl + 1, 0), Hx - 1), j])
    return (1 - fr) * a + fr * b


@pytest.mark.parametrize("n", [3, 5, 8, 13])
def test_skewed_samples_lie_on_straight_lines(orc, n):
    """P7: the elevations the oracle reads along a skewed row equal a direct interpolation of
    the base frame at f = f0 + (j - j0) tan(s'), for both the total (skewed row) and the
    singular (through the POV) lines of sight."""
    H, W = 11, 14
    dem = _rand_dem(H, W, 9, 0, 300)
    dx = 10.0
    for k in range(n):
        X, sp = _base_frame(dem, k, n)
        T = math.tan(sp)
        info = orc.sector_info(H, W, dx, n, INF, k)
        for t in range(info["t0"], info["t0"] + info["nrows"], 2):
            for q0 in range(0, info["Wx"], 3):
                f0 = t + q0 * T
                if not (-1 < f0 < info["Hx"]):
                    continue
                for delta in (1, -1):
                    try:
                        r = orc.ray(dem, dx, 1.0, n, INF, k, 0, t, q0, delta)
                    except ValueError:
                        continue  # POV on the snapping edge of the grid; skip
                    for m in range(r["M"]):
                        j = q0 + delta * (m + 1)
                        f = f0 + delta * (m + 1) * T
                        assert r["z"][m] == pytest.approx(_lerp_col(X, f, j), abs=1e-6)
        # singular rays through grid cells
        for p0 in range(0, info["Hx"], 4):
            for q0 in range(0, info["Wx"], 5):
                for delta in (1, -1):
                    r = orc.ray(dem, dx, 1.0, n, INF, k, 1, p0, q0, delta)
                    for m in range(r["M"]):
                        j = q0 + delta * (m + 1)
                        f = p0 + delta * (m + 1) * T
                        assert r["z"][m] == pytest.approx(_lerp_col(X, f, j), abs=1e-6)


# ------------------------------------------------------------------ P8/P9: symmetries

@pytest.mark.parametrize("prec", [32, 33, 64, 65])
@pytest.mark.parametrize("n", [4, 7, 10])
def test_mirror_pairs_agree_exactly(orc, n, prec):
    """P8: mirroring the grid left-right maps axis k to axis (n - k) mod n. For 0 < k, k != n/2
    the two base frames are the same array, so per-sector results agree bit for bit. The
    self-paired axes 0 and 90 deg (no skew) see a mirrored base frame: at 0 deg every row is
    reversed (forward and backward swap), at 90 deg the row order is reversed. The maps agree
    to rounding."""
    dem = fractal_dem(19, 13, 0.6, 700.0)[:, :15].copy()
    mir = np.ascontiguousarray(np.fliplr(dem))
    for k in range(n):
        a = orc.sector_V(dem, 10.0, 1.5, n, 90.0, k, prec=prec)
        b = orc.sector_V(mir, 10.0, 1.5, n, 90.0, (n - k) % n, prec=prec)
        for key in ("U", "e", "valid"):
            if k == 0:
                assert np.array_equal(a[key], b[key][:, ::-1])
            elif 2 * k == n:
                assert not a[key][0].any() and not b[key][0].any()
                assert np.array_equal(a[key][1:], b[key][1:][::-1])
            else:
                assert np.array_equal(a[key], b[key])
    ta = orc.total(dem, 10.0, 1.5, n, 90.0)
    tb = orc.total(mir, 10.0, 1.5, n, 90.0)
    np.testing.assert_allclose(np.fliplr(tb), ta, rtol=1e-13)


def test_transpose_approximately_symmetric(orc):
    """P9 (smoke only): transposing the grid is a symmetry of the continuous problem but not
    of the column-0-anchored skew; the maps agree on average within a few percent."""
    dem = fractal_dem(33, 17, 0.5, 600.0)
    ta = orc.total(dem, 10.0, 1.5, 36, 200.0)
    tb = orc.total(np.ascontiguousarray(dem.T), 10.0, 1.5, 36, 200.0).T
    rel = np.abs(ta - tb) / ta
    assert rel.mean() < 0.05


# ------------------------------------------------------------------ P10: invariances

def test_scaling_invariance_exact(orc):
    """P10: scaling elevations and observer height by 2 scales every slope by 2 exactly."""
    dem = fractal_dem(21, 17, 0.6, 400.0)
    a = orc.total(dem, 10.0, 1.5, 9, 130.0)
    b = orc.total((dem * 2).astype(np.float32), 10.0, 3.0, 9, 130.0)
    assert np.array_equal(a, b)


def test_offset_invariance_on_grid_axes(orc):
    """P10: adding a constant to the terrain changes nothing (exact where no interpolation)."""
    dem = np.round(_rand_dem(13, 11, 2, 0, 100)).astype(np.float32)
    a = orc.total(dem, 10.0, 1.5, 4, INF)
    b = orc.total(dem + np.float32(1024.0), 10.0, 1.5, 4, INF)
    assert np.array_equal(a, b)


def test_monotone_in_observer_height(orc):
    """P10: raising the observer never hides a target, so every cell is non-decreasing in h0."""
    dem = fractal_dem(20, 23, 0.6, 300.0)
    lo = orc.total(dem, 10.0, 0.5, 12, INF)
    hi = orc.total(dem, 10.0, 5.0, 12, INF)
    assert np.all(hi >= lo * (1 - 1e-13))
    assert np.any(hi > lo * 1.01)


# ------------------------------------------------------------------ P11: 1-D analytic profiles

def test_pillar_shadow_and_reappearance(orc):
    """P11: a pillar lower than the eye hides targets until their slope -h0/m beats the pillar's
    (P-h0)/a; the tie at m = h0 a / (h0 - P) = 10 stays hidden (strict comparison)."""
    W = 21
    z = np.zeros((1, W), np.float32)
    z[0, 5] = 0.5
    r = orc.ray(z, 1.0, 1.0, 1, INF, 0, 0, 0, 0, 1)
    vis = np.flatnonzero(r["vis"]) + 1
    assert list(vis) == [1, 2, 3, 4, 5] + list(range(11, W))
    assert r["cv"] == 36 + (W ** 2 - 11 ** 2)
    z[0, 5] = 3.0  # higher than the eye: nothing behind it is visible
    r = orc.ray(z, 1.0, 1.0, 1, INF, 0, 0, 0, 0, 1)
    assert r["cv"] == 36


def test_dome_and_bowl(orc):
    """P11: on a dome z = -c m^2 the slope -c m - h0/m peaks at m = sqrt(h0/c) = 10, so
    targets 1..10 are visible; on a bowl every target is visible."""
    W = 31
    m = np.arange(W, dtype=np.float64)
    dome = (-0.01 * m * m).astype(np.float32)[None, :]
    r = orc.ray(dome, 1.0, 1.0, 1, INF, 0, 0, 0, 0, 1)
    assert r["cv"] == 11 ** 2
    bowl = (0.01 * m * m).astype(np.float32)[None, :]
    r = orc.ray(bowl, 1.0, 1.0, 1, INF, 0, 0, 0, 0, 1)
    assert r["cv"] == W ** 2


# ------------------------------------------------------------------ P12: cone peak

def test_cone_shadow_boundary(orc):
    """P12: POV on flat ground looking at a cone apex D >= 2 Rc away along an axis: the rising
    flank and the apex are visible, everything behind the apex is hidden, so the forward ring
    sum is (D+1)^2, at 0 deg and, through grid diagonals, at 45 and 135 deg."""
    D = 50
    dem = cone(41, 81, 20, 60, 30.0, 8.0)
    r = orc.ray(dem, 10.0, 1.5, 1, INF, 0, 0, 20, 10, 1)
    assert r["cv"] == (D + 1) ** 2
    dem = cone(81, 81, 60, 60, 30.0, 8.0)
    s = orc.singular(dem, 10.0, 1.5, 4, INF, 10, 10)
    assert s["cv"][2 * 1] == (D + 1) ** 2          # 45 deg forward: +row, +col
    dem = cone(81, 81, 60, 20, 30.0, 8.0)
    s = orc.singular(dem, 10.0, 1.5, 4, INF, 10, 70)
    assert s["cv"][2 * 3] == (D + 1) ** 2          # 135 deg forward: +row, -col
    # and the same cone is not on the 45 deg line from there: flat, all visible
    assert s["cv"][2 * 1] == (min(81 - 10, 81 - 70)) ** 2


# ------------------------------------------------------------------ counts, edges, precision

def test_los_eval_count_closed_forms(orc):
    """LoS cell-evaluations: n = 1 unbounded is H * W (W - 1); n = 2 adds W * H (H - 1);
    bounded n = 1 is H * 2 sum_q min(q, K)."""
    H, W = 13, 29
    assert orc.los_evals(H, W, 10.0, 1, INF)[0] == H * W * (W - 1)
    assert orc.los_evals(H, W, 10.0, 2, INF)[0] == H * W * (W - 1) + W * H * (H - 1)
    K = 6  # R = 65 m, dx = 10 -> rho = 6.5
    assert orc.los_evals(H, W, 10.0, 1, 65.0)[0] == H * 2 * sum(min(q, K) for q in range(W))
    assert orc.los_evals(H, W, 10.0, 1, INF)[1] == H * W


def test_single_cell_grid(orc):
    """Degenerate grid: a single cell has no targets in any direction, so it sees its own
    rings only: sum_k 2 scale_k (rho >= 1)."""
    n, dx = 6, 10.0
    tv = orc.total(np.array([[42.0]], np.float32), dx, 1.5, n, INF)
    want = sum(2 * (math.pi / (2 * n)) * dx * dx * _inv_cos2_reduced(k, n) for k in range(n))
    assert tv[0, 0] == pytest.approx(want, rel=1e-13)


def test_rejects_bad_input(orc):
    d = np.zeros((4, 4), np.float32)
    with pytest.raises(ValueError):
        orc.total(d, 0.0, 1.5, 4, INF)
    with pytest.raises(ValueError):
        orc.total(d, 10.0, 1.5, 0, INF)
    with pytest.raises(ValueError):
        orc.total(d, 10.0, 1.5, 4, -1.0)
    with pytest.raises(ValueError):
        orc.total(d, 10.0, 1.5, 4, math.nan)
    bad = d.copy()
    bad[1, 2] = np.nan
    with pytest.raises(ValueError):
        orc.total(bad, 10.0, 1.5, 4, INF)


@pytest.mark.parametrize("prec", [32, 33])
def test_fp32_decisions_rarely_differ_from_fp64(orc, prec):
    """The single-precision visibility decision (the paper's float kernels) differs from the
    double one only at near-ties; on fractal terrain such horizon flips are rare."""
    dem = fractal_dem(64, 1, 0.6, 1500.0)
    flips = pairs = 0
    for k in (0, 17, 45, 62, 90, 133, 170):
        a = orc.sector_V(dem, 10.0, 1.5, 180, 640.0, k, prec=64)
        b = orc.sector_V(dem, 10.0, 1.5, 180, 640.0, k, prec=prec)
        v = a["valid"].astype(bool)
        pairs += int(v.sum())
        flips += int(np.sum((a["U"] != b["U"])[v] | (a["e"] != b["e"])[v]))
    assert pairs > 20000
    assert flips / pairs < 1e-3


def test_reciprocal_slope_within_one_ulp_of_quotient(orc):
    """prec 33 forms the float slope as the difference times the float reciprocal of m; on a
    ray its slopes lie within one float ulp of prec 32's correctly rounded quotients."""
    dem = fractal_dem(40, 8, 0.6, 900.0)
    for k in (0, 3, 7):
        a = orc.ray(dem, 10.0, 1.5, 12, INF, k, 0, 5, 2, 1, prec=32)
        b = orc.ray(dem, 10.0, 1.5, 12, INF, k, 0, 5, 2, 1, prec=33)
        ta = a["theta"].astype(np.float32)
        tb = b["theta"].astype(np.float32)
        assert a["M"] == b["M"] > 10
        assert np.all(np.abs(ta.view(np.int32) - tb.view(np.int32)) <= 1)


def test_double_reciprocal_slope_within_one_ulp_of_quotient(orc):
    """prec 65 forms the double slope as the difference times the double reciprocal of m; on a
    ray its slopes lie within one double ulp of prec 64's correctly rounded quotients (a float
    reciprocal, or a float difference, would be off by about 2^29 ulps)."""
    dem = fractal_dem(40, 8, 0.6, 900.0)
    for k in (0, 3, 7):
        a = orc.ray(dem, 10.0, 1.5, 12, INF, k, 0, 5, 2, 1, prec=64)
        b = orc.ray(dem, 10.0, 1.5, 12, INF, k, 0, 5, 2, 1, prec=65)
        assert a["M"] == b["M"] > 10
        assert np.all(np.abs(a["theta"].view(np.int64) - b["theta"].view(np.int64)) <= 1)
        assert np.any(a["theta"] != b["theta"])  # the two forms do differ somewhere


def test_double_reciprocal_decisions_match_quotient(orc):
    """Deciding in double with the reciprocal product agrees with the double quotient on every
    POV-sector pair of a fractal grid (a one-ulp double difference almost never decides a tie)."""
    dem = fractal_dem(64, 1, 0.6, 1500.0)
    pairs = 0
    for k in (0, 17, 45, 62, 90, 133, 170):
        a = orc.sector_V(dem, 10.0, 1.5, 180, 640.0, k, prec=64)
        b = orc.sector_V(dem, 10.0, 1.5, 180, 640.0, k, prec=65)
        v = a["valid"].astype(bool)
        pairs += int(v.sum())
        assert np.array_equal(a["U"], b["U"]) and np.array_equal(a["e"], b["e"])
    assert pairs > 20000


def test_double_reciprocal_decisions_match_quotient_whole_workload(orc):
    """The same on every one of the 180 sectors of the 128x128 workload (seed 1, 0-1500 m, 10 m,
    1.5 m, max distance 1280 m): 2.97e6 POV-sector pairs, not one decision differs."""
    from synth import WORKLOADS, workload_dem

    w = WORKLOADS["tvs128"]
    dem = workload_dem("tvs128")
    pairs = 0
    for k in range(w["n_sectors"]):
        a = orc.sector_V(dem, w["spacing"], w["obs_height"], w["n_sectors"], w["max_dist"], k, prec=64)
        b = orc.sector_V(dem, w["spacing"], w["obs_height"], w["n_sectors"], w["max_dist"], k, prec=65)
        pairs += int(a["valid"].astype(bool).sum())
        assert np.array_equal(a["U"], b["U"]) and np.array_equal(a["e"], b["e"]), f"sector {k}"
    assert pairs == 2971472


# ------------------------------------------------------------------ singular mask and multiple viewshed

@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 12, 180])
def test_half_sector_is_the_nearest_axis(orc, n):
    """Each cell offset is assigned the half-sector whose axis direction q pi / n (q >= n: the
    backward axes) is nearest to it: within half a sector, and the only one when not on a
    boundary (an independent nearest-axis reading of the assignment)."""
    for di in range(-23, 24):
        for dj in range(-23, 24):
            if di == 0 and dj == 0:
                assert orc.half_sector(n, di, dj) == -1
                continue
            q = orc.half_sector(n, di, dj)
            assert 0 <= q < 2 * n
            phi = math.atan2(di, dj) % (2 * math.pi)
            dist = [abs((phi - x * math.pi / n + math.pi) % (2 * math.pi) - math.pi) for x in range(2 * n)]
            half = math.pi / (2 * n)
            assert dist[q] <= half + 1e-12
            if dist[q] < half - 1e-9:
                assert min(d for x, d in enumerate(dist) if x != q) > half


def test_mask_flat_disc(orc):
    """Flat ground, observer above it: every target is visible, so the mask is the disc of ring
    indices below rho: all cells nearer than R - 1 cell are visible, none farther than
    R / cos(pi / 2n) + 1 cells, and the count is close to pi R^2."""
    dem = flat(81, 81, 25.0)
    n, R = 36, 300.0
    m = orc.multiple(dem, 10.0, 1.5, n, R, [(40, 40)]).astype(bool)
    ii, jj = np.mgrid[0:81, 0:81]
    d = np.hypot(ii - 40, jj - 40)
    assert m[d < R / 10.0 - 1].all()
    assert not m[d > R / 10.0 / math.cos(math.pi / (2 * n)) + 1].any()
    assert abs(m.sum() - math.pi * 30.0 ** 2) < 0.05 * math.pi * 30.0 ** 2


def test_mask_wall_shadow(orc):
    """A tall wall across the line of sight at 0 deg hides every cell behind it on that line and
    nothing in front of it or on the other side."""
    dem = flat(41, 41, 0.0)
    dem[15:26, 10] = 100.0
    m = orc.multiple(dem, 10.0, 1.5, 8, INF, [(20, 5)]).astype(bool)
    assert m[20, :11].all()      # up to and including the wall
    assert not m[20, 11:].any()  # behind it
    assert m[20, 5] and m[5:36, 5].all()


def test_mask_on_axis_cells_follow_the_ray(orc):
    """Cells on the axis directions of n = 4 (0, 45, 90, 135 deg and backward) take the visibility
    of the ray target at their index, read through the independent per-ray walk."""
    dem = fractal_dem(33, 12, 0.6, 400.0)
    i0, j0 = 14, 17
    n = 4
    mask = orc.multiple(dem, 10.0, 1.5, n, INF, [(i0, j0)]).astype(bool)
    dirs = {0: (0, 1), 1: (1, 1), 2: (1, 0), 3: (1, -1)}
    for k, (si, sj) in dirs.items():
        for delta in (1, -1):
            info = orc.sector_info(33, 33, 10.0, n, INF, k)
            # the singular ray of sector k through the POV, in its base frame
            if info["case"] == 0:
                p0, q0 = i0, j0
            elif info["case"] == 1:
                p0, q0 = j0, i0
            elif info["case"] == 2:
                p0, q0 = 33 - 1 - j0, i0
            else:
                p0, q0 = i0, 33 - 1 - j0
            r = orc.ray(dem, 10.0, 1.5, n, INF, k, 1, p0, q0, delta)
            for m in range(1, r["M"] + 1):
                # axis k points at k pi / n from +column toward +row
                i, j = i0 + delta * si * m, j0 + delta * sj * m
                if 0 <= i < 33 and 0 <= j < 33:
                    assert mask[i, j] == r["vis"][m - 1], (k, delta, m)


def test_multiple_is_the_sum_of_masks(orc):
    dem = fractal_dem(40, 4, 0.6, 600.0)[:37].copy()
    povs = [(3, 4), (20, 20), (36, 0), (0, 39), (20, 20)]
    tot = orc.multiple(dem, 10.0, 2.0, 24, 250.0, povs)
    acc = sum(orc.multiple(dem, 10.0, 2.0, 24, 250.0, [p]).astype(np.int64) for p in povs)
    assert np.array_equal(tot, acc)
    assert tot[20, 20] == 2 and tot.max() <= len(povs)
