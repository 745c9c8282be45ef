"""Seeded synthetic elevation models shared by the oracle tests, the GPU tests and the bench.

This module only makes input grids. It holds none of the viewshed arithmetic, so the
oracle and the GPU path can both take their inputs from it without sharing any code
of the method itself.

The paper's experiments use three 10 m DEMs of the Montes de Malaga Natural Park
(2000x2000, 4000x4000, 8000x8000; Section 5.1, Table 2). Those grids are not available,
so seeded fractal terrain of the same shapes and spacing stands in for them:

* ``diamond_square``: the classic midpoint-displacement fractal on a (2^m+1)^2 grid,
  cropped to the requested side and min-max normalised to [zmin, zmax] metres.
* ``add_ridges``: Gaussian ridges along random straight lines, for the rugged
  precision-study terrain.
* ``flat``, ``plane``, ``cone``, ``pillar_row``, ``dome_row``: analytic grids with
  closed-form visibility, used as pins.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "diamond_square",
    "add_ridges",
    "fractal_dem",
    "ridged_dem",
    "flat",
    "plane",
    "cone",
    "workload_dem",
    "WORKLOADS",
    "batch_workload",
    "BATCH64",
]


def _square_points(g: np.ndarray, step: int, half: int, ii: np.ndarray, jj: np.ndarray) -> tuple:
    """Mean of the in-range axis neighbours at distance ``half`` for the points ii x jj."""
    n = g.shape[0]
    I, J = np.meshgrid(ii, jj, indexing="ij")
    acc = np.zeros(I.shape, dtype=np.float64)
    cnt = np.zeros(I.shape, dtype=np.float64)
    for di, dj in ((-half, 0), (half, 0), (0, -half), (0, half)):
        I2 = I + di
        J2 = J + dj
        ok = (I2 >= 0) & (I2 < n) & (J2 >= 0) & (J2 < n)
        acc[ok] += g[I2[ok], J2[ok]]
        cnt[ok] += 1.0
    return I, J, acc / cnt


def diamond_square(side: int, seed: int, roughness: float, zmin: float, zmax: float) -> np.ndarray:
    """Seeded diamond-square terrain, ``side x side`` float32 metres in [zmin, zmax].

    Corners are U(0,1); every level adds U(-a, a) displacements with ``a`` starting
    at 1 and multiplied by ``roughness`` per level. Random numbers are drawn with
    ``numpy.random.default_rng(seed)`` in a fixed order (corners, then per level the
    diamond centres, the row-aligned edge midpoints, the column-aligned edge midpoints).
    """
    if side < 1:
        raise ValueError("side must be >= 1")
    m = max(1, math.ceil(math.log2(max(side - 1, 1))))
    size = (1 << m) + 1
    rng = np.random.default_rng(seed)
    g = np.zeros((size, size), dtype=np.float64)
    c = rng.uniform(0.0, 1.0, 4)
    g[0, 0], g[0, -1], g[-1, 0], g[-1, -1] = c
    step = size - 1
    a = 1.0
    while step > 1:
        half = step // 2
        centre = (
            g[0:-1:step, 0:-1:step]
            + g[0:-1:step, step::step]
            + g[step::step, 0:-1:step]
            + g[step::step, step::step]
        ) * 0.25
        g[half::step, half::step] = centre + rng.uniform(-a, a, centre.shape)
        IA, JA, va = _square_points(g, step, half, np.arange(0, size, step), np.arange(half, size, step))
        IB, JB, vb = _square_points(g, step, half, np.arange(half, size, step), np.arange(0, size, step))
        g[IA, JA] = va + rng.uniform(-a, a, va.shape)
        g[IB, JB] = vb + rng.uniform(-a, a, vb.shape)
        a *= roughness
        step = half
    g = g[:side, :side]
    return _normalise(g, zmin, zmax)


def _normalise(g: np.ndarray, zmin: float, zmax: float) -> np.ndarray:
    lo = float(g.min())
    hi = float(g.max())
    if hi > lo:
        out = zmin + (g - lo) * ((zmax - zmin) / (hi - lo))
    else:
        out = np.full(g.shape, zmin, dtype=np.float64)
    return np.ascontiguousarray(out.astype(np.float32))


def add_ridges(dem: np.ndarray, spacing: float, count: int, sigma_m: float, amp_lo: float, amp_hi: float,
               seed: int, zmin: float, zmax: float) -> np.ndarray:
    """Add ``count`` Gaussian ridges ``A*exp(-d^2/(2 sigma^2))`` along random lines, then renormalise.

    Each ridge is a line through a uniform random point with a uniform random direction;
    ``A`` is U(amp_lo, amp_hi) times the current elevation range; ``d`` is the distance in
    metres from a cell centre to the line.
    """
    H, W = dem.shape
    rng = np.random.default_rng(seed)
    z = dem.astype(np.float64)
    rng_range = float(z.max() - z.min()) or 1.0
    ii, jj = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    for _ in range(count):
        pi = rng.uniform(0, H)
        pj = rng.uniform(0, W)
        phi = rng.uniform(0, math.pi)
        amp = rng.uniform(amp_lo, amp_hi) * rng_range
        # distance from (i, j) to the line through (pi, pj) with direction (sin phi, cos phi), in metres
        d = np.abs((ii - pi) * math.cos(phi) - (jj - pj) * math.sin(phi)) * spacing
        z += amp * np.exp(-(d * d) / (2.0 * sigma_m * sigma_m))
    return _normalise(z, zmin, zmax)


def fractal_dem(side: int, seed: int, roughness: float, zmax: float, zmin: float = 0.0) -> np.ndarray:
    return diamond_square(side, seed, roughness, zmin, zmax)


def ridged_dem(side: int, seed: int, roughness: float, spacing: float, ridge_seed: int,
               zmax: float = 3000.0) -> np.ndarray:
    base = diamond_square(side, seed, roughness, 0.0, zmax)
    return add_ridges(base, spacing, count=6, sigma_m=200.0, amp_lo=0.3, amp_hi=0.6,
                      seed=ridge_seed, zmin=0.0, zmax=zmax)


def flat(H: int, W: int, z: float = 100.0) -> np.ndarray:
    return np.full((H, W), z, dtype=np.float32)


def plane(H: int, W: int, alpha: float, beta: float, gamma: float) -> np.ndarray:
    """z = alpha*i + beta*j + gamma (pick dyadic coefficients so float32 holds it exactly)."""
    ii, jj = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    return np.ascontiguousarray((alpha * ii + beta * jj + gamma).astype(np.float32))


def cone(H: int, W: int, ci: int, cj: int, height: float, radius_cells: float, base: float = 0.0) -> np.ndarray:
    """Flat ground at ``base`` with a right circular cone of ``height`` centred on cell (ci, cj)."""
    ii, jj = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    r = np.sqrt((ii - ci) ** 2 + (jj - cj) ** 2)
    z = base + np.where(r < radius_cells, height * (1.0 - r / radius_cells), 0.0)
    return np.ascontiguousarray(z.astype(np.float32))


# Workloads shaped like the paper's experiments (Section 5, Table 2): side, spacing (m),
# observer height (m), sectors over 180 degrees, max distance (m, inf = unbounded).
WORKLOADS = {
    # 128x128 fractal, 0-1500 m, 10 m, 1.5 m, 180 sectors, max distance = extent (1280 m)
    "tvs128": dict(side=128, seed=1, roughness=0.6, zmax=1500.0, spacing=10.0, obs_height=1.5,
                   n_sectors=180, max_dist=1280.0),
    # 2000x2000 fractal, 0-2500 m, 10 m, 1.5 m, 180 sectors, 10 km
    "tvs2000": dict(side=2000, seed=2, roughness=0.55, zmax=2500.0, spacing=10.0, obs_height=1.5,
                    n_sectors=180, max_dist=10000.0),
    # 4000x4000 fractal + 6 Gaussian ridges, 0-3000 m, 5 m, 1.5 m, 360 sectors, 10 km
    "tvs4000": dict(side=4000, seed=3, roughness=0.55, zmax=3000.0, spacing=5.0, obs_height=1.5,
                    n_sectors=360, max_dist=10000.0, ridge_seed=33),
    # 8000x8000 fractal, 0-3000 m, 10 m, 1.5 m, 180 sectors, 10 km (the largest grid shape of Table 2)
    "tvs8000": dict(side=8000, seed=6, roughness=0.55, zmax=3000.0, spacing=10.0, obs_height=1.5,
                    n_sectors=180, max_dist=10000.0),
}


def workload_dem(name: str) -> np.ndarray:
    w = WORKLOADS[name]
    if "ridge_seed" in w:
        return ridged_dem(w["side"], w["seed"], w["roughness"], w["spacing"], w["ridge_seed"], w["zmax"])
    return fractal_dem(w["side"], w["seed"], w["roughness"], w["zmax"])


# A batch of independent tiles of uneven size: square fractal tiles (roughness 0.55, 0-2500 m)
# with sides drawn uniformly from [side_lo, side_hi], 10 m spacing, observer heights uniform in
# [1.5, 30] m, max distance = tile extent; tile i uses terrain seed 4000 + i.
BATCH64 = dict(ntiles=64, seed=4, side_lo=256, side_hi=2048, roughness=0.55, zmax=2500.0, spacing=10.0,
               h_lo=1.5, h_hi=30.0, n_sectors=180)


def _batch_tile(args):
    side, i = args
    return fractal_dem(side, 4000 + i, BATCH64["roughness"], BATCH64["zmax"])


def batch_workload(ntiles: int = 64, seed: int = 4, side_lo: int = 256, side_hi: int = 2048,
                   workers: int = 1) -> list:
    """List of dicts (dem, spacing, obs_height, max_dist) for a batch of tiles. Each tile's terrain
    depends only on its index, so ``workers`` > 1 generates them in that many processes with the
    same result."""
    w = BATCH64
    rng = np.random.default_rng(seed)
    sides = rng.integers(side_lo, side_hi + 1, ntiles)
    heights = rng.uniform(w["h_lo"], w["h_hi"], ntiles)
    jobs = [(int(sides[i]), i) for i in range(ntiles)]
    if workers > 1:
        from concurrent.futures import ProcessPoolExecutor

        with ProcessPoolExecutor(max_workers=workers) as ex:
            dems = list(ex.map(_batch_tile, jobs))
    else:
        dems = [_batch_tile(j) for j in jobs]
    return [dict(dem=dems[i], spacing=w["spacing"], obs_height=float(heights[i]),
                 max_dist=int(sides[i]) * w["spacing"]) for i in range(ntiles)]
