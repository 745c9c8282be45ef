"""GPU parity cases beyond the shape table (run on an MI355X; marked `gpu`):

* one sector axis (0 deg) and two (0 and 90 deg): the per-sector ring sums bit for bit against the
  oracle in every decision mode, and the whole map against independent plain walks along grid rows
  and grid columns written here (no skew, no interpolation, no oracle code): at these angles every
  line of sight is a grid row or a grid column (Alg. 1's sector loop at s = 0 and 90 deg);
* tiles of the batch workload's sizes (256, 1024, 2048; max distance = tile extent) through the
  batched path, against the all-double oracle on 128 x 128 windows, with horizon-flip counts of
  sampled sectors (Section 4.1 steps 1a-1d per tile);
* a flip scan of the 8000 x 8000 workload: the default decisions against the correctly rounded
  double quotient (TVS_FLAG_SLOPE_F64, itself bit-exact against the oracle on the shape table)
  over a sample of sectors.
"""
import math
import sys

import numpy as np
import pytest

from synth import WORKLOADS, fractal_dem, workload_dem

pytestmark = pytest.mark.gpu
INF = math.inf
F64, EXACT, F32 = 0x1, 0x8, 0x40
# (flags, oracle precision, plain-walk slope) of every decision mode
MODES = [(0, 65, "rcp64"), (F64, 64, "quot64"), (F32, 33, "rcp32"), (F32 | EXACT, 32, "quot32")]


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


def packed(o):
    v = o["U"].astype(np.uint32) | (o["e"].astype(np.uint32) << np.uint32(30))
    v[o["valid"] == 0] = np.uint32(0xFFFFFFFF)
    return v


def _dem(H, W, kind, seed):
    if kind == "int":
        rng = np.random.default_rng(seed)
        return np.round(rng.uniform(0, 12, (H, W))).astype(np.float32)
    return fractal_dem(max(H, W), seed, 0.6, 400.0)[:H, :W].copy()


AXES = [
    # (H, W, n, R, terrain)
    (37, 53, 1, INF, "fractal"),
    (53, 37, 1, 123.4, "int"),
    (9, 6000, 1, 2000.0, "fractal"),
    (37, 53, 2, 530.0, "fractal"),
    (300, 17, 2, INF, "int"),
    (3000, 9, 2, 1500.0, "fractal"),
]


@pytest.mark.parametrize("H,W,n,R,kind", AXES)
def test_one_and_two_axes_sector_rays(tvs, orc, H, W, n, R, kind):
    dem = _dem(H, W, kind, 21)
    for k in range(n):
        for flags, prec, _ in MODES:
            note(f"axes sector_rays H={H} W={W} n={n} R={R} k={k} flags={flags}")
            g = tvs.debug_sector_rays(dem, 10.0, 1.5, n, R, k, flags=flags)
            o = orc.sector_V(dem, 10.0, 1.5, n, R, k, prec=prec)
            assert np.array_equal(g, packed(o)), f"k={k} flags={flags}"


def _slope(d, m, kind):
    if kind == "rcp64":
        return d * (1.0 / m)
    if kind == "quot64":
        return d / float(m)
    if kind == "rcp32":
        return d * (np.float32(1.0) / np.float32(m))
    return d / np.float32(m)


def _walk_forward(z, h, rho, kind):
    """Ring sums (index^2 units) of the forward line of sight of every POV of every grid row:
    targets m = 1, 2, ... while inside the row and m < rho; target m visible iff its slope
    (z_m - h) / m beats every earlier one (strictly); it owns the ring [m, m + 1) clipped at rho,
    the POV the ring [0, 1)."""
    H, W = z.shape
    cv = np.full((H, W), min(1.0, rho) ** 2)
    mx = np.full((H, W), -np.inf, dtype=z.dtype)
    m = 1
    while m < W and m < rho:
        th = _slope(z[:, m:] - h[:, :W - m], m, kind)
        vis = th > mx[:, :W - m]
        cv[:, :W - m] += np.where(vis, min(m + 1.0, rho) ** 2 - float(m) * m, 0.0)
        mx[:, :W - m] = np.maximum(mx[:, :W - m], th)
        m += 1
    return cv


def _walk_rows(dem, h0, rho, kind):
    """Forward plus backward ring sums along grid rows, elevations and slopes in the mode's
    precision (h = z + h0 formed in that precision)."""
    if kind.endswith("32"):
        z = dem.astype(np.float32)
        h = z + np.float32(h0)
    else:
        z = dem.astype(np.float64)
        h = z + h0
    fwd = _walk_forward(z, h, rho, kind)
    bwd = _walk_forward(z[:, ::-1], h[:, ::-1], rho, kind)[:, ::-1]
    return fwd + bwd


@pytest.mark.parametrize("H,W,R", [(37, 211, INF), (61, 150, 1234.5), (150, 47, 333.0)])
@pytest.mark.parametrize("flags,prec,kind", MODES)
def test_one_and_two_axes_equal_row_and_column_walks(tvs, H, W, R, flags, prec, kind):
    """n = 1: the map is (pi/2) dx^2 times the row walks; n = 2: (pi/4) dx^2 times row plus column
    walks (0 deg lines of sight run along grid rows, 90 deg along grid columns)."""
    import torch

    dx, h0 = 10.0, 1.5
    dem = fractal_dem(max(H, W), 31, 0.6, 900.0)[:H, :W].copy()
    rho = R / dx
    rows = _walk_rows(dem, h0, rho, kind)
    cols = _walk_rows(np.ascontiguousarray(dem.T), h0, rho, kind).T
    d = torch.from_numpy(dem).cuda()
    note(f"axes walks H={H} W={W} R={R} flags={flags}")
    g1 = tvs.total_viewshed(d, dx, h0, 1, R, flags=flags).cpu().numpy()
    g2 = tvs.total_viewshed(d, dx, h0, 2, R, flags=flags).cpu().numpy()
    np.testing.assert_allclose(g1, (math.pi / 2) * dx * dx * rows, rtol=1e-13)
    np.testing.assert_allclose(g2, (math.pi / 4) * dx * dx * (rows + cols), rtol=1e-13)


BATCH_TILES = [
    # (side, terrain seed, observer height): the batch workload's extreme and middle sizes,
    # roughness 0.55, 0-2500 m, 10 m, max distance = tile extent, 180 sectors
    (256, 4101, 1.5),
    (1024, 4102, 17.25),
    (2048, 4103, 30.0),
]


def test_batch_tiles_against_double_oracle(tvs, orc):
    """Per tile: the centred 128 x 128 window of the batch map equals the oracle taking the same
    decisions (rtol 1e-12) and is within 1e-4 of the all-double oracle on every cell fed by no flip;
    sampled whole sectors count the flips (POV-sector pairs whose ring sums differ from the all-double
    oracle's), at most 1e-5 of their pairs."""
    import torch

    n, dx = 180, 10.0
    specs = [(fractal_dem(side, seed, 0.55, 2500.0), h0, side * dx) for side, seed, h0 in BATCH_TILES]
    dems = [torch.from_numpy(s[0]).cuda() for s in specs]
    outs = [torch.zeros(d.shape, dtype=torch.float64, device="cuda") for d in dems]
    note("batch of tiles 256, 1024, 2048 (max distance = extent)")
    b = tvs.Batch([(dems[x], outs[x], dx, specs[x][1], specs[x][2]) for x in range(len(specs))], n)
    b.run()
    torch.cuda.synchronize()
    flips = pairs = 0
    for x, (dem, h0, R) in enumerate(specs):
        side = dem.shape[0]
        c0 = (side - 128) // 2
        g = outs[x].cpu().numpy()[c0:c0 + 128, c0:c0 + 128]
        note(f"batch tile {side}: oracle windows")
        same = orc.total(dem, dx, h0, n, R, prec=65, window=(c0, c0, 128, 128))
        np.testing.assert_allclose(g, same, rtol=1e-12)
        dbl = orc.total(dem, dx, h0, n, R, prec=64, window=(c0, c0, 128, 128))
        rel = np.abs(g / dbl - 1.0)
        fed = rel > 1e-12  # cells fed by a flipped pair
        assert fed.sum() <= 16, f"tile {side}: {int(fed.sum())} cells differ from the double oracle"
        assert rel[~fed].max() <= 1e-4
        ks = [0, 45, 97] if side <= 1024 else [37]
        for k in ks:
            note(f"batch tile {side}: flip count sector {k}")
            gv = tvs.debug_sector_rays(dem, dx, h0, n, R, k)
            o = orc.sector_V(dem, dx, h0, n, R, k, prec=64)
            v = o["valid"].astype(bool)
            pairs += int(v.sum())
            flips += int((gv != packed(o))[v].sum())
    b.close()
    note(f"batch tiles: {flips} flips in {pairs} pairs")
    assert pairs > 5e6
    assert flips <= 1e-5 * pairs


def test_workload_8000_flip_scan(tvs):
    """8000 x 8000 workload (seed 6, 0-3000 m, 10 m, 1.5 m, 10 km, 180 sectors): over 12 sectors of
    all four base-frame cases, the default decisions (double difference times the double reciprocal)
    against the correctly rounded double quotient: flipped POV-sector pairs at most 1e-5 of the pairs."""
    import torch

    w = WORKLOADS["tvs8000"]
    dem = workload_dem("tvs8000")
    d = torch.from_numpy(dem).cuda()
    args = (w["spacing"], w["obs_height"], w["n_sectors"], w["max_dist"])
    flips = pairs = 0
    for k in (0, 9, 23, 44, 45, 61, 90, 112, 134, 135, 150, 179):
        note(f"tvs8000 flip scan sector {k}")
        a = tvs.debug_sector_rays(d, *args, k)
        b = tvs.debug_sector_rays(d, *args, k, flags=F64)
        valid = b != -1  # 0xFFFFFFFF: no sample
        assert torch.equal(a == -1, ~valid)
        pairs += int(valid.sum())
        flips += int((a != b).sum())
        del a, b, valid
    torch.cuda.synchronize()
    note(f"tvs8000: {flips} flips in {pairs} pairs")
    assert pairs > 5e8
    assert flips <= 1e-5 * pairs
