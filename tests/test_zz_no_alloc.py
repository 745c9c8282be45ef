"""The allocation-free total viewshed (tvs_total_viewshed_noalloc) against the allocating entry
point (tvs_total_viewshed_async): the same kernels on the same inputs, the map bit for bit, on two
calls in a row (the second smaller, so it runs on what the first left in the shared scratch), and
the size limit rejected before any work is enqueued."""
import ctypes as C
import math
import sys

import numpy as np
import pytest

from synth import fractal_dem

pytestmark = pytest.mark.gpu


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


CALLS = [
    # (rows, cols, n_sectors, max_dist, seed): several sector groups in the 256 MiB array, then a
    # smaller grid with unbounded lines of sight
    (1200, 900, 60, 3000.0, 11),
    (300, 257, 37, math.inf, 12),
]


def test_noalloc_matches_async_twice(tvs):
    import torch

    torch.cuda.set_device(0)
    for (H, W, n, R, seed) in CALLS:
        note(f"noalloc H={H} W={W} n={n} R={R} seed={seed}")
        dem = fractal_dem(max(H, W), seed, 0.6, 1200.0)[:H, :W].copy()
        d = torch.from_numpy(dem).cuda()
        want = tvs.total_viewshed(d, 10.0, 1.5, n, R)
        got = torch.full((H, W), -1.0, dtype=torch.float64, device="cuda")
        tvs.total_viewshed_noalloc(d, 10.0, 1.5, n, R, out=got)
        torch.cuda.synchronize()
        w, g = want.cpu().numpy(), got.cpu().numpy()
        assert np.all(np.isfinite(g)) and np.all(g > 0)
        assert np.array_equal(g, w), f"{H}x{W}: max |diff| {np.max(np.abs(g - w))}"


def test_noalloc_rejects_grid_beyond_scratch(tvs):
    """A grid one of whose sectors does not fit the array: TVS_ERANGE, output untouched."""
    import torch

    torch.cuda.set_device(0)
    H = W = 6000
    note(f"noalloc size limit {H}x{W}")
    d = torch.zeros((H, W), dtype=torch.float32, device="cuda")
    out = torch.full((H, W), 7.0, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    with pytest.raises(tvs.TvsError) as ei:
        tvs.total_viewshed_noalloc(d, 10.0, 1.5, 8, 1000.0, out=out)
    assert ei.value.status == -4
    assert "allocation-free scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool(torch.all(out == 7.0))
