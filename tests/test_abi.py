"""C-ABI checks that need no GPU: the library loads, exports every declared entry point, rejects
bad arguments before touching a device, and its host-side sector plan matches the oracle's."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "libtvs.h")


@pytest.fixture(scope="module")
def tvs():
    import paper_2003_02200_amd as t

    if not os.path.exists(t.SO_PATH):
        from paper_2003_02200_amd.build import build

        build()
    t.lib()
    return t


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(tvs_\w+)\s*\(", text, re.M)))


def test_exports_every_declared_symbol(tvs):
    names = _declared()
    assert len(names) >= 11
    L = C.CDLL(tvs.SO_PATH)
    for n in names:
        assert hasattr(L, n), n


def test_abi_version(tvs):
    m = re.search(r"#define TVS_ABI_VERSION (\d+)", open(HEADER).read())
    assert tvs.abi_version() == int(m.group(1))


@pytest.mark.parametrize("kw,status", [
    (dict(spacing=0.0), -1), (dict(spacing=math.nan), -1), (dict(spacing=math.inf), -1),
    (dict(obs_height=math.nan), -1), (dict(n_sectors=0), -1), (dict(n_sectors=40000), -1),
    (dict(max_dist=0.0), -1), (dict(max_dist=-5.0), -1), (dict(max_dist=math.nan), -1),
])
def test_rejects_bad_scalars(tvs, kw, status):
    args = dict(spacing=10.0, obs_height=1.5, n_sectors=8, max_dist=math.inf)
    args.update(kw)
    with pytest.raises(tvs.TvsError) as ei:
        tvs.total_viewshed(np.zeros((4, 4), np.float32), **args)
    assert ei.value.status == status


def test_rejects_bad_flag_combinations(tvs):
    import torch  # noqa: F401  (device tensors are not needed: validation happens first)
    L = tvs.lib()
    d = np.zeros(4, np.float32)
    out = np.zeros(4, np.float64)
    vp = C.c_void_p
    for flags in (0x800, 0x400, 0x80000000, 0x41):  # 0x41: float and double decisions together
        rc = L.tvs_total_viewshed_ex(d.ctypes.data_as(vp), 2, 2, 10.0, 1.5, 4, math.inf, out.ctypes.data_as(vp),
                                     flags, None, None)
        assert rc == -1, flags


def test_rejects_bad_grid(tvs):
    L = tvs.lib()
    out = np.zeros(4, np.float64)
    d = np.zeros(4, np.float32)
    vp = C.c_void_p
    assert L.tvs_total_viewshed(None, 2, 2, 10.0, 1.5, 4, math.inf, out.ctypes.data_as(vp)) == -1
    assert L.tvs_total_viewshed(d.ctypes.data_as(vp), 2, 2, 10.0, 1.5, 4, math.inf, None) == -1
    assert L.tvs_total_viewshed(d.ctypes.data_as(vp), 0, 2, 10.0, 1.5, 4, math.inf, out.ctypes.data_as(vp)) == -1
    assert L.tvs_total_viewshed(d.ctypes.data_as(vp), 40000, 2, 10.0, 1.5, 4, math.inf,
                                out.ctypes.data_as(vp)) == -4
    assert L.tvs_total_viewshed_async(None, 2, 2, 10.0, 1.5, 4, math.inf, None, None) == -1
    tiny = np.zeros((3, 3), np.float32)
    tiny[1, 1] = np.float32(1e-30)
    with pytest.raises(tvs.TvsError) as ei:
        tvs.total_viewshed(tiny, 10.0, 1.5, 4)
    assert ei.value.status == -1
    with pytest.raises(tvs.TvsError):
        tvs.total_viewshed(np.zeros((3, 3), np.float32), 10.0, 1e-25, 4)
    bad = np.zeros((3, 3), np.float32)
    bad[2, 1] = np.inf
    with pytest.raises(tvs.TvsError) as ei:
        tvs.total_viewshed(bad, 10.0, 1.5, 4)
    assert ei.value.status == -1 and "(2, 1)" in str(ei.value)
    area = C.c_double(7.0)
    assert L.tvs_singular_viewshed(d.ctypes.data_as(vp), 2, 2, 10.0, 1.5, 4, math.inf, 2, 0, C.byref(area),
                                   None) == -1
    mask = np.full(4, 9, np.uint8)
    assert L.tvs_singular_viewshed(d.ctypes.data_as(vp), 2, 2, 10.0, 1.5, 4, math.inf, 0, 5, C.byref(area),
                                   mask.ctypes.data_as(vp)) == -1
    assert area.value == 7.0 and np.all(mask == 9)  # outputs untouched on error
    assert b"POV" in L.tvs_last_error()
    povs = np.array([0, 0, 1, 2], np.int32)  # second POV outside the 2 x 2 grid
    cnt = np.zeros(4, np.uint32)
    L.tvs_multiple_viewshed.argtypes = [vp, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_int32, C.c_double, vp,
                                        C.c_int32, C.c_uint32, vp, vp, vp]
    assert L.tvs_multiple_viewshed(d.ctypes.data_as(vp), 2, 2, 10.0, 1.5, 4, math.inf, povs.ctypes.data_as(vp), 2, 0,
                                   cnt.ctypes.data_as(vp), None, None) == -1
    assert b"POV 1" in L.tvs_last_error()
    assert L.tvs_multiple_viewshed(d.ctypes.data_as(vp), 2, 2, 10.0, 1.5, 4, math.inf, povs.ctypes.data_as(vp), 0, 0,
                                   cnt.ctypes.data_as(vp), None, None) == -1


@pytest.mark.parametrize("H,W,n,R", [(37, 53, 7, math.inf), (1, 1, 3, 5.0), (64, 17, 180, 300.0),
                                     (5, 200, 13, 77.7), (2000, 2000, 180, 10000.0), (128, 128, 180, 1280.0)])
def test_plan_matches_oracle(tvs, orc, H, W, n, R):
    """Skewed-grid shapes and the closed-form work count agree with the oracle's independent plan."""
    for k in range(0, n, max(1, n // 12)):
        o = orc.sector_info(H, W, 10.0, n, R, k)
        assert tvs.sector_shape(H, W, n, k) == (o["nrows"], o["Wx"], o["t0"])
    if H * W <= 5000 or (H, W) == (128, 128):
        assert tvs.los_evals(H, W, 10.0, n, R) == orc.los_evals(H, W, 10.0, n, R)
    if (H, W) == (2000, 2000):
        assert tvs.los_evals(H, W, 10.0, n, R) == (920007832528, 720351824)


def test_batch_rejects_bad_arguments(tvs):
    """Batch validation happens before any device work: null lists, bad tiles, bad flags."""
    L = tvs.lib()
    h = C.c_void_p()
    assert L.tvs_batch_create(None, 1, 8, 0, C.byref(h)) == -1
    t = (tvs.Tile * 2)()
    t[0] = tvs.Tile(16, 32, 4, 4, 10.0, 1.5, 100.0)  # never dereferenced: validation fails first
    t[1] = tvs.Tile(16, 32, 4, 0, 10.0, 1.5, 100.0)  # zero columns
    assert L.tvs_batch_create(t, 2, 8, 0, C.byref(h)) == -1
    assert b"tile 1" in L.tvs_last_error()
    t[1] = tvs.Tile(None, 32, 4, 4, 10.0, 1.5, 100.0)
    assert L.tvs_batch_create(t, 2, 8, 0, C.byref(h)) == -1
    t[1] = tvs.Tile(16, 32, 4, 4, 10.0, 1.5, 100.0)
    for flags in (tvs.FLAG_SWEEP_SCAN, tvs.FLAG_ACC_KAHAN32, tvs.FLAG_NO_PRUNE, 0x41, 0x200):
        assert L.tvs_batch_create(t, 2, 8, flags, C.byref(h)) == -1, flags
    assert L.tvs_batch_create(t, 2, 0, 0, C.byref(h)) == -1
    assert L.tvs_batch_create(t, 0, 8, 0, C.byref(h)) == -1
    assert L.tvs_batch_run(None, None) == -1
    assert L.tvs_batch_destroy(None) == 0
    assert L.tvs_total_viewshed_tiles(None, 1, 8, 0, None) == -1


def test_host_elevation_check_boundaries(tvs):
    """The host entry point's elevation check (finite, and 0 or at least 2^-60 m in magnitude) at its
    boundaries: rejected values give TVS_EINVAL naming the cell; accepted grids pass validation
    (what follows needs a device, so only the absence of TVS_EINVAL is checked)."""
    L = tvs.lib()
    vp = C.c_void_p
    out = np.zeros(12, np.float64)
    lim = np.float32(2.0 ** -60)
    for v, ok in ((lim, True), (-lim, True), (np.float32(-0.0), True), (np.float32(3.0e38), True),
                  (np.nextafter(lim, np.float32(0)), False), (np.float32(-1e-30), False),
                  (np.float32(1e-45), False), (np.float32(np.nan), False), (np.float32(-np.inf), False)):
        d = np.full((3, 4), 7.0, np.float32)
        d[2, 3] = v
        rc = L.tvs_total_viewshed(d.ctypes.data_as(vp), 3, 4, 10.0, 1.5, 4, math.inf, out.ctypes.data_as(vp))
        if ok:
            assert rc != -1, (v, L.tvs_last_error())
        else:
            assert rc == -1 and b"(2, 3)" in L.tvs_last_error(), v
