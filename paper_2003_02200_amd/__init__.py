"""libtvs: the sDEM total viewshed on MI355X (gfx950).

Thin ctypes binding over ``libtvs.so`` (C ABI in ``include/libtvs.h``). Every step of the
method runs in the library's HIP kernels; this module only marshals arguments. PyTorch is
used for device memory and streams. There is no CPU fallback: if the library is missing the
import of any entry point raises.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

__all__ = [
    "TvsError", "lib", "total_viewshed", "singular_viewshed", "debug_sector_rays", "sector_shape",
    "los_evals", "abi_version", "FLAG_SLOPE_F64", "FLAG_SWEEP_SCAN", "FLAG_ACC_KAHAN32", "FLAG_SLOPE_EXACT", "FLAG_NO_PRUNE",
    "FLAG_COUNT_EVALS", "FLAG_SLOPE_F32", "FLAG_AUTOTUNE", "FLAG_COMPACT", "FLAG_RELOCATE", "Stats", "Batch", "BatchInfo",
    "BatchBucket",
    "total_viewshed_tiles", "Server", "multiple_viewshed", "singular_mask", "total_viewshed_noalloc",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(_HERE, "libtvs.so")

FLAG_SLOPE_F64 = 0x1
FLAG_SWEEP_SCAN = 0x2
FLAG_ACC_KAHAN32 = 0x4
FLAG_SLOPE_EXACT = 0x8
FLAG_NO_PRUNE = 0x10
FLAG_COUNT_EVALS = 0x20
FLAG_SLOPE_F32 = 0x40
FLAG_AUTOTUNE = 0x80
FLAG_COMPACT = 0x100  # skewed row t stored in row t mod (Hx + 1): Hx + 1 rows per sector
FLAG_RELOCATE = 0x200  # relocation kernel writes skwDEM; the sweep reads it (default: rows gathered from the grid)

_STATUS = {0: "TVS_OK", -1: "TVS_EINVAL", -2: "TVS_ENOMEM", -3: "TVS_EDEVICE", -4: "TVS_ERANGE", -5: "TVS_ETIMEDOUT"}


class TvsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class Stats(C.Structure):
    _fields_ = [
        ("reloc_ms", C.c_double), ("sweep_ms", C.c_double), ("backproj_ms", C.c_double),
        ("reloc_launches", C.c_int32), ("sweep_launches", C.c_int32), ("backproj_launches", C.c_int32),
        ("chunks", C.c_int32), ("los_evals", C.c_int64), ("pov_sector_pairs", C.c_int64),
        ("reloc_bytes", C.c_int64), ("sweep_bytes", C.c_int64), ("scratch_bytes", C.c_int64),
        ("sweep_evals_done", C.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Tile(C.Structure):
    _fields_ = [("d_dem", C.c_void_p), ("d_out", C.c_void_p), ("rows", C.c_int32), ("cols", C.c_int32),
                ("spacing", C.c_double), ("obs_height", C.c_double), ("max_dist", C.c_double)]


class BatchInfo(C.Structure):
    _fields_ = [("tiles", C.c_int32), ("chunks", C.c_int32), ("kernel_launches", C.c_int32),
                ("waves_per_group", C.c_int32), ("groups", C.c_int32), ("tuned", C.c_int32),
                ("los_evals", C.c_int64), ("pov_sector_pairs", C.c_int64), ("sweep_evals_done", C.c_int64),
                ("scratch_bytes", C.c_int64), ("tune_ms", C.c_double), ("buckets", C.c_int32), ("pad", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class BatchBucket(C.Structure):
    _fields_ = [("side_class", C.c_int32), ("reach_class", C.c_int32), ("tiles", C.c_int32),
                ("longest_side", C.c_int32), ("longest_reach", C.c_int32), ("waves_per_group", C.c_int32),
                ("groups_per_cu", C.c_int32), ("tuned", C.c_int32), ("items", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerConfig(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("streams", C.c_int32), ("max_singular_batch", C.c_int32),
                ("max_total_batch", C.c_int32), ("pad", C.c_int32)]


class RequestResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("kind", C.c_int32), ("area_m2", C.c_double), ("latency_ms", C.c_double),
                ("queue_ms", C.c_double), ("rows", C.c_int32), ("cols", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("grids", C.c_int32), ("pending", C.c_int32), ("running", C.c_int32), ("pad", C.c_int32),
                ("completed", C.c_int64), ("singular_batches", C.c_int64), ("singular_batched", C.c_int64),
                ("max_concurrent_totals", C.c_int64), ("budget_bytes", C.c_int64), ("bytes_in_use", C.c_int64),
                ("peak_bytes", C.c_int64), ("total_batches", C.c_int64), ("total_batched", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


_lib = None
i32, f64, u32, vp = C.c_int32, C.c_double, C.c_uint32, C.c_void_p


def lib():
    """The loaded libtvs.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO_PATH):
            raise ImportError(f"libtvs.so not found at {SO_PATH}; build it with "
                              "`python -m paper_2003_02200_amd.build`")
        L = C.CDLL(SO_PATH)
        L.tvs_abi_version.restype = C.c_int
        L.tvs_last_error.restype = C.c_char_p
        L.tvs_total_viewshed.argtypes = [vp, i32, i32, f64, f64, i32, f64, vp]
        L.tvs_singular_viewshed.argtypes = [vp, i32, i32, f64, f64, i32, f64, i32, i32, vp, vp]
        L.tvs_total_viewshed_async.argtypes = [vp, i32, i32, f64, f64, i32, f64, vp, vp]
        L.tvs_singular_viewshed_async.argtypes = [vp, i32, i32, f64, f64, i32, f64, i32, i32, vp, vp, vp]
        L.tvs_total_viewshed_ex.argtypes = [vp, i32, i32, f64, f64, i32, f64, vp, u32, C.POINTER(Stats), vp]
        L.tvs_singular_viewshed_ex.argtypes = [vp, i32, i32, f64, f64, i32, f64, i32, i32, u32, vp, vp, vp]
        L.tvs_sector_shape.argtypes = [i32, i32, i32, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
        L.tvs_debug_sector_rays.argtypes = [vp, i32, i32, f64, f64, i32, f64, i32, u32, vp]
        L.tvs_debug_sector_rays_async.argtypes = [vp, i32, i32, f64, f64, i32, f64, i32, u32, vp, vp]
        L.tvs_batch_create.argtypes = [C.POINTER(Tile), i32, i32, u32, C.POINTER(C.c_void_p)]
        L.tvs_batch_run.argtypes = [vp, vp]
        L.tvs_batch_get_info.argtypes = [vp, C.POINTER(BatchInfo)]
        L.tvs_batch_get_bucket.argtypes = [vp, i32, C.POINTER(BatchBucket)]
        L.tvs_batch_destroy.argtypes = [vp]
        L.tvs_total_viewshed_tiles.argtypes = [C.POINTER(Tile), i32, i32, u32, vp]
        u64p = C.POINTER(C.c_uint64)
        L.tvs_server_create.argtypes = [C.POINTER(ServerConfig), C.POINTER(C.c_void_p)]
        L.tvs_server_add_grid.argtypes = [vp, vp, i32, i32, f64, C.POINTER(i32)]
        L.tvs_server_submit_total.argtypes = [vp, i32, f64, i32, f64, u32, u64p]
        L.tvs_server_submit_singular.argtypes = [vp, i32, f64, i32, f64, i32, i32, u32, u64p]
        L.tvs_server_wait.argtypes = [vp, C.c_uint64, f64, C.POINTER(RequestResult)]
        L.tvs_server_copy_map.argtypes = [vp, C.c_uint64, vp, vp]
        L.tvs_server_release.argtypes = [vp, C.c_uint64]
        L.tvs_server_get_stats.argtypes = [vp, C.POINTER(ServerStats)]
        L.tvs_server_destroy.argtypes = [vp]
        L.tvs_multiple_viewshed.argtypes = [vp, i32, i32, f64, f64, i32, f64, vp, i32, u32, vp, vp, vp]
        L.tvs_los_evals.argtypes = [i32, i32, f64, i32, f64, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.tvs_total_viewshed_noalloc.argtypes = [vp, i32, i32, f64, f64, i32, f64, vp, vp]
        for name in ("tvs_total_viewshed", "tvs_singular_viewshed", "tvs_total_viewshed_async",
                     "tvs_singular_viewshed_async", "tvs_total_viewshed_ex", "tvs_singular_viewshed_ex",
                     "tvs_sector_shape", "tvs_debug_sector_rays", "tvs_debug_sector_rays_async", "tvs_los_evals",
                     "tvs_batch_create", "tvs_batch_run", "tvs_batch_get_info", "tvs_batch_get_bucket",
                     "tvs_batch_destroy",
                     "tvs_total_viewshed_tiles", "tvs_server_create", "tvs_server_add_grid",
                     "tvs_server_submit_total", "tvs_server_submit_singular", "tvs_server_wait",
                     "tvs_server_copy_map", "tvs_server_release", "tvs_server_get_stats", "tvs_server_destroy",
                     "tvs_multiple_viewshed", "tvs_total_viewshed_noalloc"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        msg = lib().tvs_last_error()
        raise TvsError(rc, msg.decode() if msg else "")


def abi_version() -> int:
    return lib().tvs_abi_version()


def _is_torch_cuda(x) -> bool:
    try:
        import torch
    except ImportError:  # pragma: no cover
        return False
    return isinstance(x, torch.Tensor) and x.is_cuda


def _stream_handle(stream):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _host_dem(dem):
    a = np.ascontiguousarray(dem, dtype=np.float32)
    if a.ndim != 2:
        raise ValueError("dem must be a 2-D grid")
    return a


def total_viewshed(dem, spacing: float, obs_height: float, n_sectors: int, max_dist: float = math.inf,
                   flags: int = 0, stream=None, stats: bool = False):
    """Total viewshed (m^2) of every cell.

    ``dem``: numpy array (host call, synchronous) or CUDA float32 torch tensor (stream-ordered
    on ``stream`` or the current stream; returns a float64 tensor on the same device). With
    ``stats=True`` returns ``(out, Stats)``.
    """
    L = lib()
    if _is_torch_cuda(dem):
        import torch

        if dem.dtype != torch.float32 or dem.dim() != 2:
            raise ValueError("device dem must be a 2-D float32 tensor")
        d = dem.contiguous()
        H, W = d.shape
        out = torch.empty((H, W), dtype=torch.float64, device=d.device)
        st = Stats() if stats else None
        with torch.cuda.device(d.device):
            rc = L.tvs_total_viewshed_ex(C.c_void_p(d.data_ptr()), H, W, spacing, obs_height, n_sectors, max_dist,
                                         C.c_void_p(out.data_ptr()), flags, C.byref(st) if st else None,
                                         _stream_handle(stream))
        _check(rc)
        return (out, st) if stats else out
    a = _host_dem(dem)
    H, W = a.shape
    if flags or stats:
        import torch

        out, st = total_viewshed(torch.from_numpy(a).cuda(), spacing, obs_height, n_sectors, max_dist, flags,
                                 stream, True)
        torch.cuda.synchronize()
        res = out.cpu().numpy()
        return (res, st) if stats else res
    out = np.empty((H, W), np.float64)
    _check(L.tvs_total_viewshed(a.ctypes.data_as(vp), H, W, spacing, obs_height, n_sectors, max_dist,
                                out.ctypes.data_as(vp)))
    return out


def total_viewshed_noalloc(dem, spacing: float, obs_height: float, n_sectors: int, max_dist: float = math.inf,
                           out=None, stream=None):
    """tvs_total_viewshed_noalloc: the total viewshed of a device grid (CUDA float32 tensor) into
    ``out`` (a float64 tensor of the grid's shape on the same device; allocated here when None),
    with no device allocation inside the library call. Ordered on ``stream`` or the current stream."""
    import torch

    if not (_is_torch_cuda(dem) and dem.dtype == torch.float32 and dem.dim() == 2):
        raise ValueError("dem must be a 2-D float32 CUDA tensor")
    d = dem.contiguous()
    H, W = d.shape
    if out is None:
        out = torch.empty((H, W), dtype=torch.float64, device=d.device)
    if not (_is_torch_cuda(out) and out.dtype == torch.float64 and tuple(out.shape) == (H, W)
            and out.is_contiguous() and out.device == d.device):
        raise ValueError("out must be a contiguous float64 CUDA tensor of the grid's shape on its device")
    with torch.cuda.device(d.device):
        _check(lib().tvs_total_viewshed_noalloc(C.c_void_p(d.data_ptr()), H, W, spacing, obs_height, n_sectors,
                                                max_dist, C.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


def singular_viewshed(dem, spacing: float, obs_height: float, n_sectors: int, max_dist: float, pov_row: int,
                      pov_col: int, flags: int = 0, rays: bool = False, stream=None):
    """Area (m^2) visible from one cell. With ``rays=True`` also the 2n packed per-ray sums
    (forward, backward per sector; U | e << 30). Host numpy grids are uploaded with torch."""
    L = lib()
    import torch

    d = dem if _is_torch_cuda(dem) else torch.from_numpy(_host_dem(dem)).cuda()
    if d.dtype != torch.float32 or d.dim() != 2:
        raise ValueError("dem must be a 2-D float32 grid")
    d = d.contiguous()
    H, W = d.shape
    area = torch.empty(1, dtype=torch.float64, device=d.device)
    rv = torch.empty(2 * n_sectors, dtype=torch.int32, device=d.device) if rays else None
    with torch.cuda.device(d.device):
        rc = L.tvs_singular_viewshed_ex(C.c_void_p(d.data_ptr()), H, W, spacing, obs_height, n_sectors, max_dist,
                                        pov_row, pov_col, flags, C.c_void_p(area.data_ptr()),
                                        C.c_void_p(rv.data_ptr()) if rays else None, _stream_handle(stream))
    _check(rc)
    torch.cuda.current_stream(d.device).synchronize() if stream is None else stream.synchronize()
    a = float(area.item())
    if rays:
        return a, rv.cpu().numpy().view(np.uint32).copy()
    return a


def singular_mask(dem, spacing: float, obs_height: float, n_sectors: int, max_dist: float, pov_row: int,
                  pov_col: int):
    """(area, mask): the singular viewshed's area and its per-cell visibility (uint8 0/1), host
    arrays (tvs_singular_viewshed with a mask)."""
    a = _host_dem(dem)
    H, W = a.shape
    area = C.c_double()
    mask = np.empty((H, W), np.uint8)
    _check(lib().tvs_singular_viewshed(a.ctypes.data_as(vp), H, W, spacing, obs_height, n_sectors, max_dist,
                                       pov_row, pov_col, C.byref(area), mask.ctypes.data_as(vp)))
    return area.value, mask


def multiple_viewshed(dem, spacing: float, obs_height: float, n_sectors: int, max_dist: float, povs, flags: int = 0,
                      stream=None, areas: bool = False):
    """Per cell, how many of the POVs [(row, col), ...] see it (uint32 map; a device tensor for a
    device dem, else numpy). With ``areas=True`` also each POV's singular area."""
    import torch

    d = dem if _is_torch_cuda(dem) else torch.from_numpy(_host_dem(dem)).cuda()
    if d.dtype != torch.float32 or d.dim() != 2:
        raise ValueError("dem must be a 2-D float32 grid")
    d = d.contiguous()
    H, W = d.shape
    p = np.ascontiguousarray(np.asarray(povs, np.int32).reshape(-1, 2))
    cnt = torch.empty((H, W), dtype=torch.int32, device=d.device)
    ar = torch.empty(len(p), dtype=torch.float64, device=d.device)
    with torch.cuda.device(d.device):
        _check(lib().tvs_multiple_viewshed(C.c_void_p(d.data_ptr()), H, W, spacing, obs_height, n_sectors, max_dist,
                                           p.ctypes.data_as(vp), len(p), flags, C.c_void_p(cnt.data_ptr()),
                                           C.c_void_p(ar.data_ptr()), _stream_handle(stream)))
    if _is_torch_cuda(dem):
        return (cnt, ar) if areas else cnt
    torch.cuda.current_stream(d.device).synchronize() if stream is None else stream.synchronize()
    c = cnt.cpu().numpy().view(np.uint32).copy()
    return (c, ar.cpu().numpy()) if areas else c


def sector_shape(rows: int, cols: int, n_sectors: int, sector: int):
    nr, nc, t0 = i32(), i32(), i32()
    _check(lib().tvs_sector_shape(rows, cols, n_sectors, sector, C.byref(nr), C.byref(nc), C.byref(t0)))
    return nr.value, nc.value, t0.value


def debug_sector_rays(dem, spacing: float, obs_height: float, n_sectors: int, max_dist: float, sector: int,
                      flags: int = 0, stream=None):
    """Per-sector skewed viewshed (nrows x ncols, U | e << 30; 0xFFFFFFFF = no sample).

    A host numpy grid gives a numpy uint32 array (synchronous); a CUDA float32 tensor gives an
    int32 tensor on its device holding the same bits, ordered on ``stream`` or the current stream.
    """
    if _is_torch_cuda(dem):
        import torch

        if dem.dtype != torch.float32 or dem.dim() != 2:
            raise ValueError("device dem must be a 2-D float32 tensor")
        d = dem.contiguous()
        H, W = d.shape
        nr, nc, _ = sector_shape(H, W, n_sectors, sector)
        out = torch.empty((nr, nc), dtype=torch.int32, device=d.device)
        with torch.cuda.device(d.device):
            _check(lib().tvs_debug_sector_rays_async(C.c_void_p(d.data_ptr()), H, W, spacing, obs_height, n_sectors,
                                                     max_dist, sector, flags, C.c_void_p(out.data_ptr()),
                                                     _stream_handle(stream)))
        return out
    a = _host_dem(dem)
    H, W = a.shape
    nr, nc, _ = sector_shape(H, W, n_sectors, sector)
    out = np.empty((nr, nc), np.uint32)
    _check(lib().tvs_debug_sector_rays(a.ctypes.data_as(vp), H, W, spacing, obs_height, n_sectors, max_dist,
                                       sector, flags, out.ctypes.data_as(vp)))
    return out


def los_evals(rows: int, cols: int, spacing: float, n_sectors: int, max_dist: float):
    ev, pr = C.c_int64(), C.c_int64()
    _check(lib().tvs_los_evals(rows, cols, spacing, n_sectors, max_dist, C.byref(ev), C.byref(pr)))
    return ev.value, pr.value


def _tiles(tiles):
    """(dem, out, spacing, obs_height, max_dist) device tensors and scalars -> Tile array (the
    tensors must outlive every use of the array)."""
    import torch

    arr = (Tile * len(tiles))()
    for x, (dem, out, spacing, h0, R) in enumerate(tiles):
        if not (_is_torch_cuda(dem) and dem.dtype == torch.float32 and dem.dim() == 2 and dem.is_contiguous()):
            raise ValueError(f"tile {x}: dem must be a contiguous 2-D float32 CUDA tensor")
        if not (_is_torch_cuda(out) and out.dtype == torch.float64 and out.shape == dem.shape and out.is_contiguous()):
            raise ValueError(f"tile {x}: out must be a contiguous float64 CUDA tensor of the dem's shape")
        arr[x] = Tile(dem.data_ptr(), out.data_ptr(), dem.shape[0], dem.shape[1], spacing, h0, R)
    return arr


class Batch:
    """A planned batch of independent tiles (tvs_batch_create); ``run`` replays its captured
    graph on a stream. ``tiles`` is a list of (dem, out, spacing, obs_height, max_dist) with
    device tensors that must stay alive (and in place) until ``close``."""

    def __init__(self, tiles, n_sectors: int, flags: int = 0):
        self._keep = [(t[0], t[1]) for t in tiles]
        arr = _tiles(tiles)
        h = C.c_void_p()
        _check(lib().tvs_batch_create(arr, len(tiles), n_sectors, flags, C.byref(h)))
        self._h = h

    def run(self, stream=None):
        _check(lib().tvs_batch_run(self._h, _stream_handle(stream)))

    def info(self) -> BatchInfo:
        inf = BatchInfo()
        _check(lib().tvs_batch_get_info(self._h, C.byref(inf)))
        return inf

    def buckets(self):
        """The batch's buckets of tiles (one sweep launch and launch shape each), largest tiles first."""
        out = []
        for i in range(self.info().buckets):
            bk = BatchBucket()
            _check(lib().tvs_batch_get_bucket(self._h, i, C.byref(bk)))
            out.append(bk.as_dict())
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().tvs_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def total_viewshed_tiles(tiles, n_sectors: int, flags: int = 0, stream=None):
    """The plain per-tile loop (tvs_total_viewshed_tiles) over (dem, out, spacing, obs_height,
    max_dist) device tiles, enqueued on ``stream`` or the current stream."""
    arr = _tiles(tiles)
    _check(lib().tvs_total_viewshed_tiles(arr, len(tiles), n_sectors, flags, _stream_handle(stream)))


class Server:
    """A request server (tvs_server_*): resident grids, total and singular requests from any
    thread, continuous batching on the device. Results come back by ticket."""

    def __init__(self, hbm_budget_bytes: int = 0, streams: int = 0, max_singular_batch: int = 0,
                 max_total_batch: int = 0):
        cfg = ServerConfig(hbm_budget_bytes, streams, max_singular_batch, max_total_batch, 0)
        h = C.c_void_p()
        _check(lib().tvs_server_create(C.byref(cfg), C.byref(h)))
        self._h = h

    def add_grid(self, dem, spacing: float) -> int:
        a = _host_dem(dem)
        gid = i32()
        _check(lib().tvs_server_add_grid(self._h, a.ctypes.data_as(vp), a.shape[0], a.shape[1], spacing,
                                         C.byref(gid)))
        return gid.value

    def submit_total(self, grid: int, obs_height: float, n_sectors: int, max_dist: float, flags: int = 0) -> int:
        t = C.c_uint64()
        _check(lib().tvs_server_submit_total(self._h, grid, obs_height, n_sectors, max_dist, flags, C.byref(t)))
        return t.value

    def submit_singular(self, grid: int, obs_height: float, n_sectors: int, max_dist: float, pov_row: int,
                        pov_col: int, flags: int = 0) -> int:
        t = C.c_uint64()
        _check(lib().tvs_server_submit_singular(self._h, grid, obs_height, n_sectors, max_dist, pov_row, pov_col,
                                                flags, C.byref(t)))
        return t.value

    def wait(self, ticket: int, timeout_ms: float = -1.0) -> RequestResult:
        r = RequestResult()
        _check(lib().tvs_server_wait(self._h, ticket, timeout_ms, C.byref(r)))
        return r

    def map(self, ticket: int):
        """The finished total request's map as a host numpy array."""
        r = self.wait(ticket)
        out = np.empty((r.rows, r.cols), np.float64)
        _check(lib().tvs_server_copy_map(self._h, ticket, out.ctypes.data_as(vp), None))
        return out

    def release(self, ticket: int):
        _check(lib().tvs_server_release(self._h, ticket))

    def stats(self) -> ServerStats:
        st = ServerStats()
        _check(lib().tvs_server_get_stats(self._h, C.byref(st)))
        return st

    def close(self):
        if getattr(self, "_h", None):
            lib().tvs_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
