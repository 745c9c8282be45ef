"""ctypes front end of the plain CPU oracle (``tvs_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py``. The product library never imports, links or runs it.
It shares no code with the GPU path; both take their input grids from ``synth``.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tvs_oracle.c")
_SO = os.path.join(_HERE, "libtvs_oracle.so")
_lib = None

f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: plain C, no fast-math, no FMA contraction."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=gnu11",
               "-Wall", "-shared", "-fPIC", "-o", _SO + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_SO + ".tmp", _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_SO)
        L.oracle_sector_info.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_double, C.c_int,
                                         C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                         C.POINTER(C.c_longlong), C.POINTER(C.c_longlong),
                                         C.POINTER(C.c_double), C.POINTER(C.c_double),
                                         C.POINTER(C.c_longlong), C.POINTER(C.c_double),
                                         C.c_void_p, C.c_void_p]
        L.oracle_sector_V.argtypes = [f32p, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, C.c_double,
                                      C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_total.argtypes = [f32p, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, C.c_double,
                                   C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, f64p, C.POINTER(C.c_longlong)]
        L.oracle_threads.restype = C.c_int
        L.oracle_singular.argtypes = [f32p, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, C.c_double,
                                      C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double),
                                      C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_ray.argtypes = [f32p, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, C.c_double,
                                 C.c_int, C.c_int, C.c_int, C.c_longlong, C.c_longlong, C.c_int,
                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_longlong,
                                 C.POINTER(C.c_longlong), C.POINTER(C.c_double), C.POINTER(C.c_uint32),
                                 C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.oracle_multiple.argtypes = [f32p, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, C.c_double,
                                      C.c_int, i32p, C.c_int, u32p]
        L.oracle_half_sector.argtypes = [C.c_int, C.c_int, C.c_int]
        L.oracle_half_sector.restype = C.c_int
        L.oracle_los_evals.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_double,
                                       C.POINTER(C.c_longlong), C.POINTER(C.c_longlong)]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _dem(dem):
    return np.ascontiguousarray(dem, dtype=np.float32)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with status {rc}")


def sector_info(rows, cols, spacing, n, max_dist, k):
    kase, Hx, Wx = C.c_int(), C.c_int(), C.c_int()
    t0, nrows, K = C.c_longlong(), C.c_longlong(), C.c_longlong()
    T, rho, scale = C.c_double(), C.c_double(), C.c_double()
    Wmax = max(rows, cols)
    d = np.zeros(Wmax, np.int32)
    r = np.zeros(Wmax, np.float64)
    rc = lib().oracle_sector_info(rows, cols, spacing, n, max_dist, k, C.byref(kase), C.byref(Hx), C.byref(Wx),
                                  C.byref(t0), C.byref(nrows), C.byref(T), C.byref(rho), C.byref(K),
                                  C.byref(scale), _ptr(d), _ptr(r))
    _check(rc, "sector_info")
    return dict(case=kase.value, Hx=Hx.value, Wx=Wx.value, t0=t0.value, nrows=nrows.value, T=T.value,
                rho=rho.value, K=K.value, scale=scale.value, d=d[:Wx.value].copy(), r=r[:Wx.value].copy())


def sector_V(dem, spacing, obs_height, n, max_dist, k, prec=64):
    """Per-sector skewed viewshed: dict with U (u32), e (u8), valid (u8), cv (f64), all nrows x Wx."""
    dem = _dem(dem)
    H, W = dem.shape
    info = sector_info(H, W, spacing, n, max_dist, k)
    shape = (info["nrows"], info["Wx"])
    U = np.zeros(shape, np.uint32)
    e = np.zeros(shape, np.uint8)
    valid = np.zeros(shape, np.uint8)
    cv = np.zeros(shape, np.float64)
    rc = lib().oracle_sector_V(dem, H, W, spacing, obs_height, n, max_dist, k, prec,
                               _ptr(U), _ptr(e), _ptr(valid), _ptr(cv))
    _check(rc, "sector_V")
    info.update(U=U, e=e, valid=valid, cv=cv)
    return info


def total(dem, spacing, obs_height, n, max_dist, prec=64, window=None, count=False):
    """Total viewshed in m^2. ``window`` = (r0, c0, nr, nc) restricts the cells computed. With
    ``count=True`` also returns the number of line-of-sight evaluations the oracle performed."""
    dem = _dem(dem)
    H, W = dem.shape
    r0, c0, nr, nc = window if window is not None else (0, 0, H, W)
    out = np.zeros((nr, nc), np.float64)
    ev = C.c_longlong()
    rc = lib().oracle_total(dem, H, W, spacing, obs_height, n, max_dist, prec, r0, c0, nr, nc, out, C.byref(ev))
    _check(rc, "total")
    return (out, ev.value) if count else out


def threads():
    return lib().oracle_threads()


def singular(dem, spacing, obs_height, n, max_dist, i0, j0, prec=64):
    dem = _dem(dem)
    H, W = dem.shape
    area = C.c_double()
    U = np.zeros(2 * n, np.uint32)
    e = np.zeros(2 * n, np.uint8)
    cv = np.zeros(2 * n, np.float64)
    rc = lib().oracle_singular(dem, H, W, spacing, obs_height, n, max_dist, prec, i0, j0, C.byref(area),
                               _ptr(U), _ptr(e), _ptr(cv))
    _check(rc, "singular")
    return dict(area=area.value, U=U, e=e, cv=cv)


def multiple(dem, spacing, obs_height, n, max_dist, povs, prec=64):
    """Multiple viewshed: per cell, how many of the POVs [(row, col), ...] see it (u32 map);
    with one POV, that POV's visibility mask."""
    dem = _dem(dem)
    H, W = dem.shape
    p = np.ascontiguousarray(np.asarray(povs, np.int32).reshape(-1, 2))
    out = np.zeros((H, W), np.uint32)
    _check(lib().oracle_multiple(dem, H, W, spacing, obs_height, n, max_dist, prec, p, len(p), out), "multiple")
    return out


def half_sector(n, di, dj):
    return lib().oracle_half_sector(n, di, dj)


def ray(dem, spacing, obs_height, n, max_dist, k, mode, t_or_p0, q0, delta, prec=64, cap=None):
    """One line of sight: mode 0 = skewed row t through column q0; mode 1 = singular through (p0, q0)."""
    dem = _dem(dem)
    H, W = dem.shape
    cap = cap if cap is not None else 2 * max(H, W) + 2
    vis = np.zeros(cap, np.uint8)
    th = np.zeros(cap, np.float64)
    zs = np.zeros(cap, np.float64)
    M, cv, U, e, h = C.c_longlong(), C.c_double(), C.c_uint32(), C.c_int(), C.c_double()
    rc = lib().oracle_ray(dem, H, W, spacing, obs_height, n, max_dist, prec, k, mode, t_or_p0, q0, delta,
                          _ptr(vis), _ptr(th), _ptr(zs), cap, C.byref(M), C.byref(cv), C.byref(U),
                          C.byref(e), C.byref(h))
    _check(rc, "ray")
    m = M.value
    return dict(M=m, vis=vis[:m].astype(bool), theta=th[:m].copy(), z=zs[:m].copy(), cv=cv.value,
                U=U.value, e=e.value, h=h.value)


def los_evals(rows, cols, spacing, n, max_dist):
    ev, pairs = C.c_longlong(), C.c_longlong()
    rc = lib().oracle_los_evals(rows, cols, spacing, n, max_dist, C.byref(ev), C.byref(pairs))
    _check(rc, "los_evals")
    return ev.value, pairs.value


INF = math.inf
