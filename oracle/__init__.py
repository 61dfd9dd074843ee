"""ctypes binding of the plain C CPU oracle (vg_oracle.c).

Test infrastructure only: the test suite, the smoke check and the CPU-baseline
leg of the benchmark use this module.  The GPU library never imports it, and it
imports nothing from the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vg_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-Wall", "-Wextra"]

UNKNOWN, FREE, OCCUPIED, TRACED, OUTSIDE = 0, 1, 2, 3, 255


def build() -> str:
    """Compile liboracle.so with gcc (fp32 ops rounded as written: no contraction)."""
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i32, i64, f32, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double
        L.og_fan_sizes.argtypes = [f32, f32, f64, f64, P]
        L.og_fan_sizes.restype = ctypes.c_int
        L.og_spin_ray_count.argtypes = [i32, f64, P]
        L.og_spin_ray_count.restype = i64
        L.og_origin.argtypes = [P, P, f32, P]
        L.og_quantize.argtypes = [P, P, f32, P, P]
        L.og_trace_ray.argtypes = [P, P, i64, i32, i32, i32, P, P, P, i64]
        L.og_trace_ray.restype = i64
        L.og_integrate_pinhole.argtypes = [i32, i32, i32, f32, P, i32, P, P, P, i32, i32,
                                           f64, f64, f64, f64, f64, f64, f32, f32, P, P, P]
        L.og_integrate_pinhole.restype = ctypes.c_int
        L.og_integrate_spinning.argtypes = [i32, i32, i32, f32, P, i32, P, P, P, i32, i32,
                                            P, P, f64, f32, f32, P, P, P]
        L.og_integrate_spinning.restype = ctypes.c_int
        L.og_integrate_points.argtypes = [i32, i32, i32, f32, P, i32, P, P, P, i64,
                                          f64, f64, f32, P, P, P]
        L.og_integrate_points.restype = ctypes.c_int
        L.og_merge.argtypes = [i64, P, P]
        L.og_shift.argtypes = [i32, i32, i32, P, P, i32, i32, i32]
        L.og_center_offset.argtypes = [i32, i32, i32, f32, P, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f32(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    if n is not None:
        assert a.size == n
    return a


def fan_sizes(depth: float, vox_size: float, fov_x: float, fov_y: float):
    """(vox_depth, hw, hh) or None when out of range."""
    out = np.zeros(3, np.int32)
    rc = lib().og_fan_sizes(depth, vox_size, fov_x, fov_y, _p(out))
    return None if rc else tuple(int(v) for v in out)


def spin_ray_count(vox_depth: int, tan_half_vfov: float, with_table: bool = False):
    hz = np.zeros(8 * vox_depth, np.int32) if with_table else None
    n = lib().og_spin_ray_count(vox_depth, tan_half_vfov, _p(hz) if with_table else None)
    return (int(n), hz) if with_table else int(n)


def origin(base, shift, vox_size):
    out = np.zeros(3, np.float32)
    lib().og_origin(_p(_f32(base, 3)), _p(np.asarray(shift, np.int32)), vox_size, _p(out))
    return out


def quantize(R, tv, vox_size, pc):
    q = np.zeros(3, np.float32)
    lib().og_quantize(_p(_f32(R, 9)), _p(_f32(tv, 3)), vox_size, _p(_f32(pc, 3)), _p(q))
    return q


def trace_ray(o, d, m2, dims, ms=None, max_out=1 << 16):
    """One Alg. 2 walk.  Returns (voxels[n,3], values[n]) over every walk step."""
    gx, gy, gz = dims
    xyz = np.zeros((max_out, 3), np.int32)
    val = np.zeros(max_out, np.uint8)
    msp = None
    if ms is not None:
        assert ms.dtype == np.uint8 and ms.flags.c_contiguous and ms.size == gx * gy * gz
        msp = _p(ms)
    n = lib().og_trace_ray(_p(_f32(o, 3)), _p(_f32(d, 3)), int(m2), gx, gy, gz, msp,
                           _p(xyz), _p(val), max_out)
    if n < 0:
        raise ValueError("invalid ray")
    n = min(n, max_out)
    return xyz[:n].copy(), val[:n].copy()


def _grid_args(loc):
    assert loc.dtype == np.uint8 and loc.ndim == 3 and loc.flags.c_contiguous
    gz, gy, gx = loc.shape
    return gx, gy, gz


def integrate_pinhole(loc, origin_w, vox_size, vox_inf, depth, intr, R, t, want_ms=True):
    """Steps 1-4 on one pinhole z-depth image.  loc: uint8[gz, gy, gx], updated
    in place.  intr: dict(fx, fy, cx, cy, fov_x, fov_y, depth_min, depth_max).
    Returns (ms or None, stats dict)."""
    gx, gy, gz = _grid_args(loc)
    depth = np.ascontiguousarray(depth, dtype=np.float32)
    H, W = depth.shape
    ms = np.zeros_like(loc) if want_ms else None
    st = np.zeros(5, np.int64)
    rc = lib().og_integrate_pinhole(
        gx, gy, gz, vox_size, _p(_f32(origin_w, 3)), vox_inf, _p(loc),
        _p(ms) if want_ms else None, _p(depth), W, H,
        intr["fx"], intr["fy"], intr["cx"], intr["cy"], intr["fov_x"], intr["fov_y"],
        intr["depth_min"], intr["depth_max"], _p(_f32(R, 9)), _p(_f32(t, 3)), _p(st))
    if rc:
        raise ValueError("oracle rejected the frame")
    return ms, dict(updates=int(st[0]), steps=int(st[1]), occupied=int(st[2]), rays=int(st[3]),
                    steps_after_hit=int(st[4]))


def integrate_spinning(loc, origin_w, vox_size, vox_inf, rng_img, col_tab, row_tab, vfov,
                       depth_min, depth_max, R, t, want_ms=True):
    gx, gy, gz = _grid_args(loc)
    rng_img = np.ascontiguousarray(rng_img, dtype=np.float32)
    H, W = rng_img.shape
    col_tab = _f32(col_tab, 2 * W)
    row_tab = _f32(row_tab, 2 * H)
    ms = np.zeros_like(loc) if want_ms else None
    st = np.zeros(5, np.int64)
    rc = lib().og_integrate_spinning(
        gx, gy, gz, vox_size, _p(_f32(origin_w, 3)), vox_inf, _p(loc),
        _p(ms) if want_ms else None, _p(rng_img), W, H, _p(col_tab), _p(row_tab),
        vfov, depth_min, depth_max, _p(_f32(R, 9)), _p(_f32(t, 3)), _p(st))
    if rc:
        raise ValueError("oracle rejected the frame")
    return ms, dict(updates=int(st[0]), steps=int(st[1]), occupied=int(st[2]), rays=int(st[3]),
                    steps_after_hit=int(st[4]))


def integrate_points(loc, origin_w, vox_size, vox_inf, points, fov_x, fov_y, depth, R, t,
                     want_ms=True):
    gx, gy, gz = _grid_args(loc)
    pts = np.ascontiguousarray(points, dtype=np.float32).reshape(-1, 3)
    ms = np.zeros_like(loc) if want_ms else None
    st = np.zeros(5, np.int64)
    rc = lib().og_integrate_points(
        gx, gy, gz, vox_size, _p(_f32(origin_w, 3)), vox_inf, _p(loc),
        _p(ms) if want_ms else None, _p(pts), pts.shape[0], fov_x, fov_y, depth,
        _p(_f32(R, 9)), _p(_f32(t, 3)), _p(st))
    if rc:
        raise ValueError("oracle rejected the frame")
    return ms, dict(updates=int(st[0]), steps=int(st[1]), occupied=int(st[2]), rays=int(st[3]),
                    steps_after_hit=int(st[4]))


def merge(ms, loc):
    assert ms.shape == loc.shape and ms.dtype == loc.dtype == np.uint8
    lib().og_merge(ms.size, _p(np.ascontiguousarray(ms)), _p(loc))


def shift(loc, d):
    gx, gy, gz = _grid_args(loc)
    out = np.empty_like(loc)
    lib().og_shift(gx, gy, gz, _p(loc), _p(out), int(d[0]), int(d[1]), int(d[2]))
    return out


def center_offset(dims_xyz, vox_size, origin_w, t_w_c):
    gx, gy, gz = dims_xyz
    d = np.zeros(3, np.int32)
    lib().og_center_offset(gx, gy, gz, vox_size, _p(_f32(origin_w, 3)), _p(_f32(t_w_c, 3)), _p(d))
    return tuple(int(v) for v in d)
