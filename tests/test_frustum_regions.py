"""The frame regions of vg_frustum.h, built for the host, against the CPU
oracle: every voxel a frame gives a measurement state (occupied, free or
traced, Alg. 1-2) lies in a column run the merge reads, and every measured
point's voxel in a run the x dilation reads -- for level and random 6-DoF
cameras, inside and outside their grids, vox_inf 0-3.  The merge may then
skip the other runs without changing a voxel (the GPU parity tests check the
kernels themselves)."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2112_13169_amd import scenes

HERE = os.path.dirname(os.path.abspath(__file__))
P = ctypes.c_void_p


@pytest.fixture(scope="module")
def fr(tmp_path_factory):
    so = str(tmp_path_factory.mktemp("frustum") / "frustum_check.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
                           "-Wall", "-shared", "-fPIC", "-o", so,
                           os.path.join(HERE, "frustum_check.cpp")])
    L = ctypes.CDLL(so)
    i32 = ctypes.c_int32
    L.fr_marks_outside.argtypes = [P, i32, i32, i32, P, P, i32, i32, i32, i32, i32, P, i32, P]
    L.fr_marks_outside.restype = ctypes.c_int64
    L.fr_seeds_outside.argtypes = [P, ctypes.c_int64, P, P, i32, i32, i32, i32, i32, P, i32]
    L.fr_seeds_outside.restype = ctypes.c_int64
    return L


def _p(a):
    return a.ctypes.data_as(P)


def _seed_voxels(f, origin):
    """Voxels of the valid measured points, as the seed pass computes them:
    fp32 slopes from double, camera point (d ku, d kv, d), the fixed-order
    transform, floor of the fp32 quotient; points whose cube cannot reach the
    grid dropped."""
    intr = f.intr
    H, W = f.depth.shape
    ku = ((np.arange(W, dtype=np.float64) - intr["cx"]) / intr["fx"]).astype(np.float32)
    kv = ((np.arange(H, dtype=np.float64) - intr["cy"]) / intr["fy"]).astype(np.float32)
    d = f.depth
    ok = (d >= np.float32(intr["depth_min"])) & (d <= np.float32(intr["depth_max"]))
    vv, uu = np.nonzero(ok)
    dd = d[vv, uu].astype(np.float32)
    pc = (dd * ku[uu], dd * kv[vv], dd)
    R = np.asarray(f.R, np.float32).reshape(3, 3)
    tv = (np.asarray(f.t, np.float32) - np.asarray(origin, np.float32)).astype(np.float32)
    s = np.float32(f.vox_size)
    q = []
    for i in range(3):
        a = R[i, 0] * pc[0]
        b = R[i, 1] * pc[1]
        pv = ((a + b) + R[i, 2] * pc[2]) + tv[i]
        q.append(np.floor(pv / s))
    q = np.stack(q, 1)
    r = f.vox_inf
    keep = np.all((q >= -r) & (q <= np.asarray(f.dims, np.float32) - 1 + r), axis=1)
    return np.ascontiguousarray(q[keep].astype(np.int32))


def _check(L, f, origin):
    intr = f.intr
    vd, hw, hh = oracle.fan_sizes(intr["depth_max"], f.vox_size, intr["fov_x"], intr["fov_y"])
    tv = (np.asarray(f.t, np.float32) - np.asarray(origin, np.float32)).astype(np.float32)
    o = (tv / np.float32(f.vox_size)).astype(np.float32)
    H, W = f.depth.shape
    k = [np.float32((0.0 - intr["cx"]) / intr["fx"]), np.float32((W - 1.0 - intr["cx"]) / intr["fx"]),
         np.float32((0.0 - intr["cy"]) / intr["fy"]), np.float32((H - 1.0 - intr["cy"]) / intr["fy"])]
    slopes = np.array([min(k[0], k[1]), max(k[0], k[1]), min(k[2], k[3]), max(k[2], k[3])],
                      np.float32)
    R = np.ascontiguousarray(np.asarray(f.R, np.float32).reshape(-1))
    gx, gy, gz = f.dims
    loc = np.zeros((gz, gy, gx), np.uint8)
    ms, _ = oracle.integrate_pinhole(loc, origin, f.vox_size, f.vox_inf, f.depth, intr, f.R, f.t)
    ms = np.ascontiguousarray(ms)
    admitted = np.zeros(1, np.int64)
    bad = L.fr_marks_outside(_p(ms), gx, gy, gz, _p(R), _p(o), 1, vd, hw, hh, 1, _p(slopes),
                             f.vox_inf, _p(admitted))
    q = _seed_voxels(f, origin)
    bad_seeds = L.fr_seeds_outside(_p(q), len(q), _p(R), _p(o), 1, vd, hw, hh, 1, _p(slopes),
                                   f.vox_inf)
    marked = int(np.count_nonzero(ms))
    assert marked > 0 and len(q) > 0
    return bad, bad_seeds, int(admitted[0]), marked


@pytest.mark.parametrize("index", range(4))
def test_level_cameras(fr, index):
    f = scenes.make_frame("plain-medium", index, size=(320, 240))
    bad, bad_seeds, admitted, marked = _check(fr, f, f.origin)
    assert (bad, bad_seeds) == (0, 0)
    # the regions leave out much of the grid
    assert admitted < 0.6 * np.prod(f.dims), admitted


@pytest.mark.parametrize("seed", range(6))
def test_random_poses_and_inflation(fr, seed):
    rng = np.random.default_rng(500 + seed)
    f = scenes.random_pose_frame(rng, 160, 120, (90.0, 60.0), (0.3, 5.0), (96, 80, 64), 0.08,
                                 seed % 4, 60, 15)
    bad, bad_seeds, _, _ = _check(fr, f, f.origin)
    assert (bad, bad_seeds) == (0, 0)


@pytest.mark.parametrize("offset", [(5.0, 0.3, 0.1), (-4.0, 2.5, -1.0), (0.2, 0.1, 3.5)])
def test_cameras_outside_their_grids(fr, offset):
    f = scenes.make_frame("plain-small", 80, size=(80, 60))
    origin = (f.origin + np.asarray(offset, np.float32)).astype(np.float32)
    bad, bad_seeds, _, _ = _check(fr, f, origin)
    assert (bad, bad_seeds) == (0, 0)


def test_wide_fov_and_off_centre_principal_point(fr):
    rng = np.random.default_rng(77)
    f = scenes.random_pose_frame(rng, 120, 90, (120.0, 100.0), (0.3, 4.0), (80, 80, 60), 0.1, 2,
                                 40, 10)
    f.intr = dict(f.intr, cx=f.intr["cx"] + 17.0, cy=f.intr["cy"] - 9.0)
    bad, bad_seeds, _, _ = _check(fr, f, f.origin)
    assert (bad, bad_seeds) == (0, 0)


@pytest.mark.parametrize("yaw", [0.0, np.pi / 2, np.pi, np.pi / 2 + 1e-6, -1e-7, np.pi / 4])
def test_axis_aligned_and_nearly_aligned_cameras(fr, yaw):
    """Planes whose normals are (nearly) perpendicular to the grid's x axis:
    their bounds are tested per row, not per column."""
    f = scenes.make_frame("plain-medium", 9, size=(160, 120), yaw=yaw, dims=(120, 110, 60))
    bad, bad_seeds, _, _ = _check(fr, f, f.origin)
    assert (bad, bad_seeds) == (0, 0)
