"""CPU-side checks of the C-ABI library: it loads, exports every symbol that
include/vg.h declares, and its host-only logic (argument validation, ray-fan
sizes, scratch sizing, status strings) behaves as documented.  No kernel is
launched here."""
import ctypes
import math

import numpy as np
import pytest

import oracle
from paper_2112_13169_amd import scenes
from paper_2112_13169_amd import vg


def test_library_loads_and_exports_every_declared_symbol():
    L = vg.lib()
    declared = vg.header_symbols()
    assert len(declared) >= 12
    for name in declared:
        assert hasattr(L, name), name


@pytest.mark.parametrize("wl", ["plain-small", "plain-medium", "large-pinhole"])
def test_fan_sizes_match_oracle(wl):
    fr = scenes.make_frame(wl, 0, size=(16, 12))
    s = vg.pinhole_sensor(fr.intr)
    vd, hw, hh, rays = vg.vg_fan_sizes(s, fr.vox_size)
    assert (vd, hw, hh) == oracle.fan_sizes(fr.intr["depth_max"], fr.vox_size, fr.intr["fov_x"],
                                            fr.intr["fov_y"])
    assert rays == (2 * hw + 1) * (2 * hh + 1)


def test_paper_standard_fan_through_the_library():
    intr = scenes.pinhole_intrinsics(320, 240, 85.0, 101.0, 0.3, 6.5)
    vd, hw, hh, rays = vg.vg_fan_sizes(vg.pinhole_sensor(intr), np.float32(0.15))
    assert (vd, 2 * hw + 1, 2 * hh + 1, rays) == (43, 79, 105, 8295)


def test_spinning_fan_matches_oracle():
    fake = ctypes.c_float(0.0)
    s = vg.vg_sensor(vg.VG_SPINNING, 0, 0, 0, 0, 0, 0, 0, 0, math.radians(45.0), 0.3, 12.0,
                     ctypes.addressof(fake), ctypes.addressof(fake))
    vd, hw, hh, rays = vg.vg_fan_sizes(s, np.float32(0.025))
    assert vd == 480
    n, hz = oracle.spin_ray_count(vd, math.tan(math.radians(22.5)), with_table=True)
    assert rays == n and hh == hz.max()


def test_fan_sizes_rejects_bad_sensors():
    intr = scenes.pinhole_intrinsics(16, 12, 90.0, 60.0, 0.3, 5.0)
    s = vg.pinhole_sensor(intr)
    with pytest.raises(vg.VgError):
        vg.vg_fan_sizes(s, 0.0)
    s.fov_x = math.pi
    with pytest.raises(vg.VgError):
        vg.vg_fan_sizes(s, 0.1)
    s = vg.pinhole_sensor(intr)
    s.depth = float("nan")
    with pytest.raises(vg.VgError):
        vg.vg_fan_sizes(s, 0.1)
    s = vg.pinhole_sensor(intr)
    s.kind = 7
    with pytest.raises(vg.VgError):
        vg.vg_fan_sizes(s, 0.1)


def test_scratch_and_grid_bytes():
    a = vg.vg_scratch_bytes(100, 100, 50, 2)
    c = vg.vg_scratch_bytes(100, 100, 50, 3)
    assert a > 128 * 100 * 50 and c > a
    assert vg.vg_grid_bytes(100, 100, 50) == 128 * 100 * 50     # rows padded to 32 voxels
    assert vg.vg_grid_bytes(200, 200, 100) == 224 * 200 * 100
    assert vg.vg_scratch_bytes(0, 1, 1, 1) == 0
    assert vg.vg_grid_bytes(2048, 2048, 1024) == 0               # >= 2^31 bytes
    assert vg.vg_grid_bytes(1024, 1024, 1024) == 0               # = 2^30: the limit
    assert vg.vg_grid_bytes(1024, 1024, 1023) == 1024 * 1024 * 1023
    assert vg.vg_scratch_bytes(8, 8, 8, 17) == 0                 # vox_inf above 16


def test_create_grid_argument_errors_leave_no_handle():
    L = vg.lib()
    P = ctypes.c_void_p
    org = (ctypes.c_float * 3)(0, 0, 0)
    fake_a, fake_b, fake_s = P(0x100000), P(0x200000), P(0x300000)
    big = vg.vg_scratch_bytes(4, 4, 4, 1)
    gb = vg.vg_grid_bytes(4, 4, 4)

    def create(gx=4, gy=4, gz=4, s=0.1, origin=org, r=1, a=fake_a, b=fake_b, nb=gb,
               scr=fake_s, nbytes=big):
        h = P(1234)
        st = L.vg_create_grid(gx, gy, gz, s, origin, r, a, b, nb, scr, nbytes, None,
                              ctypes.byref(h))
        return st, h.value

    for kw in [dict(gx=0), dict(gz=-1), dict(gx=2048, gy=2048, gz=1024), dict(s=0.0),
               dict(s=float("nan")), dict(r=-1), dict(r=17), dict(gy=70000),
               dict(origin=(ctypes.c_float * 3)(0, float("inf"), 0)), dict(a=P(0)),
               dict(scr=P(0)), dict(scr=P(0x300010)), dict(a=P(0x100004))]:
        st, h = create(**kw)
        assert st == vg.VG_ERR_ARG and h is None, kw
    for kw in [dict(nbytes=100), dict(nb=gb - 1)]:
        st, h = create(**kw)
        assert st == vg.VG_ERR_BUDGET and h is None, kw
    assert L.vg_create_grid(4, 4, 4, 0.1, org, 1, fake_a, fake_b, gb, fake_s, big, None,
                            None) == vg.VG_ERR_ARG


def test_null_handle_calls_are_argument_errors():
    L = vg.lib()
    s = vg.pinhole_sensor(scenes.pinhole_intrinsics(16, 12, 90.0, 60.0, 0.3, 5.0))
    pose = vg.make_pose(np.eye(3), [0, 0, 0])
    assert L.vg_integrate_frame(None, None, 64, ctypes.byref(s), ctypes.byref(pose),
                                None) == vg.VG_ERR_ARG
    assert L.vg_shift_grid(None, 1, 0, 0, None) == vg.VG_ERR_ARG
    assert L.vg_integrate_frame_shifted(None, None, 64, ctypes.byref(s), ctypes.byref(pose),
                                        1, 0, 0, None) == vg.VG_ERR_ARG
    assert L.vg_read_grid(None, None, 1, None) == vg.VG_ERR_ARG
    assert L.vg_destroy_grid(None) == vg.VG_ERR_ARG
    assert vg.vg_status_str(vg.VG_ERR_BUDGET) == "scratch workspace too small"
    assert vg.vg_status_str(12345) == "unknown status"


def test_batch_argument_errors_before_any_device_work():
    L = vg.lib()
    P = ctypes.c_void_p
    ws = P(0x400000)
    need = vg.vg_batch_workspace_bytes(2)
    assert need > 0 and vg.vg_batch_workspace_bytes(2) < vg.vg_batch_workspace_bytes(3)
    assert vg.vg_batch_workspace_bytes(-1) == 0 and vg.vg_batch_workspace_bytes(4097) == 0
    frames = (vg.vg_frame * 2)()
    assert L.vg_integrate_batch(frames, 0, None, 0, None) == vg.VG_OK       # nothing to do
    assert L.vg_integrate_batch(frames, -1, ws, need, None) == vg.VG_ERR_ARG
    assert L.vg_integrate_batch(None, 2, ws, need, None) == vg.VG_ERR_ARG
    assert L.vg_integrate_batch(frames, 2, None, need, None) == vg.VG_ERR_ARG
    assert L.vg_integrate_batch(frames, 2, P(0x400010), need, None) == vg.VG_ERR_ARG
    assert L.vg_integrate_batch(frames, 2, ws, need - 1, None) == vg.VG_ERR_BUDGET
    # a frame without a grid is an argument error (checked before any launch)
    assert L.vg_integrate_batch(frames, 2, ws, need, None) == vg.VG_ERR_ARG
    assert ctypes.sizeof(vg.vg_frame) == 184


def test_ray_tile_argument_range():
    L = vg.lib()
    assert L.vg_set_ray_tile(None, 3) == vg.VG_ERR_ARG
