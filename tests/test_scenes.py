"""The seeded input generator: its culled renderers equal brute-force casting of
every primitive against every pixel (culling only saves time), and the
workload recipes give frames of the stated shapes."""
import math

import numpy as np
import pytest

from paper_2112_13169_amd import scenes


def _brute(scene, t, dirs, dmin, dmax):
    z = scenes._cast(scene, np.asarray(t, float), dirs)
    return np.where((z >= dmin) & (z <= dmax), z, np.nan).astype(np.float32)


def _pinhole_dirs(intr, R):
    ku, kv = scenes._pixel_dirs(intr)
    cam = np.stack(np.broadcast_arrays(ku[None, :], kv[:, None], np.ones((1, 1))), axis=-1)
    return cam @ np.asarray(R, float).T


@pytest.mark.parametrize("frame", [0, 37])
def test_pinhole_culling_matches_brute_force_in_a_world(frame):
    traj = scenes.make_trajectory("large-pinhole", n_frames=40)
    intr = scenes.pinhole_intrinsics(96, 54, 90.0, 60.0, 0.3, 12.0)
    R = scenes.level_camera(traj.yaws[frame])
    t = traj.positions[frame]
    got = scenes.render_pinhole(traj.scene, R, t, intr)
    want = _brute(traj.scene, t, _pinhole_dirs(intr, R), 0.3, 12.0)
    assert np.array_equal(got, want, equal_nan=True)
    assert 0.3 < np.isfinite(got).mean() <= 1.0


def test_pinhole_culling_matches_brute_force_six_dof():
    rng = np.random.default_rng(4)
    intr = scenes.pinhole_intrinsics(80, 60, 90.0, 60.0, 0.3, 6.0)
    for _ in range(3):
        R = scenes.random_rotation(rng)
        t = np.array([0.0, 0.0, rng.uniform(0.5, 3.0)])
        scene = scenes.world_scene(rng, (16.0, 16.0), 120, 40, height=(0.0, 4.0),
                                   avoid=t[None, :], keep_out=0.4)
        got = scenes.render_pinhole(scene, R, t, intr)
        want = _brute(scene, t, _pinhole_dirs(intr, R), 0.3, 6.0)
        assert np.array_equal(got, want, equal_nan=True)


@pytest.mark.parametrize("seed", range(2))
def test_spinning_culling_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    W, H = 256, 24
    col, row = scenes.spinning_tables(W, H, 45.0)
    pos = np.array([0.3, -0.2, 1.5])
    scene = scenes.world_scene(rng, (30.0, 30.0), 300, 100, height=(0.0, 8.0),
                               avoid=pos[None, :], keep_out=0.6)
    R = scenes.random_rotation(rng) if seed else np.eye(3)
    got = scenes.render_spinning(scene, R, pos, col, row, 0.3, 12.0)
    c, r = col.astype(float), row.astype(float)
    cam = np.stack([r[0::2, None] * c[None, 0::2], r[0::2, None] * c[None, 1::2],
                    np.broadcast_to(r[1::2, None], (H, W))], axis=-1)
    want = _brute(scene, pos, cam @ R.T, 0.3, 12.0)
    assert np.array_equal(got, want, equal_nan=True)


def test_sequence_and_batch_recipes():
    traj = scenes.make_trajectory("served", robot=3, n_frames=30)
    step = np.linalg.norm(np.diff(traj.positions[:, :2], axis=0), axis=1)
    assert np.allclose(step, 2.0 / 30.0, atol=1e-9)           # 2 m/s at 30 Hz
    fr = scenes.trajectory_frame(traj, 5, robot=3)
    assert fr.depth.shape == (480, 640) and fr.dims == (200, 200, 100) and fr.vox_inf == 2
    sp = scenes.make_trajectory("large-spinning", n_frames=3)
    fs = scenes.trajectory_frame(sp, 1)
    assert fs.kind == "spinning" and fs.depth.shape == (128, 2048)
    assert math.isclose(fs.intr["vfov"], math.radians(45.0))
    rng = np.random.default_rng(8)
    for _ in range(4):
        fb = scenes.batched_frame(rng, max_side=120)
        assert (fb.depth.shape[1], fb.depth.shape[0]) in [(320, 240), (640, 480), (848, 480),
                                                          (1280, 720)]
        assert fb.vox_inf in (1, 2, 3) and 0.05 <= fb.vox_size <= 0.1
        assert 4.0 <= fb.intr["depth_max"] <= 10.0
        gx, gy, gz = fb.dims
        assert gx == gy and 100 <= gx <= 120 and 100 <= gz <= 120
