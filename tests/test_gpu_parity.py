"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, voxel
by voxel, bit-exact (the grid is integer data; every fp32 decision is taken
in the same precision and operation order on both sides)."""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2112_13169_amd import scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2112_13169_amd import vg


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


class GpuGrid:
    """One grid on the GPU plus an oracle twin fed the same frames."""

    def __init__(self, dims, vox_size, origin, vox_inf, init=None):
        self.dims = tuple(dims)
        gx, gy, gz = dims
        self.buf = vg.GridBuffers(dims, vox_inf)
        self.h = vg.vg_create_grid(dims, vox_size, origin, vox_inf, self.buf.loc, self.buf.spare,
                                   self.buf.scratch)
        self.vox_size = np.float32(vox_size)
        self.vox_inf = vox_inf
        self.base = np.asarray(origin, np.float32)
        self.shift_total = np.zeros(3, np.int32)
        self.ref = np.zeros((gz, gy, gx), np.uint8)
        if init is not None:
            self.write(init)

    def origin(self):
        return oracle.origin(self.base, self.shift_total, self.vox_size)

    def write(self, arr):
        arr = np.ascontiguousarray(arr, np.uint8)
        src = torch.from_numpy(arr.reshape(-1)).cuda()
        vg.vg_write_grid(self.h, src)
        torch.cuda.synchronize()
        self.ref = arr.reshape(self.ref.shape).copy()

    def read(self):
        out = torch.empty(self.ref.size, dtype=torch.uint8, device="cuda")
        vg.vg_read_grid(self.h, out)
        torch.cuda.synchronize()
        return out.cpu().numpy().reshape(self.ref.shape)

    def integrate(self, fr, pitch_pad=0):
        H, W = fr.depth.shape
        host = np.full((H, W + pitch_pad), np.nan, np.float32)
        host[:, :W] = fr.depth
        dev = torch.from_numpy(host).cuda()[:, :W]
        if fr.kind == "spinning":
            tabs = (torch.from_numpy(fr.col_tab).cuda(), torch.from_numpy(fr.row_tab).cuda())
            sensor = vg.spinning_sensor(W, H, *tabs, fr.intr["vfov"], fr.intr["depth_min"],
                                        fr.intr["depth_max"])
            vg.vg_integrate_frame(self.h, dev, sensor, vg.make_pose(fr.R, fr.t))
            return oracle.integrate_spinning(
                self.ref, self.origin(), self.vox_size, self.vox_inf, fr.depth, fr.col_tab,
                fr.row_tab, fr.intr["vfov"], fr.intr["depth_min"], fr.intr["depth_max"],
                np.asarray(fr.R, np.float32).reshape(-1), np.asarray(fr.t, np.float32))
        vg.vg_integrate_frame(self.h, dev, vg.pinhole_sensor(fr.intr), vg.make_pose(fr.R, fr.t))
        ms, st = oracle.integrate_pinhole(self.ref, self.origin(), self.vox_size, self.vox_inf,
                                          fr.depth, fr.intr, fr.R, fr.t)
        return ms, st

    def shift(self, d):
        vg.vg_shift_grid(self.h, *d)
        self.ref = oracle.shift(self.ref, d)
        self.shift_total += np.asarray(d, np.int32)

    def check(self, what):
        got = self.read()
        if not np.array_equal(got, self.ref):
            bad = np.argwhere(got != self.ref)
            z, y, x = bad[0]
            raise AssertionError(f"{what}: {len(bad)} voxels differ; first (x={x},y={y},z={z}) "
                                 f"gpu={got[z, y, x]} oracle={self.ref[z, y, x]}")

    def close(self):
        vg.vg_destroy_grid(self.h)


def _fan_rays(fr):
    return vg.vg_fan_sizes(vg.pinhole_sensor(fr.intr), fr.vox_size)[3]


@pytest.mark.parametrize("index", range(4))
def test_plain_small_frames(index):
    fr = scenes.make_frame("plain-small", index)
    _say(f"plain-small frame {index}")
    g = GpuGrid(fr.dims, fr.vox_size, fr.origin, fr.vox_inf)
    g.integrate(fr)
    g.check(f"plain-small {index}")
    g.close()


def test_plain_medium_full_size():
    """The benchmark's workload (640x480, 200x200x100 at 0.05 m, vox_inf 2),
    full grid compared."""
    fr = scenes.make_frame("plain-medium", 0)
    _say("plain-medium frame 0")
    g = GpuGrid(fr.dims, fr.vox_size, fr.origin, fr.vox_inf)
    g.integrate(fr)
    g.check("plain-medium 0")
    g.close()


def test_large_pinhole_full_size():
    """1280x720 at 0.3-12 m into 400x400x200 at 0.025 m with vox_inf 3 (32 M
    voxels, 533 355 rays), full grid compared."""
    fr = scenes.make_frame("large-pinhole", 0)
    _say("large-pinhole frame 0")
    g = GpuGrid(fr.dims, fr.vox_size, fr.origin, fr.vox_inf)
    _, st = g.integrate(fr)
    assert st["rays"] == _fan_rays(fr) == 533355
    g.check("large-pinhole 0")
    g.close()


@pytest.mark.parametrize("name,frames", [("large-pinhole", (0, 1, 2)),
                                         ("large-spinning", (0, 1))])
def test_large_sequences_with_shifts(name, frames):
    """Consecutive frames of a 2 m/s trajectory through a 2000-primitive world,
    the 400x400x200 grid re-centred on the sensor before each frame."""
    traj = scenes.make_trajectory(name, n_frames=max(frames) + 1)
    first = scenes.trajectory_frame(traj, frames[0])
    g = GpuGrid(first.dims, first.vox_size, first.origin, first.vox_inf)
    for i in frames:
        fr = first if i == frames[0] else scenes.trajectory_frame(traj, i)
        d = oracle.center_offset(fr.dims, fr.vox_size, g.origin(), fr.t)
        assert d == vg.vg_center_offset(g.h, fr.t)
        _say(f"{name} frame {i} shift {d}")
        g.shift(d)
        g.integrate(fr)
        g.check(f"{name} frame {i}")
    g.close()


@pytest.mark.parametrize("seed", range(3))
def test_batched_recipe_frames(seed):
    """Independent frames as a batch draws them: resolution up to 1280x720,
    range to U[4, 10] m, random 6-DoF pose, own grid of up to 256x256x128 at
    0.05-0.1 m, vox_inf 1-3."""
    fr = scenes.batched_frame(np.random.default_rng([scenes.SEED_BASE + 2, seed]))
    _say(f"batched-recipe seed {seed}: {fr.depth.shape} dims {fr.dims} r {fr.vox_inf}")
    g = GpuGrid(fr.dims, fr.vox_size, fr.origin, fr.vox_inf)
    g.integrate(fr)
    g.check(f"batched-recipe {seed}")
    g.close()


def test_sequence_with_recentring_shifts():
    """Frames of different poses integrated into one resident grid, the grid
    re-centred on each camera before its frame (step 5, Sec. IV-E)."""
    frames = [scenes.make_frame("plain-small", i) for i in range(4, 10)]
    g = GpuGrid(frames[0].dims, frames[0].vox_size, frames[0].origin, frames[0].vox_inf)
    rng = np.random.default_rng(0)
    for k, fr in enumerate(frames):
        # keep the cameras close to each other so the shifts keep content
        fr.t = (frames[0].t + rng.uniform(-1.0, 1.0, 3) * np.array([1, 1, 0.2])).astype(
            np.float32)
        d = oracle.center_offset(fr.dims, fr.vox_size, g.origin(), fr.t)
        assert d == vg.vg_center_offset(g.h, fr.t)
        _say(f"sequence frame {k} shift {d}")
        g.shift(d)
        g.check(f"sequence shift {k}")
        g.integrate(fr)
        g.check(f"sequence frame {k}")
    g.close()


@pytest.mark.parametrize("seed", range(3))
def test_random_six_dof_poses(seed):
    rng = np.random.default_rng(500 + seed)
    W, H = [(320, 240), (160, 120), (200, 150)][seed]
    dims = [(96, 80, 64), (128, 100, 72), (64, 64, 64)][seed]
    r = [1, 2, 3][seed]
    fr = scenes.random_pose_frame(rng, W, H, (90.0, 60.0), (0.3, 4.0), dims, 0.07, r, 40, 10)
    _say(f"six-dof seed {seed}")
    init = rng.integers(0, 3, dims[::-1]).astype(np.uint8)
    g = GpuGrid(dims, fr.vox_size, fr.origin, r, init=init)
    g.integrate(fr)
    g.check(f"six-dof {seed}")
    g.close()


def test_stage_parity_measurement_grid():
    """Writing 0xFF into the grid first exposes the measurement grid: after
    the frame, 2 = occupied, 1 = free, 0 = unknown-and-traced, 0xFF = untouched."""
    fr = scenes.make_frame("plain-small", 11)
    _say("stage parity")
    gx, gy, gz = fr.dims
    g = GpuGrid(fr.dims, fr.vox_size, fr.origin, fr.vox_inf,
                init=np.full((gz, gy, gx), 0xFF, np.uint8))
    ms, st = g.integrate(fr)
    got = g.read()
    rebuilt = np.select([got == 2, got == 1, got == 0], [oracle.OCCUPIED, oracle.FREE,
                                                         oracle.TRACED], oracle.UNKNOWN)
    assert np.array_equal(rebuilt.astype(np.uint8), ms)
    assert int((got != 0xFF).sum()) == st["updates"]
    g.close()


def test_points_input():
    fr = scenes.make_frame("plain-small", 12)
    H, W = fr.depth.shape
    ku = ((np.arange(W) - fr.intr["cx"]) / fr.intr["fx"]).astype(np.float32)
    kv = ((np.arange(H) - fr.intr["cy"]) / fr.intr["fy"]).astype(np.float32)
    pts = np.stack([fr.depth * ku[None, :], fr.depth * kv[:, None], fr.depth], -1).reshape(-1, 3)
    pts[::7] = np.nan        # invalid entries are skipped
    _say("points input")
    g = GpuGrid(fr.dims, fr.vox_size, fr.origin, fr.vox_inf)
    vg.vg_integrate_points(g.h, torch.from_numpy(np.ascontiguousarray(pts)).cuda(),
                           vg.pinhole_sensor(fr.intr), vg.make_pose(fr.R, fr.t))
    oracle.integrate_points(g.ref, g.origin(), g.vox_size, g.vox_inf, pts, fr.intr["fov_x"],
                            fr.intr["fov_y"], fr.intr["depth_max"], fr.R, fr.t)
    g.check("points")
    g.close()


@pytest.mark.parametrize("vfov", [45.0, 30.0])
def test_spinning_sensor(vfov):
    rng = np.random.default_rng(77)
    W, H = 512, 32
    col, row = scenes.spinning_tables(W, H, vfov)
    pos = np.array([0.3, -0.2, 1.2])
    R = scenes.random_rotation(rng) if vfov == 30.0 else np.eye(3)
    scene = scenes.world_scene(rng, (12.0, 12.0), 60, 20, height=(0.0, 3.0),
                               avoid=pos[None, :], keep_out=0.6)
    img = scenes.render_spinning(scene, R, pos, col, row, 0.3, 4.0, 0.005, rng)
    dims = (96, 96, 48)
    s = np.float32(0.1)
    origin = scenes.centred_origin(pos, dims, s)
    dcol, drow = torch.from_numpy(col).cuda(), torch.from_numpy(row).cuda()
    sensor = vg.spinning_sensor(W, H, dcol, drow, math.radians(vfov), 0.3, 4.0)
    rays = vg.vg_fan_sizes(sensor, s)[3]
    _say(f"spinning vfov {vfov} rays {rays}")
    g = GpuGrid(dims, s, origin, 1)
    vg.vg_integrate_frame(g.h, torch.from_numpy(img).cuda(), sensor, vg.make_pose(R, pos))
    _, st = oracle.integrate_spinning(g.ref, g.origin(), s, 1, img, col, row, math.radians(vfov),
                                      0.3, 4.0, R.astype(np.float32).reshape(-1),
                                      pos.astype(np.float32))
    assert st["rays"] == rays
    g.check(f"spinning {vfov}")
    g.close()


def test_edge_cases():
    fr = scenes.make_frame("plain-small", 13, size=(40, 30))
    # all-invalid frame: nothing occupied, the whole fan becomes free
    _say("edge: all-NaN")
    g = GpuGrid(fr.dims, fr.vox_size, fr.origin, fr.vox_inf)
    fr_nan = scenes.make_frame("plain-small", 13, size=(40, 30))
    fr_nan.depth[:] = np.nan
    g.integrate(fr_nan)
    g.check("all-NaN")
    # strided rows
    _say("edge: row pitch")
    g.integrate(fr, pitch_pad=13)
    g.check("pitch")
    g.close()
    # camera outside the grid: rays start outside and enter
    _say("edge: camera outside")
    for off in ([6.0, 0.2, 0.1], [-6.0, 0.3, 0.0], [0.1, 0.2, 3.0]):
        g = GpuGrid(fr.dims, fr.vox_size, fr.origin + np.array(off, np.float32), fr.vox_inf)
        g.integrate(fr)
        g.check(f"camera outside {off}")
        g.close()
    # vox_inf 0 and a grid smaller than the fan
    for r, dims in [(0, (30, 20, 10)), (3, (7, 5, 3)), (1, (1, 1, 1))]:
        _say(f"edge: r={r} dims={dims}")
        g = GpuGrid(dims, fr.vox_size, (fr.t - np.array(dims) * fr.vox_size / 2).astype(np.float32),
                    r)
        g.integrate(fr)
        g.check(f"r={r} dims={dims}")
        g.close()


def test_empty_image_and_empty_point_cloud():
    fr = scenes.make_frame("plain-small", 14, size=(16, 12))
    g = GpuGrid(fr.dims, fr.vox_size, fr.origin, fr.vox_inf)
    _say("edge: empty point cloud")
    vg.vg_integrate_points(g.h, torch.zeros((0, 3), dtype=torch.float32, device="cuda"),
                           vg.pinhole_sensor(fr.intr), vg.make_pose(fr.R, fr.t))
    oracle.integrate_points(g.ref, g.origin(), g.vox_size, g.vox_inf, np.zeros((0, 3)),
                            fr.intr["fov_x"], fr.intr["fov_y"], fr.intr["depth_max"], fr.R, fr.t)
    g.check("empty points")
    g.close()


def test_stamp_wraparound_over_many_frames():
    """The per-frame occupancy stamp is a byte that wraps after 255 frames."""
    fr = scenes.make_frame("plain-small", 15, size=(24, 18), dims=(24, 24, 12))
    g = GpuGrid(fr.dims, fr.vox_size, fr.origin, fr.vox_inf)
    rng = np.random.default_rng(9)
    _say("stamp wraparound")
    base = fr.depth.copy()
    for k in range(300):
        fr.depth = np.where(rng.uniform(size=base.shape) < 0.5, base,
                            np.float32(rng.uniform(0.4, 5.0))).astype(np.float32)
        g.integrate(fr)
        if k % 50 == 0 or k >= 250:
            g.check(f"frame {k}")
    g.close()


def test_shift_parity():
    rng = np.random.default_rng(21)
    dims = (37, 29, 17)
    init = rng.integers(0, 3, dims[::-1]).astype(np.uint8)
    g = GpuGrid(dims, 0.1, [0, 0, 0], 1, init=init)
    for d in [(1, 0, 0), (-3, 2, 1), (0, 0, -5), (40, 0, 0), (-2, -30, 3), (0, 0, 0)]:
        _say(f"shift {d}")
        g.shift(d)
        g.check(f"shift {d}")
    assert np.allclose(vg.vg_grid_origin(g.h), g.origin())
    g.close()


def test_determinism_and_budget():
    fr = scenes.make_frame("plain-small", 16)
    outs = []
    for _ in range(2):
        g = GpuGrid(fr.dims, fr.vox_size, fr.origin, fr.vox_inf)
        g.integrate(fr)
        outs.append(g.read())
        g.close()
    assert np.array_equal(outs[0], outs[1])
    # buffers smaller than the grid needs are refused
    gx, gy, gz = fr.dims
    small = torch.empty(vg.vg_scratch_bytes(gx, gy, gz, fr.vox_inf) - 256, dtype=torch.uint8,
                        device="cuda")
    buf = vg.GridBuffers(fr.dims, fr.vox_inf)
    with pytest.raises(vg.VgError) as ei:
        vg.vg_create_grid(fr.dims, fr.vox_size, fr.origin, fr.vox_inf, buf.loc, buf.spare, small)
    assert ei.value.status == vg.VG_ERR_BUDGET
    with pytest.raises(vg.VgError) as ei:
        vg.vg_create_grid(fr.dims, fr.vox_size, fr.origin, fr.vox_inf, buf.loc[:-32],
                          buf.spare, buf.scratch)
    assert ei.value.status == vg.VG_ERR_BUDGET


def test_profile_events_time_stages_without_changing_results():
    """The measurement hook: every stage's (start, stop) pair completes with a
    non-negative duration, the shift uses the set of the frame after it, a
    zero shift records markers, and the grid is the same as without events."""
    fr = scenes.make_frame("plain-small", 17)
    g = GpuGrid(fr.dims, fr.vox_size, fr.origin, fr.vox_inf)
    events = [torch.cuda.Event(enable_timing=True) for _ in range(2 * vg.PROFILE_EVENTS)]
    vg.vg_set_profile_events(g.h, events)
    _say("profile events")
    for k, d in enumerate([(2, -1, 0), (0, 0, 0)]):
        g.shift(d)
        g.integrate(fr)
        g.check(f"profiled frame {k}")
    torch.cuda.synchronize()
    vg.vg_set_profile_events(g.h, [])
    E = vg.PROFILE_EVENTS
    for k in range(2):
        for j, name in enumerate(vg.PROFILE_STAGES):
            ms = events[E * k + 2 * j].elapsed_time(events[E * k + 2 * j + 1])
            assert 0.0 <= ms < 1000.0, (k, name, ms)
    g.close()


def test_ring_buffer_wraps_and_resolves_across_the_seam():
    """Many small shifts whose ring offsets wrap round the grid several times,
    with frames integrated in between (the merge writes across the ring's
    seam), reads to device and to host memory, and a checkpoint written back
    (the ring restarts at 0) -- all against the oracle."""
    fr = scenes.make_frame("plain-small", 18, size=(64, 48), dims=(45, 38, 21))
    g = GpuGrid(fr.dims, fr.vox_size, fr.origin, fr.vox_inf)
    rng = np.random.default_rng(31)
    for k in range(24):
        d = tuple(int(v) for v in rng.integers(-9, 10, 3))
        _say(f"ring step {k} shift {d}")
        g.shift(d)
        fr.t = (g.origin() + np.asarray(fr.dims, np.float32) * g.vox_size *
                rng.uniform(0.3, 0.7, 3).astype(np.float32)).astype(np.float32)
        g.integrate(fr)
        g.check(f"ring step {k}")
        if k % 6 == 5:
            host = torch.empty(g.ref.size, dtype=torch.uint8, pin_memory=True)
            vg.vg_read_grid(g.h, host)
            torch.cuda.synchronize()
            assert np.array_equal(host.numpy().reshape(g.ref.shape), g.ref), f"host read {k}"
        if k == 11:
            g.write(g.ref)          # checkpoint round trip: the ring restarts at 0
            g.check("after write")
    g.close()


def test_shift_fused_into_the_frame():
    """vg_integrate_frame_shifted (the shift's clear inside the walk launch)
    against the oracle's shift-then-integrate: small shifts whose ring offsets
    wrap (slabs on every axis), a shift past the grid (the whole grid clears),
    a zero shift; and an out-of-range shift is refused with the grid untouched."""
    fr = scenes.make_frame("plain-small", 21, size=(64, 48), dims=(45, 38, 21))
    g = GpuGrid(fr.dims, fr.vox_size, fr.origin, fr.vox_inf)
    rng = np.random.default_rng(41)
    shifts = [tuple(int(v) for v in rng.integers(-9, 10, 3)) for _ in range(10)]
    shifts[4] = (0, 0, 0)
    shifts[7] = (60, -3, 2)          # past the grid along x
    for k, d in enumerate(shifts):
        _say(f"fused shift {k} {d}")
        g.ref = oracle.shift(g.ref, d)
        g.shift_total += np.asarray(d, np.int32)
        fr.t = (g.origin() + np.asarray(fr.dims, np.float32) * g.vox_size *
                rng.uniform(0.3, 0.7, 3).astype(np.float32)).astype(np.float32)
        dev = torch.from_numpy(fr.depth).cuda()
        vg.vg_integrate_frame_shifted(g.h, dev, vg.pinhole_sensor(fr.intr),
                                      vg.make_pose(fr.R, fr.t), d)
        oracle.integrate_pinhole(g.ref, g.origin(), g.vox_size, g.vox_inf, fr.depth, fr.intr,
                                 fr.R, fr.t, want_ms=False)
        g.check(f"fused shift {k}")
    before = g.read()
    with pytest.raises(vg.VgError):
        vg.vg_integrate_frame_shifted(g.h, torch.from_numpy(fr.depth).cuda(),
                                      vg.pinhole_sensor(fr.intr), vg.make_pose(fr.R, fr.t),
                                      (1 << 25, 0, 0))
    assert np.array_equal(g.read(), before)
    assert np.array_equal(vg.vg_grid_origin(g.h), g.origin())
    g.close()


def test_shift_fused_into_the_medium_frame():
    """The benchmark's step on full-size frames: random poses, so every shift
    clears the whole grid inside the walk launch."""
    frames = [scenes.make_frame("plain-medium", k) for k in (2, 3)]
    f0 = frames[0]
    g = GpuGrid(f0.dims, f0.vox_size, f0.origin, f0.vox_inf)
    for k, fr in enumerate(frames):
        d = vg.vg_center_offset(g.h, fr.t)
        _say(f"medium fused shift {d}")
        g.ref = oracle.shift(g.ref, d)
        g.shift_total += np.asarray(d, np.int32)
        vg.vg_integrate_frame_shifted(g.h, torch.from_numpy(fr.depth).cuda(),
                                      vg.pinhole_sensor(fr.intr), vg.make_pose(fr.R, fr.t), d)
        oracle.integrate_pinhole(g.ref, g.origin(), g.vox_size, g.vox_inf, fr.depth, fr.intr,
                                 fr.R, fr.t, want_ms=False)
        g.check(f"medium fused {k}")
    g.close()


@pytest.mark.parametrize("index", range(3))
def test_paper_standard_frames(index):
    """The paper's standard parameters (320x240, 85 x 101 deg, 6.5 m, 100 x 100
    x 20 voxels of 0.15 m, vox_inf 2; 8 295 rays) on the synthetic scene."""
    fr = scenes.make_frame("paper-standard", index)
    _say(f"paper-standard frame {index}")
    g = GpuGrid(fr.dims, fr.vox_size, fr.origin, fr.vox_inf)
    _, st = g.integrate(fr)
    assert st["rays"] == _fan_rays(fr) == 8295
    g.check(f"paper-standard {index}")
    g.close()
