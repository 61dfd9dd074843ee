"""GPU parity of the code paths chosen by size: inflation radii past the tiled
dilation (vox_inf 4 .. 16), occupied cubes stamped directly at those radii,
rows wider than the tiled dilation takes (512 voxels), batch rounds of grids
257-512 voxels wide (16-word tiles) and batch rounds with vox_inf > 3 (the
untiled batch dilation); and an fp32 canary of the transform, quantisation and
walk set-up (Alg. 1 transform and quantise, Sec. IV-B; Alg. 2 set-up,
Sec. IV-C): single points within a few ulps of voxel boundaries under generic
rotations, and denormal coordinates.  Every case is compared with the CPU
oracle voxel for voxel."""
import sys

import numpy as np
import pytest

import oracle
from paper_2112_13169_amd import scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2112_13169_amd import vg
    from test_gpu_batch import DevFrame, Twin, _workspace

# A frame walked on its own stamps each point's cube directly when its points
# times (2 vox_inf + 1)^3 stay at or below this many stores (one launch);
# above it the separable dilation runs.
DIRECT_STORES = 16 << 20
# The tiled y/z dilation takes rows of at most 16 words (512 voxels) and
# vox_inf <= 3; otherwise the untiled kernel runs.
TILED_MAX_WORDS = 16
TILED_MAX_INF = 3


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _words(gx):
    return (gx + 31) // 32


def _stores(fr):
    H, W = fr.depth.shape
    return W * H * (2 * fr.vox_inf + 1) ** 3


def _one_frame(fr, what):
    t = Twin(fr.dims, fr.vox_size, fr.origin, fr.vox_inf)
    d = DevFrame(t, fr)
    vg.vg_integrate_frame(t.h, d.data, vg.pinhole_sensor(fr.intr), vg.make_pose(fr.R, fr.t))
    t.oracle_frame(fr)
    t.check(what)
    t.close()


@pytest.mark.parametrize("vox_inf,size", [(4, (160, 120)), (16, (20, 20))])
def test_direct_stamping_at_large_vox_inf(vox_inf, size):
    """Cubes of 9^3 and 33^3 voxels stamped per point (one launch)."""
    fr = scenes.make_frame("plain-small", 80 + vox_inf, size=size, vox_inf=vox_inf)
    assert _stores(fr) <= DIRECT_STORES
    _say(f"direct stamping vox_inf {vox_inf} {size}")
    _one_frame(fr, f"direct vox_inf {vox_inf}")


@pytest.mark.parametrize("workload,vox_inf,size", [("plain-medium", 4, None),
                                                   ("plain-small", 16, None),
                                                   ("plain-medium", 6, (320, 240))])
def test_separable_dilation_at_large_vox_inf(workload, vox_inf, size):
    """The untiled y/z dilation (vox_inf > 3) after the x dilation's widest
    windows (vox_inf 16: 32 neighbours of a 32-voxel word)."""
    fr = scenes.make_frame(workload, 90 + vox_inf, vox_inf=vox_inf, size=size)
    assert _stores(fr) > DIRECT_STORES and vox_inf > TILED_MAX_INF
    _say(f"separable dilation {workload} vox_inf {vox_inf}")
    _one_frame(fr, f"separable vox_inf {vox_inf}")


@pytest.mark.parametrize("dims,vox_inf", [((600, 120, 60), 2), ((1000, 64, 40), 3),
                                          ((530, 96, 48), 5)])
def test_rows_wider_than_the_tiled_dilation(dims, vox_inf):
    """Grids wider than 512 voxels take the untiled y/z dilation; the merge's
    16-column chunks run over 19 .. 32 words per row."""
    fr = scenes.make_frame("plain-medium", 100 + dims[0], dims=dims, vox_inf=vox_inf)
    assert _words(dims[0]) > TILED_MAX_WORDS and _stores(fr) > DIRECT_STORES
    _say(f"wide grid {dims} vox_inf {vox_inf}")
    _one_frame(fr, f"wide grid {dims}")


# 8-deep y/z dilation tiles are used where a launch has at least this many
# of them (256 / kw row slots along y, 8 slices along z); 2-deep ones elsewhere.
DEEP_TILE_MIN = 512


def _deep_tiles(dims):
    ty = 256 // (8 if _words(dims[0]) <= 8 else 16)
    return -(-dims[1] // ty) * -(-dims[2] // 8)


@pytest.mark.parametrize("dims,vox_inf", [((64, 1000, 165), 3), ((40, 900, 150), 1),
                                          ((300, 600, 140), 0)])
def test_deep_yz_dilation_tiles(dims, vox_inf):
    """Grids with many y rows and z slices take 8-deep y/z dilation tiles
    (8 output slices per tile, 8 + 2 vox_inf input slices staged in LDS),
    including a partial last tile along y and along z."""
    assert _deep_tiles(dims) >= DEEP_TILE_MIN and dims[1] % 32 and dims[2] % 8
    fr = scenes.make_frame("plain-medium", 120 + dims[1], dims=dims, vox_inf=vox_inf,
                           size=(320, 240))
    _say(f"deep dilation tiles {dims} vox_inf {vox_inf}")
    _one_frame(fr, f"deep tiles {dims}")


def _round_of_grids(specs, seed):
    """One frame per grid (a single batch round), each grid centred on its
    frame's camera."""
    frs = []
    for k, (dims, vox, r, workload, size) in enumerate(specs):
        frs.append(scenes.make_frame(workload, seed + k, dims=dims, vox_size=vox, vox_inf=r,
                                     size=size))
    twins = [Twin(f.dims, f.vox_size, f.origin, f.vox_inf) for f in frs]
    dev = [DevFrame(t, f) for t, f in zip(twins, frs)]
    vg.vg_integrate_batch([d.desc for d in dev], _workspace(len(dev)))
    for t, f in zip(twins, frs):
        t.oracle_frame(f)
    return twins


def test_batch_round_of_grids_257_to_512_wide():
    """A batch round whose widest grid needs the 16-word dilation tile (rows
    of 257-512 voxels), next to a narrower grid that the same tile covers."""
    specs = [((300, 280, 60), 0.05, 2, "plain-medium", None),
             ((480, 264, 48), 0.05, 3, "plain-medium", (320, 240)),
             ((200, 200, 64), 0.05, 1, "plain-medium", None),
             ((512, 260, 40), 0.1, 3, "plain-small", None)]
    for dims, _, r, _, _ in specs:
        assert _words(dims[0]) <= TILED_MAX_WORDS and r <= TILED_MAX_INF
    assert max(_words(d[0]) for d, *_ in specs) > 8
    _say("batch round, grids 257-512 wide")
    twins = _round_of_grids(specs, 120)
    for k, t in enumerate(twins):
        t.check(f"wide batch grid {k} {specs[k][0]}")
        t.close()


@pytest.mark.parametrize("with_wide", [False, True])
def test_batch_round_untiled_dilation(with_wide):
    """A batch round with vox_inf > 3 on some grid (and, with_wide, a grid
    wider than 512 voxels): every frame of the round takes the untiled batch
    dilation."""
    specs = [((128, 128, 64), 0.1, 4, "plain-small", None),
             ((100, 100, 50), 0.1, 16, "plain-small", None),
             ((160, 160, 80), 0.05, 2, "plain-medium", (320, 240))]
    if with_wide:
        specs.append(((640, 100, 50), 0.1, 1, "plain-small", None))
    _say(f"batch round, untiled dilation, wide={with_wide}")
    twins = _round_of_grids(specs, 140 + int(with_wide))
    for k, t in enumerate(twins):
        t.check(f"untiled batch grid {k} {specs[k][0]} vox_inf {specs[k][2]}")
        t.close()


# ------------------------------------------------------------------ fp32 canary

def _ulp_neighbours(x, rng, spread=3):
    """x moved by a random whole number of ulps in [-spread, spread], per
    component (float32)."""
    x = np.asarray(x, np.float32).copy()
    for i in range(x.size):
        k = int(rng.integers(-spread, spread + 1))
        v = x.flat[i]
        direction = np.float32(np.inf) if k > 0 else np.float32(-np.inf)
        for _ in range(abs(k)):
            v = np.nextafter(v, direction, dtype=np.float32)
        x.flat[i] = v
    return x


def _canary_sensor(depth):
    intr = scenes.pinhole_intrinsics(64, 48, 90.0, 60.0, 0.05, depth)
    return intr


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_fp32_canary_boundary_points(seed):
    """Points whose transformed coordinates lie within a few ulps of a voxel
    boundary on every axis, under a generic (non-dyadic) rotation: the fp32
    transform in its fixed operation order, the correctly rounded division by
    vox_size and floorf decide each voxel, on both sides.  vox_inf 0, so each
    point marks exactly its own voxel."""
    rng = np.random.default_rng([2112, seed])
    dims = (64, 64, 64)
    s = np.float32([0.1, 0.07, 0.13][seed])
    R = scenes.random_rotation(rng).astype(np.float32)
    t = np.float32([0.37, -1.21, 0.83]) + np.float32(rng.uniform(-1, 1, 3))
    origin = scenes.centred_origin(t, dims, s)
    tv = (t - origin).astype(np.float32)
    # boundary targets on a lattice of spacing 4 (isolated voxels)
    ks = np.stack(np.meshgrid(*[np.arange(4, 61, 4)] * 3, indexing="ij"), -1).reshape(-1, 3)
    ks = ks[rng.permutation(len(ks))[:400]]
    pts = []
    for k in ks:
        pv = k.astype(np.float64) * np.float64(s)                  # a voxel corner (metres)
        pc = R.astype(np.float64).T @ (pv - tv.astype(np.float64))
        pts.append(_ulp_neighbours(pc.astype(np.float32), rng))
    pts = np.ascontiguousarray(np.array(pts, np.float32))
    # the oracle's own quantisation puts many of them on either side
    q = np.array([oracle.quantize(R, tv, s, p) for p in pts])
    below = (q < ks).sum()
    assert 0 < below < q.size, "points should straddle the boundaries"
    intr = _canary_sensor(2.0)
    _say(f"fp32 canary: {len(pts)} boundary points, vox {s}, {below} coordinates below")
    tw = Twin(dims, s, origin, 0)
    vg.vg_integrate_points(tw.h, torch.from_numpy(pts).cuda(), vg.pinhole_sensor(intr),
                           vg.make_pose(R, t))
    oracle.integrate_points(tw.ref, tw.origin(), tw.s, 0, pts, intr["fov_x"], intr["fov_y"],
                            intr["depth_max"], R, t)
    tw.check(f"fp32 canary seed {seed}")
    tw.close()


def test_fp32_canary_denormal_coordinates():
    """Denormal camera-frame coordinates with the camera at the grid corner
    (t^v = 0 exactly): products and quotients stay denormal, and a negative
    one floors to voxel -1 (outside, dropped at vox_inf 0) where a flush to
    zero would give voxel 0.  Identity and generic rotations."""
    dims = (32, 32, 32)
    s = np.float32(0.1)
    t = np.float32([1.5, -0.75, 0.25])
    origin = t.copy()                      # camera exactly at the grid's corner
    intr = _canary_sensor(1.0)
    tiny = np.float32(1e-40)               # denormal in fp32
    pts_id = np.array([[-tiny, 0.55, 0.25], [tiny, 0.35, 0.45], [0.25, -tiny, 0.15],
                       [0.45, 0.15, -tiny], [-tiny, -tiny, 0.65], [3 * tiny, 0.05, -2 * tiny]],
                      np.float32)
    rng = np.random.default_rng(4242)
    Rg = scenes.random_rotation(rng).astype(np.float32)
    pts_g = np.array([[1e-39, -2e-39, 3e-39], [-4e-39, 1e-39, 2e-40], [5e-40, 5e-40, -5e-40]],
                     np.float32)
    for name, R, pts in (("identity", np.eye(3, dtype=np.float32), pts_id),
                         ("generic", Rg, pts_g)):
        q = np.array([oracle.quantize(R, np.zeros(3, np.float32), s, p) for p in pts])
        assert (q == -1).any(), "some coordinate must floor to -1"
        _say(f"fp32 canary, denormals, {name} rotation: q = {q.tolist()}")
        tw = Twin(dims, s, origin, 0)
        vg.vg_integrate_points(tw.h, torch.from_numpy(np.ascontiguousarray(pts)).cuda(),
                               vg.pinhole_sensor(intr), vg.make_pose(R, t))
        oracle.integrate_points(tw.ref, tw.origin(), tw.s, 0, pts, intr["fov_x"],
                                intr["fov_y"], intr["depth_max"], R, t)
        tw.check(f"denormal canary, {name}")
        tw.close()


def test_walk_block_order_across_frames_and_tile_shapes():
    """Large one-frame walks take their ray blocks in the order the previous
    walk of the grid built (longest estimated walks first); the order is only
    used for the launch shape it was built for.  Frames of the large pinhole
    sequence into one grid, re-centred before each, with the ray tile
    changed between some of them (an order built for another shape is not
    used) and kept between others (it is): every grid equals the oracle's."""
    traj = scenes.make_trajectory("large-pinhole", n_frames=60)
    first = scenes.trajectory_frame(traj, 0)
    t = Twin(first.dims, first.vox_size, first.origin, first.vox_inf)
    sensor = vg.pinhole_sensor(first.intr)
    for i, tile in [(0, 2), (10, 2), (20, 3), (30, 3), (40, 2), (50, 2)]:
        fr = first if i == 0 else scenes.trajectory_frame(traj, i)
        vg.vg_set_ray_tile(t.h, tile)
        d = oracle.center_offset(fr.dims, fr.vox_size, t.origin(), fr.t)
        _say(f"block order: frame {i} ray tile {tile} shift {d}")
        df = DevFrame(t, fr)
        vg.vg_integrate_frame_shifted(t.h, df.data, sensor, vg.make_pose(fr.R, fr.t), d)
        t.oracle_frame(fr, d)
        t.check(f"block order frame {i}")
    t.close()
