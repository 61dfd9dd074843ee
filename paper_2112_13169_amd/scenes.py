"""Seeded synthetic inputs: scenes, poses and rendered depth / range images.

This module draws random numbers and renders images; it holds none of the
voxel-grid method's arithmetic (no quantisation, no ray fan, no walk, no merge).
Both the GPU library's tests and the CPU oracle consume its outputs.

The paper measures on frames from a Gazebo world flown by an exploration
planner (Sec. V); neither is available, so seeded analytic scenes of the same
shapes stand in for them: a ground plane plus axis-aligned boxes and spheres,
rendered exactly in double precision, then cast to float32.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 2112131690


# ----------------------------------------------------------------- cameras

def pinhole_intrinsics(width, height, fov_x_deg, fov_y_deg, depth_min, depth_max):
    """Pinhole model with square-pixel centres at integer (u, v) and the
    principal point at the image centre."""
    fov_x = math.radians(fov_x_deg)
    fov_y = math.radians(fov_y_deg)
    return dict(
        fx=(width / 2.0) / math.tan(fov_x / 2.0),
        fy=(height / 2.0) / math.tan(fov_y / 2.0),
        cx=(width - 1) / 2.0,
        cy=(height - 1) / 2.0,
        fov_x=fov_x,
        fov_y=fov_y,
        depth_min=float(depth_min),
        depth_max=float(depth_max),
        width=int(width),
        height=int(height),
    )


def level_camera(yaw):
    """Camera-to-world rotation of a level optical camera (z forward, x right,
    y down) looking along heading `yaw` in the ENU world frame."""
    c, s = math.cos(yaw), math.sin(yaw)
    z_c = np.array([c, s, 0.0])
    x_c = np.array([s, -c, 0.0])
    y_c = np.array([0.0, 0.0, -1.0])
    return np.stack([x_c, y_c, z_c], axis=1)  # columns are the camera axes


def random_rotation(rng):
    """Uniform random rotation from a normalised 4-D normal quaternion."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def spinning_tables(width, height, vfov_deg):
    """Per-column (cos az, sin az) and per-row (cos el, sin el) tables of a
    spinning range sensor: 360 deg over the columns, +-vfov/2 over the rows
    (row 0 at the top).  Rounded once from double to float32."""
    az = 2.0 * math.pi * np.arange(width) / width
    half = math.radians(vfov_deg) / 2.0
    el = half - (2.0 * half) * np.arange(height) / max(height - 1, 1)
    col = np.stack([np.cos(az), np.sin(az)], axis=1).astype(np.float32).reshape(-1)
    row = np.stack([np.cos(el), np.sin(el)], axis=1).astype(np.float32).reshape(-1)
    return col, row


# ------------------------------------------------------------------ scenes

@dataclass
class Scene:
    ground: bool = True
    boxes: np.ndarray = field(default_factory=lambda: np.zeros((0, 2, 3)))  # [n, lo/hi, xyz]
    spheres: np.ndarray = field(default_factory=lambda: np.zeros((0, 4)))   # [n, cx cy cz r]


def _pixel_dirs(intr):
    W, H = intr["width"], intr["height"]
    ku = (np.arange(W) - intr["cx"]) / intr["fx"]
    kv = (np.arange(H) - intr["cy"]) / intr["fy"]
    return ku, kv


def _frustum_point(rng, R, t, intr, zmin, zmax):
    """A point uniform in the camera frustum volume between depths zmin, zmax."""
    ku, kv = _pixel_dirs(intr)
    u = rng.uniform(ku[0], ku[-1])
    v = rng.uniform(kv[0], kv[-1])
    z = (zmin ** 3 + rng.uniform() * (zmax ** 3 - zmin ** 3)) ** (1.0 / 3.0)
    return t + R @ np.array([z * u, z * v, z])


def frustum_scene(rng, R, t, intr, n_boxes, n_spheres, box_side=(0.2, 1.5),
                  sphere_r=(0.1, 0.8), keep_out=0.3):
    """Ground plane plus boxes / spheres with centres uniform in the frustum."""
    boxes, spheres = [], []
    zlo = max(intr["depth_min"], 0.5)
    zhi = intr["depth_max"]
    while len(boxes) < n_boxes:
        c = _frustum_point(rng, R, t, intr, zlo, zhi)
        half = rng.uniform(box_side[0], box_side[1], 3) / 2.0
        lo, hi = c - half, c + half
        if np.linalg.norm(np.maximum(np.maximum(lo - t, t - hi), 0.0)) > keep_out:
            boxes.append(np.stack([lo, hi]))
    while len(spheres) < n_spheres:
        c = _frustum_point(rng, R, t, intr, zlo, zhi)
        r = rng.uniform(sphere_r[0], sphere_r[1])
        if np.linalg.norm(c - t) - r > keep_out:
            spheres.append(np.array([*c, r]))
    return Scene(True, np.array(boxes).reshape(-1, 2, 3), np.array(spheres).reshape(-1, 4))


def world_scene(rng, extent, n_boxes, n_spheres, box_side=(0.2, 1.5), sphere_r=(0.1, 0.8),
                height=(0.0, 6.0), avoid=None, keep_out=0.5):
    """Ground plane plus primitives uniform over a world box of `extent`
    (x, y sizes centred on 0); `avoid` is an [n, 3] path kept clear."""
    ex, ey = extent
    boxes, spheres = [], []

    def clear(lo, hi):
        if avoid is None:
            return True
        d = np.maximum(np.maximum(lo - avoid, avoid - hi), 0.0)
        return np.min(np.linalg.norm(d, axis=1)) > keep_out

    while len(boxes) < n_boxes:
        c = np.array([rng.uniform(-ex / 2, ex / 2), rng.uniform(-ey / 2, ey / 2),
                      rng.uniform(*height)])
        half = rng.uniform(box_side[0], box_side[1], 3) / 2.0
        if clear(c - half, c + half):
            boxes.append(np.stack([c - half, c + half]))
    while len(spheres) < n_spheres:
        c = np.array([rng.uniform(-ex / 2, ex / 2), rng.uniform(-ey / 2, ey / 2),
                      rng.uniform(*height)])
        r = rng.uniform(*sphere_r)
        if clear(c - r, c + r):
            spheres.append(np.array([*c, r]))
    return Scene(True, np.array(boxes).reshape(-1, 2, 3), np.array(spheres).reshape(-1, 4))


# --------------------------------------------------------------- rendering

def _cast(scene, origin, dirs):
    """Nearest positive ray parameter t for rays origin + t*dirs (dirs [..., 3]),
    inf where nothing is hit.  Exact analytic intersection in double."""
    shape = dirs.shape[:-1]
    d = dirs.reshape(-1, 3)
    best = np.full(d.shape[0], np.inf)
    with np.errstate(divide="ignore", invalid="ignore"):
        if scene.ground:
            tg = -origin[2] / d[:, 2]
            ok = (d[:, 2] < 0) & (tg > 0)
            best = np.where(ok, np.minimum(best, tg), best)
        inv = 1.0 / d
        for lo, hi in scene.boxes:
            t0 = (lo - origin) * inv
            t1 = (hi - origin) * inv
            tn = np.nanmax(np.minimum(t0, t1), axis=1)
            tf = np.nanmin(np.maximum(t0, t1), axis=1)
            hit = (tf >= tn) & (tf > 0)
            th = np.where(tn > 0, tn, tf)
            best = np.where(hit & (th < best), th, best)
        for cx, cy, cz, r in scene.spheres:
            oc = origin - np.array([cx, cy, cz])
            a = np.einsum("ij,ij->i", d, d)
            b = d @ oc
            c = oc @ oc - r * r
            disc = b * b - a * c
            sq = np.sqrt(np.maximum(disc, 0.0))
            t_near = (-b - sq) / a
            t_far = (-b + sq) / a
            th = np.where(t_near > 0, t_near, t_far)
            hit = (disc >= 0) & (th > 0)
            best = np.where(hit & (th < best), th, best)
    return best.reshape(shape)


def _box_corners(lo, hi):
    return np.array([[x, y, z] for x in (lo[0], hi[0]) for y in (lo[1], hi[1])
                     for z in (lo[2], hi[2])])


def _screen_rect(corners, R, t, intr):
    """Pixel rectangle (u0, u1, v0, v1), end-exclusive, that holds the image of
    a box with the given 8 world corners (ordered as _box_corners makes them);
    None when nothing of it lies in front of the camera inside the image, or
    when it lies wholly deeper than depth_max (its hits could only be invalid
    depths, and it cannot hide a valid one).  A box that straddles the camera
    plane is clipped to z >= eps first."""
    W, H = intr["width"], intr["height"]
    eps = 1e-6
    pc = (corners - t) @ np.asarray(R)
    z = pc[:, 2]
    if np.all(z <= eps) or np.all(z > intr["depth_max"]):
        return None
    pts = [pc[z > eps]]
    if np.any(z <= eps):
        cut = []
        for i in range(8):
            for bit in (1, 2, 4):
                j = i | bit
                if j != i and (z[i] > eps) != (z[j] > eps):
                    a = (eps - z[i]) / (z[j] - z[i])
                    cut.append(pc[i] + a * (pc[j] - pc[i]))
        pts.append(np.array(cut))
    p = np.concatenate(pts)
    zz = np.maximum(p[:, 2], eps)
    u = intr["fx"] * p[:, 0] / zz + intr["cx"]
    v = intr["fy"] * p[:, 1] / zz + intr["cy"]
    lo_u, hi_u = np.clip([u.min(), u.max()], -4.0 * W, 5.0 * W)
    lo_v, hi_v = np.clip([v.min(), v.max()], -4.0 * H, 5.0 * H)
    u0, u1 = max(int(math.floor(lo_u)) - 1, 0), min(int(math.ceil(hi_u)) + 2, W)
    v0, v1 = max(int(math.floor(lo_v)) - 1, 0), min(int(math.ceil(hi_v)) + 2, H)
    if u0 >= u1 or v0 >= v1:
        return None
    return u0, u1, v0, v1


def render_pinhole(scene, R, t, intr, noise_k=0.0, rng=None):
    """z-depth image (float32, NaN where nothing valid is seen).  With the ray
    direction R @ (ku, kv, 1) the ray parameter equals the z-depth.  Each
    primitive is intersected only with the pixels of its screen rectangle."""
    ku, kv = _pixel_dirs(intr)
    R = np.asarray(R, float)
    t = np.asarray(t, float)
    cam = np.stack(np.broadcast_arrays(ku[None, :], kv[:, None], np.ones((1, 1))), axis=-1)
    dirs = cam @ R.T
    z = _cast(Scene(scene.ground), t, dirs)
    for lo, hi in scene.boxes:
        rect = _screen_rect(_box_corners(lo, hi), R, t, intr)
        if rect is None:
            continue
        u0, u1, v0, v1 = rect
        sub = _cast(Scene(False, np.array([[lo, hi]])), t, dirs[v0:v1, u0:u1])
        z[v0:v1, u0:u1] = np.minimum(z[v0:v1, u0:u1], sub)
    for s in scene.spheres:
        c, r = s[:3], s[3]
        rect = _screen_rect(_box_corners(c - r, c + r), R, t, intr)
        if rect is None:
            continue
        u0, u1, v0, v1 = rect
        sub = _cast(Scene(False, np.zeros((0, 2, 3)), s[None, :]), t, dirs[v0:v1, u0:u1])
        z[v0:v1, u0:u1] = np.minimum(z[v0:v1, u0:u1], sub)
    if noise_k > 0.0:
        with np.errstate(invalid="ignore"):
            z = z + rng.standard_normal(z.shape) * (noise_k * z * z)
    z = np.where((z >= intr["depth_min"]) & (z <= intr["depth_max"]), z, np.nan)
    return z.astype(np.float32)


def _angular_window(c, rad, R, t, el, n_cols):
    """Rows and columns of a spinning image whose rays can meet a body inside
    the sphere (c, rad): (None, None) when every ray may, else a row slice and
    a column index array (wrapping at 360 deg).  Conservative by one pixel."""
    d = np.asarray(R).T @ (np.asarray(c, float) - t)
    dist = float(np.linalg.norm(d))
    if dist <= rad * 1.001 + 1e-9:
        return None, None
    alpha = math.asin(min(1.0, rad / dist))
    theta = math.asin(max(-1.0, min(1.0, d[2] / dist)))
    d_el = abs(el[0] - el[-1]) / max(len(el) - 1, 1)
    keep = np.nonzero((el >= theta - alpha - d_el) & (el <= theta + alpha + d_el))[0]
    if keep.size == 0:
        return slice(0, 0), np.zeros(0, np.int64)
    rows = slice(int(keep[0]), int(keep[-1]) + 1)
    if abs(theta) + alpha >= 0.5 * math.pi - 1e-6:
        return rows, np.arange(n_cols)
    beta = math.asin(min(1.0, math.sin(alpha) / math.cos(abs(theta))))
    step = 2.0 * math.pi / n_cols
    phi = math.atan2(d[1], d[0])
    j0 = int(math.floor((phi - beta) / step)) - 1
    j1 = int(math.ceil((phi + beta) / step)) + 1
    if j1 - j0 + 1 >= n_cols:
        return rows, np.arange(n_cols)
    return rows, np.arange(j0, j1 + 1) % n_cols


def render_spinning(scene, R, t, col_tab, row_tab, depth_min, depth_max, noise_k=0.0, rng=None):
    """Range image of a spinning sensor (sensor frame z up).  Each primitive is
    intersected only with the rays of its angular window; primitives wholly
    beyond depth_max are skipped (they could only produce invalid ranges)."""
    ca, sa = col_tab[0::2].astype(float), col_tab[1::2].astype(float)
    ce, se = row_tab[0::2].astype(float), row_tab[1::2].astype(float)
    cam = np.stack([ce[:, None] * ca[None, :], ce[:, None] * sa[None, :],
                    np.broadcast_to(se[:, None], (se.size, ca.size))], axis=-1)
    R = np.asarray(R, float)
    t = np.asarray(t, float)
    dirs = cam @ R.T
    el = np.arctan2(se, ce)
    rho = _cast(Scene(scene.ground), t, dirs)
    bodies = [(0.5 * (lo + hi), 0.5 * float(np.linalg.norm(hi - lo)),
               Scene(False, np.array([[lo, hi]]))) for lo, hi in scene.boxes]
    bodies += [(sp[:3], float(sp[3]), Scene(False, np.zeros((0, 2, 3)), sp[None, :]))
               for sp in scene.spheres]
    for c, rad, body in bodies:
        if np.linalg.norm(np.asarray(c) - t) - rad > depth_max:
            continue
        rows, cols = _angular_window(c, rad, R, t, el, ca.size)
        if rows is None:
            rho = np.minimum(rho, _cast(body, t, dirs))
            continue
        if cols.size == 0:
            continue
        sub = _cast(body, t, dirs[rows][:, cols])
        rho[rows, cols] = np.minimum(rho[rows][:, cols], sub)
    if noise_k > 0.0:
        with np.errstate(invalid="ignore"):
            rho = rho + rng.standard_normal(rho.shape) * (noise_k * rho * rho)
    rho = np.where((rho >= depth_min) & (rho <= depth_max), rho, np.nan)
    return rho.astype(np.float32)


def drop_iid(img, rng, frac):
    out = img.copy()
    out[rng.uniform(size=img.shape) < frac] = np.nan
    return out


def drop_blocks(img, rng, frac, block=8):
    out = img.copy()
    H, W = img.shape
    n = int(round(frac * H * W / (block * block)))
    for _ in range(n):
        y = rng.integers(0, max(H - block + 1, 1))
        x = rng.integers(0, max(W - block + 1, 1))
        out[y:y + block, x:x + block] = np.nan
    return out


# ------------------------------------------------------------ workloads

@dataclass
class Frame:
    """One depth frame with the grid it is integrated into."""
    depth: np.ndarray            # float32 [H, W]
    R: np.ndarray                # float32 [3, 3], camera -> world
    t: np.ndarray                # float32 [3]
    intr: dict
    dims: tuple                  # (gx, gy, gz)
    vox_size: float
    vox_inf: int
    origin: np.ndarray           # float32 [3], grid origin centring the camera
    kind: str = "pinhole"
    col_tab: np.ndarray = None
    row_tab: np.ndarray = None


def centred_origin(t, dims, vox_size):
    """Grid origin (float32) that puts the camera at the grid centre."""
    t = np.asarray(t, np.float64)
    half = np.array(dims, np.float64) * float(np.float32(vox_size)) / 2.0
    return (t - half).astype(np.float32)


WORKLOADS = {
    # plain single frame, small: 160x120, 90x60 deg, 0.3-5 m, ground + 20 boxes,
    # 2 % i.i.d. invalid pixels, grid 100x100x50 at 0.1 m, vox_inf 1
    "plain-small": dict(W=160, H=120, fov=(90.0, 60.0), rng=(0.3, 5.0), boxes=20, spheres=0,
                        noise=0.0, drop=("iid", 0.02), dims=(100, 100, 50), vox=0.1, inf=1),
    # plain single frame, medium: 640x480, 0.3-8 m, 200 boxes + 50 spheres,
    # noise N(0, (0.005 d^2)^2), 5 % invalid in 8x8 blocks, 200x200x100 at 0.05 m, vox_inf 2
    "plain-medium": dict(W=640, H=480, fov=(90.0, 60.0), rng=(0.3, 8.0), boxes=200, spheres=50,
                         noise=0.005, drop=("blocks", 0.05), dims=(200, 200, 100), vox=0.05,
                         inf=2),
    # large pinhole: 1280x720, 0.3-12 m, dense clutter, 400x400x200 at 0.025 m, vox_inf 3
    "large-pinhole": dict(W=1280, H=720, fov=(90.0, 60.0), rng=(0.3, 12.0), boxes=1500,
                          spheres=500, noise=0.005, drop=("blocks", 0.05), dims=(400, 400, 200),
                          vox=0.025, inf=3),
    # the paper's standard parameters (Sec. V): 320x240, field of view 85 x 101
    # deg as printed, 0.3-6.5 m, a 15 x 15 x 3 m grid of 0.15 m voxels (200 000),
    # vox_inf 2; its Gazebo world is not available, so the small workload's
    # scene model stands in (ground + 20 boxes, 2 % i.i.d. invalid pixels).
    # Last in the table, so that the seeds of the entries above stay as they were.
    "paper-standard": dict(W=320, H=240, fov=(85.0, 101.0), rng=(0.3, 6.5), boxes=20,
                           spheres=0, noise=0.0, drop=("iid", 0.02), dims=(100, 100, 20),
                           vox=0.15, inf=2),
}


def make_frame(workload, index=0, seed=None, dims=None, vox_size=None, vox_inf=None,
               size=None, yaw=None, position=None):
    """Seeded pinhole frame of a named workload.  Optional overrides shrink the
    grid or image for fast tests without changing the scene model."""
    w = WORKLOADS[workload]
    if seed is None:
        seed = SEED_BASE + 1000 * list(WORKLOADS).index(workload) + index
    rng = np.random.default_rng(seed)
    W, H = size if size is not None else (w["W"], w["H"])
    intr = pinhole_intrinsics(W, H, *w["fov"], *w["rng"])
    yaw = rng.uniform(0.0, 2.0 * math.pi) if yaw is None else yaw
    pos = (np.array([rng.uniform(-10, 10), rng.uniform(-10, 10), 1.0])
           if position is None else np.asarray(position, float))
    R = level_camera(yaw)
    scene = frustum_scene(rng, R, pos, intr, w["boxes"], w["spheres"])
    depth = render_pinhole(scene, R, pos, intr, w["noise"], rng)
    kind, frac = w["drop"]
    depth = drop_iid(depth, rng, frac) if kind == "iid" else drop_blocks(depth, rng, frac)
    dims = tuple(dims) if dims is not None else w["dims"]
    vs = float(np.float32(vox_size if vox_size is not None else w["vox"]))
    r = w["inf"] if vox_inf is None else vox_inf
    return Frame(depth=depth, R=R.astype(np.float32), t=pos.astype(np.float32), intr=intr,
                 dims=dims, vox_size=vs, vox_inf=r, origin=centred_origin(pos, dims, vs))


def random_pose_frame(rng, W, H, fov, rng_m, dims, vox_size, vox_inf, n_boxes, n_spheres,
                      noise=0.005):
    """A frame with a uniformly random 6-DoF camera orientation."""
    intr = pinhole_intrinsics(W, H, *fov, *rng_m)
    R = random_rotation(rng)
    pos = np.array([rng.uniform(-10, 10), rng.uniform(-10, 10), rng.uniform(0.5, 3.0)])
    scene = frustum_scene(rng, R, pos, intr, n_boxes, n_spheres)
    depth = render_pinhole(scene, R, pos, intr, noise, rng)
    depth = drop_blocks(depth, rng, 0.05)
    vs = float(np.float32(vox_size))
    return Frame(depth=depth, R=R.astype(np.float32), t=pos.astype(np.float32), intr=intr,
                 dims=tuple(dims), vox_size=vs, vox_inf=vox_inf,
                 origin=centred_origin(pos, dims, vs))


def smooth_trajectory(rng, n, speed=2.0, rate=30.0, extent=(40.0, 40.0), z=(1.0, 3.0)):
    """Positions and headings of a smooth random walk reflecting at the walls."""
    dt = 1.0 / rate
    p = np.array([rng.uniform(-extent[0] / 4, extent[0] / 4),
                  rng.uniform(-extent[1] / 4, extent[1] / 4), rng.uniform(*z)])
    yaw = rng.uniform(0, 2 * math.pi)
    vz = 0.0
    out_p, out_yaw = [], []
    for _ in range(n):
        out_p.append(p.copy())
        out_yaw.append(yaw)
        yaw += rng.normal(0.0, 0.15)
        vz = 0.9 * vz + rng.normal(0.0, 0.1)
        step = np.array([math.cos(yaw), math.sin(yaw), 0.0]) * speed * dt
        p = p + step + np.array([0.0, 0.0, vz * dt])
        for a, lim in ((0, extent[0] / 2 - 1), (1, extent[1] / 2 - 1)):
            if abs(p[a]) > lim:
                p[a] = math.copysign(lim, p[a])
                yaw = math.pi - yaw if a == 0 else -yaw
        if not z[0] <= p[2] <= z[1]:
            p[2] = min(max(p[2], z[0]), z[1])
            vz = -vz
    return np.array(out_p), np.array(out_yaw)


def yaw_rotation(yaw):
    """Sensor-to-world rotation of a level spinning sensor (z up) whose
    azimuth 0 points along heading `yaw`."""
    c, s = math.cos(yaw), math.sin(yaw)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


# Sequences of frames flown through one seeded world along smooth random
# walks (2 m/s, 30 Hz).  "served": 640x480 pinhole frames with the medium
# frame's noise and holes in a 40 x 40 x 10 m world of 800 boxes + 200
# spheres, grid 200x200x100 at 0.05 m, vox_inf 2.  "large-pinhole" /
# "large-spinning": a 30 x 30 x 8 m world of 1500 boxes + 500 spheres seen by
# a 1280x720 pinhole camera or a 128 x 2048 spinning range sensor (vertical
# fov 45 deg), 0.3-12 m, grid 400x400x200 at 0.025 m, vox_inf 3.
SEQUENCES = {
    "served": dict(extent=(40.0, 40.0), height=(0.0, 10.0), boxes=800, spheres=200,
                   sensor="pinhole", W=640, H=480, fov=(90.0, 60.0), rng=(0.3, 8.0),
                   noise=0.005, drop=0.05, dims=(200, 200, 100), vox=0.05, inf=2),
    "large-pinhole": dict(extent=(30.0, 30.0), height=(0.0, 8.0), boxes=1500, spheres=500,
                          sensor="pinhole", W=1280, H=720, fov=(90.0, 60.0), rng=(0.3, 12.0),
                          noise=0.005, drop=0.05, dims=(400, 400, 200), vox=0.025, inf=3),
    "large-spinning": dict(extent=(30.0, 30.0), height=(0.0, 8.0), boxes=1500, spheres=500,
                           sensor="spinning", W=2048, H=128, vfov=45.0, rng=(0.3, 12.0),
                           noise=0.005, drop=0.0, dims=(400, 400, 200), vox=0.025, inf=3),
}


@dataclass
class Trajectory:
    """One robot's path through a seeded world, and how its frames are taken."""
    name: str
    spec: dict
    scene: Scene
    positions: np.ndarray        # [n, 3]
    yaws: np.ndarray             # [n]
    seed: int


def make_trajectory(name, robot=0, n_frames=300, seed=None):
    """A world and robot `robot`'s walk through it; primitives are kept 0.5 m
    clear of that walk."""
    return make_fleet(name, [robot], n_frames, seed)[0]


def make_fleet(name, robots, n_frames=300, seed=None):
    """One world shared by several robots (primitives kept 0.5 m clear of
    every walk) and each robot's walk through it."""
    spec = SEQUENCES[name]
    if seed is None:
        seed = SEED_BASE + 5000 + 100 * list(SEQUENCES).index(name)
    walks = []
    for robot in robots:
        walk_rng = np.random.default_rng([seed, robot])
        walks.append(smooth_trajectory(walk_rng, n_frames, extent=spec["extent"]))
    avoid = np.concatenate([p for p, _ in walks])
    scene = world_scene(np.random.default_rng([seed, 1 << 20]), spec["extent"], spec["boxes"],
                        spec["spheres"], height=spec["height"], avoid=avoid, keep_out=0.5)
    return [Trajectory(name, spec, scene, p, y, seed) for p, y in walks]


def trajectory_frame(traj, i, robot=0):
    """Frame `i` of a trajectory: the rendered image, the pose and the grid
    centred on the camera."""
    spec = traj.spec
    rng = np.random.default_rng([traj.seed, robot, i + 1])
    pos = traj.positions[i]
    dims = spec["dims"]
    vs = float(np.float32(spec["vox"]))
    if spec["sensor"] == "pinhole":
        intr = pinhole_intrinsics(spec["W"], spec["H"], *spec["fov"], *spec["rng"])
        R = level_camera(traj.yaws[i])
        depth = render_pinhole(traj.scene, R, pos, intr, spec["noise"], rng)
        if spec["drop"] > 0:
            depth = drop_blocks(depth, rng, spec["drop"])
        return Frame(depth=depth, R=R.astype(np.float32), t=pos.astype(np.float32), intr=intr,
                     dims=dims, vox_size=vs, vox_inf=spec["inf"],
                     origin=centred_origin(pos, dims, vs))
    col, row = spinning_tables(spec["W"], spec["H"], spec["vfov"])
    R = yaw_rotation(traj.yaws[i])
    img = render_spinning(traj.scene, R, pos, col, row, *spec["rng"], spec["noise"], rng)
    intr = dict(width=spec["W"], height=spec["H"], vfov=math.radians(spec["vfov"]),
                depth_min=spec["rng"][0], depth_max=spec["rng"][1])
    return Frame(depth=img, R=R.astype(np.float32), t=pos.astype(np.float32), intr=intr,
                 dims=dims, vox_size=vs, vox_inf=spec["inf"],
                 origin=centred_origin(pos, dims, vs), kind="spinning", col_tab=col, row_tab=row)


def batched_frame(rng, max_side=None):
    """One frame of a batch of independent frames: resolution drawn from
    {320x240, 640x480, 848x480, 1280x720}, range 0.3 m to U[4, 10] m, a
    uniformly random 6-DoF pose, the medium frame's scene model, and its own
    grid (gx = gy in 100..256, gz in 100..128, voxel U[0.05, 0.1] m, vox_inf
    in {1, 2, 3}) centred on the camera.  `max_side` caps the grid sides (for
    quick tests)."""
    W, H = [(320, 240), (640, 480), (848, 480), (1280, 720)][int(rng.integers(0, 4))]
    dmax = float(rng.uniform(4.0, 10.0))
    gxy = int(rng.integers(100, 257))
    gz = int(rng.integers(100, 129))
    if max_side is not None:
        gxy, gz = min(gxy, max_side), min(gz, max_side)
    vox = float(rng.uniform(0.05, 0.1))
    r = int(rng.integers(1, 4))
    return random_pose_frame(rng, W, H, (90.0, 60.0), (0.3, dmax), (gxy, gxy, gz), vox, r,
                             200, 50)
