"""Python binding of libvg.so (include/vg.h): same names, argument marshalling
only.  PyTorch supplies device memory and streams; every step of the voxel
grid path runs in the library's HIP kernels.  There is no fallback: if the
library is missing this module raises on load."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvg.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "vg.h")

VG_OK, VG_ERR_ARG, VG_ERR_HIP, VG_ERR_BUDGET, VG_ERR_STATE = 0, -1, -2, -3, -4
VG_UNKNOWN, VG_FREE, VG_OCCUPIED = 0, 1, 2
VG_PINHOLE, VG_SPINNING = 0, 1
PROFILE_EVENTS = 10  # events per set of vg_set_profile_events: (start, stop) per stage
PROFILE_STAGES = ("seed", "dilate", "rays", "resolve", "shift")


class VgError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: {vg_status_str(status)} ({status})")
        self.status = status


class vg_pose(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3)]


class vg_sensor(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("fx", ctypes.c_double), ("fy", ctypes.c_double), ("cx", ctypes.c_double),
        ("cy", ctypes.c_double), ("fov_x", ctypes.c_double), ("fov_y", ctypes.c_double),
        ("depth_min", ctypes.c_float), ("depth", ctypes.c_float),
        ("col_tab", ctypes.c_void_p), ("row_tab", ctypes.c_void_p),
    ]


class vg_frame(ctypes.Structure):
    _fields_ = [
        ("grid", ctypes.c_void_p), ("shift", ctypes.c_int32 * 3), ("is_points", ctypes.c_int32),
        ("data", ctypes.c_void_p), ("row_pitch_bytes", ctypes.c_int64),
        ("n_points", ctypes.c_int64), ("sensor", vg_sensor), ("T_w_c", vg_pose),
    ]


_lib = None


def lib():
    """Load libvg.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2112_13169_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
        sp = ctypes.POINTER(vg_sensor)
        pp = ctypes.POINTER(vg_pose)
        L.vg_fan_sizes.argtypes = [sp, f32, P]
        L.vg_scratch_bytes.argtypes = [i32, i32, i32, i32]
        L.vg_grid_bytes.argtypes = [i32, i32, i32]
        L.vg_grid_bytes.restype = ctypes.c_size_t
        L.vg_scratch_bytes.restype = ctypes.c_size_t
        L.vg_create_grid.argtypes = [i32, i32, i32, f32, P, i32, P, P, ctypes.c_size_t, P,
                                     ctypes.c_size_t, P, ctypes.POINTER(P)]
        L.vg_integrate_frame.argtypes = [P, P, i64, sp, pp, P]
        L.vg_integrate_frame_shifted.argtypes = [P, P, i64, sp, pp, i32, i32, i32, P]
        L.vg_integrate_points.argtypes = [P, P, i64, sp, pp, P]
        L.vg_shift_grid.argtypes = [P, i32, i32, i32, P]
        L.vg_center_offset.argtypes = [P, P, P]
        L.vg_center_offset_after.argtypes = [P, P, P, P]
        L.vg_grid_origin.argtypes = [P, P]
        L.vg_read_grid.argtypes = [P, P, i32, P]
        L.vg_write_grid.argtypes = [P, P, i32, P]
        L.vg_destroy_grid.argtypes = [P]
        L.vg_set_profile_events.argtypes = [P, P, i32]
        L.vg_batch_workspace_bytes.argtypes = [i32]
        L.vg_batch_workspace_bytes.restype = ctypes.c_size_t
        L.vg_integrate_batch.argtypes = [ctypes.POINTER(vg_frame), i32, P, ctypes.c_size_t, P]
        L.vg_integrate_batch_timed.argtypes = [ctypes.POINTER(vg_frame), i32, P, ctypes.c_size_t,
                                               P, P]
        L.vg_integrate_batch_static.argtypes = [ctypes.POINTER(vg_frame), i32, P]
        L.vg_set_ray_tile.argtypes = [P, i32]
        L.vg_rebind_grid.argtypes = [P, P, P, ctypes.c_size_t, P, ctypes.c_size_t, P]
        L.vg_status_str.argtypes = [i32]
        L.vg_status_str.restype = ctypes.c_char_p
        for name in ("vg_fan_sizes", "vg_create_grid", "vg_integrate_frame",
                     "vg_integrate_frame_shifted",
                     "vg_integrate_points", "vg_shift_grid", "vg_center_offset",
                     "vg_grid_origin", "vg_read_grid", "vg_write_grid", "vg_destroy_grid",
                     "vg_set_profile_events", "vg_integrate_batch", "vg_set_ray_tile",
                     "vg_rebind_grid", "vg_center_offset_after", "vg_integrate_batch_timed",
                     "vg_integrate_batch_static"):
            getattr(L, name).restype = i32
        _lib = L
    return _lib


def header_symbols():
    """Function names declared in include/vg.h."""
    with open(HEADER) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"^\w[\w\s\*]*?\b(vg_\w+)\s*\(", text, re.M)))


def _check(status, what):
    if status != VG_OK:
        raise VgError(status, what)


def _stream(stream):
    """hipStream_t of a torch stream (None: torch's current stream)."""
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


# ----------------------------------------------------------- descriptors

def pinhole_sensor(intr):
    """vg_sensor of a pinhole camera from an intrinsics dict (fx, fy, cx, cy,
    fov_x, fov_y [rad], depth_min, depth_max, width, height)."""
    return vg_sensor(VG_PINHOLE, intr["width"], intr["height"], 0, intr["fx"], intr["fy"],
                     intr["cx"], intr["cy"], intr["fov_x"], intr["fov_y"], intr["depth_min"],
                     intr["depth_max"], None, None)


def spinning_sensor(width, height, col_tab_dev, row_tab_dev, vfov, depth_min, depth_max):
    """vg_sensor of a spinning range sensor; the tables are device tensors."""
    return vg_sensor(VG_SPINNING, width, height, 0, 0.0, 0.0, 0.0, 0.0, 0.0, vfov, depth_min,
                     depth_max, col_tab_dev.data_ptr(), row_tab_dev.data_ptr())


def make_pose(R, t):
    p = vg_pose()
    p.R[:] = [float(v) for v in np.asarray(R, np.float32).reshape(-1)]
    p.t[:] = [float(v) for v in np.asarray(t, np.float32).reshape(-1)]
    return p


# ------------------------------------------------------------ entry points

def vg_status_str(status):
    return lib().vg_status_str(status).decode()


def vg_fan_sizes(sensor, vox_size):
    out = np.zeros(4, np.int64)
    _check(lib().vg_fan_sizes(ctypes.byref(sensor), vox_size,
                              out.ctypes.data_as(ctypes.c_void_p)), "vg_fan_sizes")
    return tuple(int(v) for v in out)


def vg_grid_bytes(gx, gy, gz):
    return int(lib().vg_grid_bytes(gx, gy, gz))


def vg_scratch_bytes(gx, gy, gz, vox_inf):
    return int(lib().vg_scratch_bytes(gx, gy, gz, vox_inf))


def _opt_ptr(t):
    return None if t is None else _ptr(t)


def vg_create_grid(dims, vox_size, origin_w, vox_inf, loc, spare, scratch, stream=None):
    """dims = (gx, gy, gz); loc: uint8 device tensor of vg_grid_bytes(gx, gy,
    gz) elements; spare: unused (None); scratch: uint8 device tensor of
    vg_scratch_bytes(gx, gy, gz, vox_inf) elements (256-byte aligned)."""
    gx, gy, gz = (int(v) for v in dims)
    org = (ctypes.c_float * 3)(*[float(v) for v in np.asarray(origin_w, np.float32)])
    h = ctypes.c_void_p()
    nb = loc.numel() if spare is None else min(loc.numel(), spare.numel())
    _check(lib().vg_create_grid(gx, gy, gz, vox_size, org, int(vox_inf), _ptr(loc),
                                _opt_ptr(spare), nb, _ptr(scratch),
                                scratch.numel() * scratch.element_size(), _stream(stream),
                                ctypes.byref(h)), "vg_create_grid")
    return h


def vg_rebind_grid(g, loc, spare, scratch, stream=None):
    """Bind new device buffers (as for vg_create_grid) to an existing grid."""
    nb = loc.numel() if spare is None else min(loc.numel(), spare.numel())
    _check(lib().vg_rebind_grid(g, _ptr(loc), _opt_ptr(spare), nb, _ptr(scratch),
                                scratch.numel() * scratch.element_size(), _stream(stream)),
           "vg_rebind_grid")


def vg_integrate_frame(g, depth, sensor, pose, stream=None):
    """depth: float32 device tensor [height, width] (rows may be strided)."""
    assert depth.dtype.itemsize == 4 and depth.dim() == 2 and depth.stride(1) == 1
    _check(lib().vg_integrate_frame(g, _ptr(depth), depth.stride(0) * 4, ctypes.byref(sensor),
                                    ctypes.byref(pose), _stream(stream)), "vg_integrate_frame")


def vg_integrate_frame_shifted(g, depth, sensor, pose, shift, stream=None):
    """vg_shift_grid(g, *shift) then vg_integrate_frame(g, depth, ...), in one
    call (the shift's clear runs inside the frame's walk launch)."""
    assert depth.dtype.itemsize == 4 and depth.dim() == 2 and depth.stride(1) == 1
    dx, dy, dz = (int(v) for v in shift)
    _check(lib().vg_integrate_frame_shifted(g, _ptr(depth), depth.stride(0) * 4,
                                            ctypes.byref(sensor), ctypes.byref(pose), dx, dy, dz,
                                            _stream(stream)), "vg_integrate_frame_shifted")


def vg_integrate_points(g, points, sensor, pose, stream=None):
    """points: float32 device tensor [n, 3] in the camera frame."""
    assert points.dtype.itemsize == 4 and points.is_contiguous()
    n = points.numel() // 3
    _check(lib().vg_integrate_points(g, _ptr(points), n, ctypes.byref(sensor), ctypes.byref(pose),
                                     _stream(stream)), "vg_integrate_points")


def vg_shift_grid(g, dx, dy, dz, stream=None):
    _check(lib().vg_shift_grid(g, int(dx), int(dy), int(dz), _stream(stream)), "vg_shift_grid")


def vg_center_offset(g, t_w_c):
    t = (ctypes.c_float * 3)(*[float(v) for v in np.asarray(t_w_c, np.float32)])
    d = (ctypes.c_int32 * 3)()
    _check(lib().vg_center_offset(g, t, d), "vg_center_offset")
    return tuple(d)


def vg_center_offset_after(g, pending, t_w_c):
    p = (ctypes.c_int32 * 3)(*[int(v) for v in pending])
    t = (ctypes.c_float * 3)(*[float(v) for v in np.asarray(t_w_c, np.float32)])
    d = (ctypes.c_int32 * 3)()
    _check(lib().vg_center_offset_after(g, p, t, d), "vg_center_offset_after")
    return tuple(d)


def sequence_shifts(g, positions):
    """Re-centring shifts of consecutive frames of one grid (camera positions
    in order), as they will be when applied one after another."""
    pending = np.zeros(3, np.int64)
    out = []
    for t in positions:
        d = vg_center_offset_after(g, pending, t)
        out.append(d)
        pending += np.asarray(d, np.int64)
    return out


def vg_grid_origin(g):
    o = (ctypes.c_float * 3)()
    _check(lib().vg_grid_origin(g, o), "vg_grid_origin")
    return np.array(o, np.float32)


def vg_read_grid(g, dst, stream=None):
    """dst: uint8 tensor of gx*gy*gz elements (device or host), linear layout."""
    _check(lib().vg_read_grid(g, _ptr(dst), int(dst.is_cuda), _stream(stream)), "vg_read_grid")


def vg_write_grid(g, src, stream=None):
    _check(lib().vg_write_grid(g, _ptr(src), int(src.is_cuda), _stream(stream)), "vg_write_grid")


def vg_set_profile_events(g, events):
    """events: list of torch.cuda.Event (enable_timing=True) or None (not
    recorded), PROFILE_EVENTS per set: the (start, stop) pair of each stage of
    PROFILE_STAGES in turn; [] turns recording off.  Each event is recorded once
    on the current device before its handle is passed on."""
    n = len(events)
    assert n % PROFILE_EVENTS == 0
    arr = (ctypes.c_void_p * max(n, 1))()
    for i, e in enumerate(events):
        if e is None:
            arr[i] = None
            continue
        if not e.cuda_event:
            e.record()          # torch creates the hipEvent_t lazily
        arr[i] = e.cuda_event
    _check(lib().vg_set_profile_events(g, arr if n else None, n // PROFILE_EVENTS),
           "vg_set_profile_events")


def frame_image(g, image, sensor, pose, shift=(0, 0, 0)):
    """vg_frame of a depth / range image (float32 device tensor [height, width],
    rows may be strided).  Keep `image` alive until the batch has run."""
    assert image.dtype.itemsize == 4 and image.dim() == 2 and image.stride(1) == 1
    f = vg_frame()
    f.grid = g.value if isinstance(g, ctypes.c_void_p) else g
    f.shift[:] = [int(v) for v in shift]
    f.is_points = 0
    f.data = image.data_ptr()
    f.row_pitch_bytes = image.stride(0) * 4
    f.n_points = 0
    f.sensor = sensor
    f.T_w_c = pose
    return f


def frame_points(g, points, sensor, pose, shift=(0, 0, 0)):
    """vg_frame of a point cloud (float32 device tensor [n, 3])."""
    assert points.dtype.itemsize == 4 and points.is_contiguous()
    f = vg_frame()
    f.grid = g.value if isinstance(g, ctypes.c_void_p) else g
    f.shift[:] = [int(v) for v in shift]
    f.is_points = 1
    f.data = points.data_ptr()
    f.row_pitch_bytes = 0
    f.n_points = points.numel() // 3
    f.sensor = sensor
    f.T_w_c = pose
    return f


def vg_batch_workspace_bytes(max_frames):
    return int(lib().vg_batch_workspace_bytes(int(max_frames)))


def vg_integrate_batch(frames, workspace, stream=None):
    """frames: list of vg_frame; workspace: uint8 device tensor of at least
    vg_batch_workspace_bytes(len(frames)) elements (256-byte aligned)."""
    n = len(frames)
    arr = (vg_frame * max(n, 1))(*frames)
    _check(lib().vg_integrate_batch(arr, n, _ptr(workspace),
                                    workspace.numel() * workspace.element_size(),
                                    _stream(stream)), "vg_integrate_batch")


VG_STATIC_BATCH_MAX_FRAMES = 256


def vg_integrate_batch_static(frames, stream=None):
    """vg_integrate_batch with the library's own device tables (no workspace
    argument, nothing allocated): at most VG_STATIC_BATCH_MAX_FRAMES frames."""
    n = len(frames)
    arr = (vg_frame * max(n, 1))(*frames)
    _check(lib().vg_integrate_batch_static(arr, n, _stream(stream)),
           "vg_integrate_batch_static")


BATCH_STAGES = ("shift", "seed", "dilate_x", "dilate_yz", "rays", "resolve")


def vg_integrate_batch_timed(frames, workspace, events, stream=None):
    """vg_integrate_batch recording events: 2 * len(BATCH_STAGES) torch
    events (or None), the (start, stop) pair of each stage in turn."""
    n = len(frames)
    assert len(events) == 2 * len(BATCH_STAGES)
    ev = (ctypes.c_void_p * len(events))()
    for i, e in enumerate(events):
        if e is None:
            ev[i] = None
            continue
        if not e.cuda_event:
            e.record()
        ev[i] = e.cuda_event
    arr = (vg_frame * max(n, 1))(*frames)
    _check(lib().vg_integrate_batch_timed(arr, n, _ptr(workspace),
                                          workspace.numel() * workspace.element_size(), ev,
                                          _stream(stream)), "vg_integrate_batch_timed")


def vg_set_ray_tile(g, log2_width):
    _check(lib().vg_set_ray_tile(g, int(log2_width)), "vg_set_ray_tile")


def vg_destroy_grid(g):
    _check(lib().vg_destroy_grid(g), "vg_destroy_grid")


# ------------------------------------------------------------ allocation

class GridBuffers:
    """Device buffers one grid needs, allocated with torch (the library itself
    never allocates): the grid's ring buffer `loc` and its scratch, sized for
    the grid and vox_inf (`spare` is None: shifts work in place).  sets > 1
    gives the scratch that many plane sets, so that a batch runs up to `sets`
    consecutive frames of the grid together."""

    def __init__(self, dims, vox_inf, device="cuda", sets=1):
        import torch
        gx, gy, gz = dims
        n = vg_grid_bytes(gx, gy, gz)
        nbytes = vg_scratch_bytes(gx, gy, gz, vox_inf) * int(sets)
        if n == 0 or nbytes == 0:
            raise ValueError("invalid grid size")
        self.dims = tuple(dims)
        self.loc = torch.empty(n, dtype=torch.uint8, device=device)
        self.spare = None
        self.scratch = torch.empty(nbytes, dtype=torch.uint8, device=device)
        assert self.scratch.data_ptr() % 256 == 0
