#!/usr/bin/env python3
"""Benchmark: frames/s and voxel-updates/s of depth-frame -> voxel-grid
integration on one MI355X, with p50/p99 frame latency, batched against plain,
per-kernel times, the roofline of the dominant kernel and the CPU oracle timed
beside it.

Headline workload (one "step" = one frame through the whole path, in one
vg_integrate_frame_shifted call: re-centre shift, seed, dilation, walk,
merge): the large pinhole sequence -- 300 consecutive 1280x720 float32
z-depth frames (90x60 deg, 0.3-12 m, depth noise N(0, (0.005 d^2)^2), 5 %
invalid pixels in 8x8 blocks) of a 2 m/s, 30 Hz walk through a seeded
30x30x8 m world of 1500 boxes + 500 spheres, integrated into a resident
400x400x200 uint8 grid (32 M voxels) at 0.025 m with vox_inf 3, re-centred on
the camera before every frame.  Depth images are resident on the GPU before
any timed region.  The timed region is K steps that continue the sequence
after W warm-up steps; p50/p99 latency, per-stage and per-walk-launch times
come from dedicated passes over the whole sequence; the same sequence also
runs as 8-frame batches (vg_integrate_batch), whose final grid must equal the
plain path's.  The first frames are checked against the CPU oracle (which
also gives the single-thread CPU baseline), and a sample of frames is run
through the oracle on every host thread for the voxel-update and walk-step
counts (the CPU oracle runs on a bounded sample only).

Other workloads are extra keys of the same line: the 128x2048 spinning
sequence into the same grid, the medium (640x480 -> 200x200x100 at 0.05 m)
and small (160x120 -> 100x100x50 at 0.1 m) frame pools, batches of
independent frames (16 medium frames, and 64 frames of the batch recipe:
320x240 .. 1280x720, random 6-DoF poses, own grids), the served fleet (16
robots x 300 frames at 30 Hz, continuous batching) and the paper's standard
parameters beside its Table II.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "frames/s + voxel-updates/s at 1 GPU, p50/p99 frame latency; batched vs plain, bit-exact"
WORKLOAD = "large-pinhole"

# Algorithmic operations of one walk step (Alg. 2 inner loop, Amanatides &
# Woo): choose the axis with the nearest boundary (2 compares, 1 select), step
# the voxel coordinate (1 add), advance that axis' boundary parameter (1 fp32
# add, 1 select), the per-axis step count and the squared lattice distance of
# the termination rule (3 integer ops), the termination test (1 compare), the
# in-grid test (3 compares, 1 and), the linear voxel index (2 integer
# multiply-adds), the occupancy read and test (2), the free / traced choice
# (1) and the mark store (1): 20.
OPS_PER_STEP = 20
# MI355X: 256 CUs x 4 SIMDs x 16 lanes, one 32-bit VALU op per lane per clock
# at 2.4 GHz (packed fp32 excluded: the library is built without it).
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
CAL_BYTES = 64 << 20            # calibration copy: 64 MiB read + 64 MiB written
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "traffic_large-pinhole.json")
TRAFFIC_FILE_MEDIUM = os.path.join(PROFILES, "traffic.json")
TRAFFIC_FILE_BATCHED = os.path.join(PROFILES, "traffic_batched.json")
SECTIONS = ("headline", "spinning", "medium", "small", "batched", "served", "paper")

STAGE_KERNELS = {"k_dilate": ["k_dilate_x<false>", "k_dilate_x<true>", "k_dilate_yz"] +
                             [f"k_dilate_yz_tile<{w}, {z}>" for w in (8, 16) for z in (2, 8)],
                 "k_rays": [f"{k}<{g}, {b}, {l}>" for k in ("k_rays", "k_rays_w")
                            for g in ("false", "true") for b in ("false", "true")
                            for l in ("false", "true")],
                 "k_resolve": [f"k_resolve<{b}, {w}>" for b in ("false", "true")
                               for w in ("false", "true")]}


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


_WORKERS = None


def host_workers():
    """Worker processes / threads for host work: at most 16 (one GPU's share
    of the host) and no more than this process may use; --host-workers sets
    it."""
    if _WORKERS is not None:
        return _WORKERS
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return platform.processor() or "unknown"


def host_info():
    try:
        nproc = int(subprocess.run(["nproc"], capture_output=True, text=True,
                                   timeout=10).stdout.strip())
    except Exception:
        nproc = os.cpu_count()
    return {"lscpu_model": cpu_model(), "nproc": nproc, "cpu_count": os.cpu_count()}


def pct(a, nd=5):
    a = np.asarray(a, float)
    return {"p50": round(float(np.percentile(a, 50)), nd),
            "p99": round(float(np.percentile(a, 99)), nd),
            "mean": round(float(a.mean()), nd), "samples": int(a.size)}


def calibration_copy(torch):
    """A plain device copy of CAL_BYTES, untimed: under rocprofv3 --pmc its
    FETCH_SIZE / WRITE_SIZE calibrate the counters of the path's kernels (the
    source is written first, then 4x its size of other data pushes it out of
    the L2 caches, so the copy reads it all from beyond the L2)."""
    cal_src = torch.empty(CAL_BYTES, dtype=torch.uint8, device="cuda").fill_(1)
    cal_evict = torch.empty(4 * CAL_BYTES, dtype=torch.uint8, device="cuda").fill_(2)
    cal_dst = torch.empty_like(cal_src)
    cal_dst.copy_(cal_src)
    torch.cuda.synchronize()
    del cal_src, cal_dst, cal_evict


def measured_traffic(stage, path, workload):
    """Memory-side bytes per launch of a stage's kernels from the committed
    counter summary, or None if absent or taken on kernel sources that have
    changed since."""
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    from paper_2112_13169_amd.prof_summary import kernel_source_hash
    if t.get("source_hash") != kernel_source_hash() or t.get("workload") != workload:
        return None
    # a stage may launch one of several kernels (template forms): the mean
    # over the profiled run's launches of the stage
    got = [t["kernels"][k] for k in STAGE_KERNELS.get(stage, [stage]) if k in t.get("kernels", {})]
    if not got:
        return None
    n = sum(k.get("launches", 1) for k in got)
    return float(sum(k["hbm_bytes_per_launch"] * k.get("launches", 1) for k in got)) / n


def frame_counter_bytes(path, workload):
    """Memory-side bytes per frame of the one-frame path (seed, dilations,
    walk, merge, clear) from the committed counter summary: every such
    kernel's bytes over the profiled run, per walk launch (one per frame);
    None if absent or stale."""
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    from paper_2112_13169_amd.prof_summary import kernel_source_hash
    if t.get("source_hash") != kernel_source_hash() or t.get("workload") != workload:
        return None
    ks = t.get("kernels", {})
    frames = sum(v.get("launches", 0) for k, v in ks.items()
                 if k.startswith(("k_rays<", "k_rays_w<")))
    if not frames:
        return None
    stages = ("k_seed", "k_dilate_", "k_rays<", "k_rays_w<", "k_resolve<", "k_clear")
    total = sum(v["hbm_bytes_per_launch"] * v.get("launches", 1) for k, v in ks.items()
                if k.startswith(stages))
    return float(total) / frames


def frame_memory(f0, upd, fps):
    """Bytes per frame of the one-frame path at its measured rate: the
    algorithmic bytes (4 B per pixel of depth read, 5 B per voxel update:
    its mark store and the merge's two mark reads, local-grid read and
    write) and the memory-side bytes of the committed counter summary."""
    if not upd:
        return None
    H, W = f0.depth.shape
    alg = 4.0 * W * H + 5.0 * upd
    ctr = frame_counter_bytes(TRAFFIC_FILE, WORKLOAD)
    out = {"algorithmic_bytes_per_frame": round(alg),
           "algorithmic_gb_per_s": round(alg * fps / 1e9, 1),
           "counter_bytes_per_frame": round(ctr) if ctr else None,
           "counter_gb_per_s": round(ctr * fps / 1e9, 1) if ctr else None,
           "counter_frac_of_hbm_peak": round(ctr * fps / 1e9 / HBM_PEAK_GBS, 4) if ctr else None,
           "hbm_peak_gb_per_s": HBM_PEAK_GBS,
           "note": "counter bytes: FETCH_SIZE and WRITE_SIZE of every kernel of the one-frame "
                   "path in the committed profile, calibrated on a device copy, per frame"}
    return out


# ------------------------------------------------ inputs (worker processes)

_TRAJ = {}


def _seq_frame(arg):
    from paper_2112_13169_amd import scenes
    name, n, k = arg
    if (name, n) not in _TRAJ:
        _TRAJ[(name, n)] = scenes.make_trajectory(name, n_frames=n)
    return scenes.trajectory_frame(_TRAJ[(name, n)], k)


def _pool_map(fn, args, chunksize=4):
    """fn over args in forked worker processes, or in this process with one
    worker (a profiler that sets up the GPU before the program starts leaves
    no state a fork may copy)."""
    if host_workers() == 1:
        out = []
        for i, a in enumerate(args):
            out.append(fn(a))
            if (i + 1) % 16 == 0:
                log(f"rendered {i + 1}/{len(args)}")
        return out
    import multiprocessing as mp
    with mp.get_context("fork").Pool(host_workers()) as pool:
        return pool.map(fn, args, chunksize=chunksize)


def save_frames(path, frames):
    """A rendered sequence as <path>.npz (arrays) + <path>.json (sensor and
    grid description)."""
    f0 = frames[0]
    arrays = dict(depth=np.stack([f.depth for f in frames]), R=np.stack([f.R for f in frames]),
                  t=np.stack([f.t for f in frames]), origin=np.stack([f.origin for f in frames]))
    if f0.kind == "spinning":
        arrays.update(col_tab=f0.col_tab, row_tab=f0.row_tab)
    np.savez(path + ".npz", **arrays)
    with open(path + ".json", "w") as fh:
        json.dump(dict(intr=f0.intr, dims=list(f0.dims), vox_size=f0.vox_size,
                       vox_inf=f0.vox_inf, kind=f0.kind, n=len(frames)), fh)


def load_frames(path):
    from paper_2112_13169_amd import scenes
    with open(path + ".json") as fh:
        meta = json.load(fh)
    # each array read once (indexing the archive itself would decompress the
    # whole array again for every frame)
    with np.load(path + ".npz") as a:
        arr = {k: a[k] for k in a.files}
    col, row = ((arr["col_tab"], arr["row_tab"]) if meta["kind"] == "spinning"
                else (None, None))
    return [scenes.Frame(depth=arr["depth"][k], R=arr["R"][k], t=arr["t"][k], intr=meta["intr"],
                         dims=tuple(meta["dims"]), vox_size=meta["vox_size"],
                         vox_inf=meta["vox_inf"], origin=arr["origin"][k], kind=meta["kind"],
                         col_tab=col, row_tab=row) for k in range(meta["n"])]


def sequence_frames(name, n, cache=None):
    """The first n frames of a named trajectory (scenes.SEQUENCES), rendered
    in worker processes, or read from `cache` (a directory) when it holds
    them (a cache lets a profiled run skip the rendering)."""
    if n <= 0:
        return []
    path = os.path.join(cache, f"{name}-{n}") if cache else None
    if path and os.path.exists(path + ".json"):
        return load_frames(path)
    frames = _pool_map(_seq_frame, [(name, n, k) for k in range(n)])
    if path:
        os.makedirs(cache, exist_ok=True)
        save_frames(path, frames)
    return frames


def _batch_frame(arg):
    from paper_2112_13169_amd import scenes
    key, k = arg
    return scenes.batched_frame(np.random.default_rng([scenes.SEED_BASE + 2, key, k]))


def batch_recipe_frames(n, key=64):
    """n independent frames of the batch recipe (seeded per frame)."""
    return _pool_map(_batch_frame, [(key, k) for k in range(n)], 1) if n > 0 else []


_FLEET = {}


def _fleet_frame(arg):
    from paper_2112_13169_amd import scenes
    n_robots, n_frames, r, k = arg
    key = (n_robots, n_frames)
    if key not in _FLEET:
        _FLEET[key] = scenes.make_fleet("served", range(n_robots), n_frames)
    return scenes.trajectory_frame(_FLEET[key][r], k, robot=r)


def served_frames(n_robots, n_frames):
    """frames[r][k]: robot r's k-th frame of the served fleet."""
    if n_robots <= 0 or n_frames <= 0:
        return {}
    args = [(n_robots, n_frames, r, k) for r in range(n_robots) for k in range(n_frames)]
    flat = _pool_map(_fleet_frame, args, 8)
    return {r: flat[r * n_frames:(r + 1) * n_frames] for r in range(n_robots)}


def _pool_frame(arg):
    from paper_2112_13169_amd import scenes
    workload, i = arg
    return scenes.make_frame(workload, i)


def pool_frames(workload, n):
    return _pool_map(_pool_frame, [(workload, i) for i in range(n)]) if n > 0 else []


# ------------------------------------------------------------ GPU sequences

class Sequence:
    """Frames of one grid on the GPU: depth resident, sensor and poses built
    once, fresh grids on demand."""

    def __init__(self, frames, torch, vg):
        self.frames, self.torch, self.vg = frames, torch, vg
        f0 = frames[0]
        self.f0 = f0
        self.dev = [torch.from_numpy(f.depth).cuda() for f in frames]
        if f0.kind == "spinning":
            self.tabs = (torch.from_numpy(f0.col_tab).cuda(), torch.from_numpy(f0.row_tab).cuda())
            H, W = f0.depth.shape
            self.sensor = vg.spinning_sensor(W, H, *self.tabs, f0.intr["vfov"],
                                             f0.intr["depth_min"], f0.intr["depth_max"])
        else:
            self.sensor = vg.pinhole_sensor(f0.intr)
        self.poses = [vg.make_pose(f.R, f.t) for f in frames]
        self.n = len(frames)
        self.nvox = int(np.prod(f0.dims))
        self.tile = 3
        self.keep = []

    def new_grid(self, sets=1):
        """A fresh grid; sets > 1: its scratch holds that many plane sets, so
        a batch runs up to `sets` consecutive frames together."""
        vg = self.vg
        b = vg.GridBuffers(self.f0.dims, self.f0.vox_inf, sets=sets)
        h = vg.vg_create_grid(self.f0.dims, self.f0.vox_size, self.f0.origin, self.f0.vox_inf,
                              b.loc, b.spare, b.scratch)
        vg.vg_set_ray_tile(h, self.tile)
        self.keep.append((h, b))
        return h

    def drop(self, h):
        self.vg.vg_destroy_grid(h)
        self.keep = [(g, b) for g, b in self.keep if g is not h]

    def step(self, h, k):
        """Frame k mod n: re-centre on its camera and integrate it (one call)."""
        i = k % self.n
        self.vg.vg_integrate_frame_shifted(h, self.dev[i], self.sensor, self.poses[i],
                                           self.vg.vg_center_offset(h, self.frames[i].t))

    def batch(self, h, i0, m, ws):
        """Frames i0 .. i0+m-1 as one batch, each re-centring the grid."""
        idx = list(range(i0, min(i0 + m, self.n)))
        sh = self.vg.sequence_shifts(h, [self.frames[i].t for i in idx])
        self.vg.vg_integrate_batch([self.vg.frame_image(h, self.dev[i], self.sensor,
                                                        self.poses[i], d)
                                    for i, d in zip(idx, sh)], ws)

    def read(self, h):
        out = self.torch.empty(self.nvox, dtype=self.torch.uint8, device="cuda")
        self.vg.vg_read_grid(h, out)
        return out


def run_sequence(seq, K, W, B, torch, vg, timed=True, pass_steps=None):
    """The plain path (one frame per call) and B-frame batches over a
    sequence.  The stage, walk and latency passes each run pass_steps steps
    (default: the whole sequence once) from a fresh grid.  Returns the figures
    and the plain path's grid after those steps."""
    E = vg.PROFILE_EVENTS
    names = list(vg.PROFILE_STAGES)
    n = seq.n if pass_steps is None else pass_steps

    def ev():
        return torch.cuda.Event(enable_timing=True)

    res = {}
    # timed region: K steps continuing the sequence after W warm-up steps
    if timed:
        h = seq.new_grid()
        for k in range(W):
            seq.step(h, k)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for k in range(W, W + K):
            seq.step(h, k)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        res["timed"] = {"steps": K, "warmup": W, "wall_s": wall,
                        "ms_per_step": wall * 1e3 / K, "frames_per_s": K / wall}
        seq.drop(h)

    # stage pass: every stage timed by its own launches, every frame
    h = seq.new_grid()
    st_ev = [ev() for _ in range(E * n)]
    vg.vg_set_profile_events(h, st_ev)
    for k in range(n):
        seq.step(h, k)
    torch.cuda.synchronize()
    vg.vg_set_profile_events(h, [])
    stage = {}
    for j, nm in enumerate(names):
        if nm != "shift":     # its clear runs inside the walk launch (markers only)
            stage["k_" + nm] = np.array([st_ev[E * k + 2 * j].elapsed_time(st_ev[E * k + 2 * j + 1])
                                         for k in range(n)])
    res["stage_ms"] = {k: round(float(v.mean()), 5) for k, v in stage.items()}
    seq.drop(h)

    # walk pass: only the walk's own launches record events (every frame)
    h = seq.new_grid()
    j = names.index("rays")
    row_ev = []
    for k in range(n):
        row = [None] * E
        row[2 * j], row[2 * j + 1] = ev(), ev()
        row_ev += row
    vg.vg_set_profile_events(h, row_ev)
    for k in range(n):
        seq.step(h, k)
    torch.cuda.synchronize()
    vg.vg_set_profile_events(h, [])
    res["walk_ms"] = np.array([row_ev[E * k + 2 * j].elapsed_time(row_ev[E * k + 2 * j + 1])
                               for k in range(n)])
    plain_grid = seq.read(h)
    torch.cuda.synchronize()
    seq.drop(h)

    # latency pass: start of the frame's call (shift marker) .. end of its merge
    h = seq.new_grid()
    i_shift, i_res = names.index("shift"), names.index("resolve")
    lat_ev = []
    for k in range(n):
        row = [None] * E
        row[2 * i_shift], row[2 * i_res + 1] = ev(), ev()
        lat_ev += row
    vg.vg_set_profile_events(h, lat_ev)
    for k in range(n):
        seq.step(h, k)
    torch.cuda.synchronize()
    vg.vg_set_profile_events(h, [])
    res["latency_ms"] = pct([lat_ev[E * k + 2 * i_shift].elapsed_time(lat_ev[E * k + 2 * i_res + 1])
                             for k in range(n)])
    seq.drop(h)

    # the whole sequence, plain, wall clock (no events)
    h = seq.new_grid()
    for k in range(n):
        seq.step(h, k)
    torch.cuda.synchronize()
    seq.drop(h)
    h = seq.new_grid()
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for k in range(n):
        seq.step(h, k)
    torch.cuda.synchronize()
    plain_wall = time.perf_counter() - w0
    seq.drop(h)

    # B-frame batches over the whole sequence: a warm pass, a timed pass (wall
    # clock) whose final grid is compared with the plain path's, and a pass
    # with an event pair around every batch (latency)
    if B > 0:
        ws = torch.empty(vg.vg_batch_workspace_bytes(B), dtype=torch.uint8, device="cuda")
        h = seq.new_grid(sets=B)
        for i0 in range(0, n, B):
            seq.batch(h, i0, B, ws)
        torch.cuda.synchronize()
        seq.drop(h)
        h = seq.new_grid(sets=B)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for i0 in range(0, n, B):
            seq.batch(h, i0, B, ws)
        torch.cuda.synchronize()
        batch_wall = time.perf_counter() - w0
        same = bool(torch.equal(seq.read(h), plain_grid))
        seq.drop(h)
        h = seq.new_grid(sets=B)
        pairs = []
        for i0 in range(0, n, B):
            a, b = ev(), ev()
            a.record()
            seq.batch(h, i0, B, ws)
            b.record()
            pairs.append((a, b))
        torch.cuda.synchronize()
        seq.drop(h)
        res["batched"] = {
            "frames_per_batch": B, "frames": n,
            "frames_per_s": round(n / batch_wall, 1),
            "ms_per_frame": round(batch_wall * 1e3 / n, 5),
            "plain_frames_per_s_same_pass": round(n / plain_wall, 1),
            "speedup_vs_plain": round(plain_wall / batch_wall, 4),
            "batch_latency_ms": pct([a.elapsed_time(b) for a, b in pairs]),
            "bit_exact_vs_plain": same,
            "plane_sets": B,
            "note": "the whole sequence as consecutive batches of frames_per_batch frames, "
                    "each frame re-centring the grid (vg_integrate_batch) on a grid with "
                    "plane_sets plane sets, so each batch is one round: steps 2-3 of its "
                    "frames in one launch per stage and one merge; a frame's latency "
                    "in a batch is its batch's latency; plain_frames_per_s_same_pass is the "
                    "one-frame-per-call path over the same frames, wall clock"}
    res["plain_sequence"] = {"frames": n, "frames_per_s": round(n / plain_wall, 1),
                             "ms_per_frame": round(plain_wall * 1e3 / n, 5)}
    return res, plain_grid


# ------------------------------------------------------------- oracle legs

def recentre_plan(frames, oracle):
    """Per frame of a sequence started on a fresh grid at frames[0].origin:
    the re-centring shift and the grid origin the frame is integrated at."""
    f0 = frames[0]
    base = f0.origin.astype(np.float32)
    total = np.zeros(3, np.int32)
    plan = []
    for f in frames:
        d = oracle.center_offset(f0.dims, f0.vox_size, oracle.origin(base, total, f0.vox_size), f.t)
        total = total + np.asarray(d, np.int32)
        plan.append((d, oracle.origin(base, total, f0.vox_size)))
    return plan


def oracle_step(loc, f, d, org, oracle):
    loc = oracle.shift(loc, d)
    if f.kind == "spinning":
        _, st = oracle.integrate_spinning(loc, org, f.vox_size, f.vox_inf, f.depth, f.col_tab,
                                          f.row_tab, f.intr["vfov"], f.intr["depth_min"],
                                          f.intr["depth_max"],
                                          np.asarray(f.R, np.float32).reshape(-1),
                                          np.asarray(f.t, np.float32), want_ms=False)
    else:
        _, st = oracle.integrate_pinhole(loc, org, f.vox_size, f.vox_inf, f.depth, f.intr, f.R,
                                         f.t, want_ms=False)
    return loc, st


def oracle_sequence(frames, plan, seconds, oracle, min_frames=2):
    """The oracle on the first frames of a sequence, one after another on one
    thread (re-centre + integrate), until `seconds` of CPU time (at least
    min_frames).  Returns (frames run, per-frame seconds, final grid)."""
    f0 = frames[0]
    loc = np.zeros(f0.dims[::-1], np.uint8)
    times = []
    for i, f in enumerate(frames):
        if i >= min_frames and sum(times) >= seconds:
            break
        c0 = time.perf_counter()
        loc, _ = oracle_step(loc, f, *plan[i], oracle)
        times.append(time.perf_counter() - c0)
    return len(times), times, loc


def oracle_stats(frames, plan, idx, oracle):
    """Voxel updates and in-grid walk steps of the sampled frames (they depend
    on the frame and the grid origin, not on the grid's content), from the
    oracle on every host thread (one frame per thread at a time)."""
    from concurrent.futures import ThreadPoolExecutor
    threads = host_workers()

    def one(i):
        f = frames[i]
        loc = np.zeros(f.dims[::-1], np.uint8)
        c0 = time.perf_counter()
        _, st = oracle_step(loc, f, (0, 0, 0), plan[i][1], oracle)
        return st, time.perf_counter() - c0

    w0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as pool:
        got = list(pool.map(one, idx))
    wall = time.perf_counter() - w0
    return [g[0] for g in got], [g[1] for g in got], wall, threads


def walk_roofline(steps, walk_ms, kernel, traffic, note):
    units = float(np.mean(steps))
    achieved = float(np.sum(steps)) * OPS_PER_STEP / (float(np.sum(walk_ms)) * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": round(ALU_PEAK_TOPS, 1),
            "unit": "TOP/s", "frac": round(achieved / ALU_PEAK_TOPS, 4), "traffic": traffic,
            "kernel": kernel, "units_per_launch": round(units, 1),
            "unit_kind": "in-grid walk steps", "ops_per_unit": OPS_PER_STEP,
            "kernel_ms": round(float(np.mean(walk_ms)), 5), "note": note}


# ------------------------------------------------------------------ headline

def run_headline(frames, args, torch, vg, autotune):
    import oracle
    seq = Sequence(frames, torch, vg)
    f0 = seq.f0
    vd, hw, hh, rays = vg.vg_fan_sizes(seq.sensor, f0.vox_size)
    # ray-bundle shape from the autotuner (one fan class), on a scratch grid
    if args.ray_tile is not None:
        seq.tile = int(args.ray_tile)
    elif not args.no_tune:
        th = seq.new_grid()
        table = autotune.tune([(seq.sensor, f0.vox_size, th,
                                lambda: vg.vg_integrate_frame(th, seq.dev[0], seq.sensor,
                                                              seq.poses[0]))], vg, torch, reps=3)
        seq.tile = autotune.choose(table, seq.sensor, f0.vox_size, vg)
        seq.drop(th)
    log(f"headline: {seq.n} frames, ray tile {1 << seq.tile}x{64 >> seq.tile}")
    res, plain_grid = run_sequence(seq, args.steps, args.warmup, args.seq_batch, torch, vg)
    log("headline GPU passes done")

    out = {"plain_grid": plain_grid, "res": res}
    plan = recentre_plan(frames, oracle)
    # parity and the single-thread CPU baseline: the first frames, in order
    if args.cpu_seconds > 0:
        nc, times, ref = oracle_sequence(frames, plan, args.cpu_seconds, oracle)
        h = seq.new_grid()
        for k in range(nc):
            seq.step(h, k)
        got = seq.read(h).cpu().numpy()
        seq.drop(h)
        out["bit_exact"] = bool(np.array_equal(got, ref.reshape(-1)))
        out["oracle_frames"] = nc
        out["cpu_baseline"] = {
            "value": round(nc / sum(times), 4), "unit": "frames/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {nc} frames of the same sequence (re-centre + integrate), "
                      f"one after another on one thread, {sum(times):.1f} s; the GPU grid "
                      f"after the same frames is compared with the oracle's",
            **host_info()}
        log(f"oracle: {nc} frames in {sum(times):.1f} s, bit-exact={out['bit_exact']}")
    # voxel updates and walk steps of sampled frames, on every host thread
    if args.stat_frames > 0:
        S = min(args.stat_frames, seq.n)
        idx = sorted({int(round(j * (seq.n - 1) / max(S - 1, 1))) for j in range(S)})
        stats, secs, wall, threads = oracle_stats(frames, plan, idx, oracle)
        out["stats_idx"] = idx
        out["stats"] = stats
        out["cpu_baseline_parallel"] = {
            "value": round(len(idx) / wall, 4), "unit": "frames/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{len(idx)} frames spread over the sequence, each integrated into a "
                      f"fresh grid at its re-centred origin, {threads} threads (one frame "
                      f"each at a time), {wall:.1f} s wall",
            **host_info()}
        log(f"oracle stats: {len(idx)} frames on {threads} threads in {wall:.1f} s")
    # PCIe-inclusive rate: each frame uploaded from pinned host memory first
    host = [torch.from_numpy(f.depth).pin_memory() for f in frames]
    stage_dev = torch.empty_like(seq.dev[0])
    h = seq.new_grid()
    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
             for _ in range(seq.n)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for k, (a, b) in enumerate(pairs):
        a.record()
        stage_dev.copy_(host[k], non_blocking=True)
        vg.vg_integrate_frame_shifted(h, stage_dev, seq.sensor, seq.poses[k],
                                      vg.vg_center_offset(h, frames[k].t))
        b.record()
    torch.cuda.synchronize()
    out["with_h2d"] = {"frames_per_s": round(seq.n / (time.perf_counter() - w0), 1),
                       "latency_ms": pct([a.elapsed_time(b) for a, b in pairs]),
                       "note": "each frame's 3.7 MB depth image is first copied from pinned host "
                               "memory on the same stream; not the headline value"}
    seq.drop(h)
    out.update(vd=vd, hw=hw, hh=hh, rays=rays, tile=seq.tile, n=seq.n)
    return out


# ------------------------------------------------------- other workloads

def run_pool(workload, frames, K, W, torch, vg, oracle, check=8):
    """A pool of seeded frames of random pose cycled through one resident
    grid, each frame re-centring it (one call per frame): frames/s, latency
    over every step, stage times; the first `check` frames against the
    oracle."""
    seq = Sequence(frames, torch, vg)
    res, _ = run_sequence(seq, K, W, 0, torch, vg, pass_steps=K)
    plan = recentre_plan(frames, oracle)
    nc = min(check, len(frames))
    ref = np.zeros(seq.f0.dims[::-1], np.uint8)
    for i in range(nc):
        ref, _ = oracle_step(ref, frames[i], *plan[i], oracle)
    h = seq.new_grid()
    for k in range(nc):
        seq.step(h, k)
    same = bool(np.array_equal(seq.read(h).cpu().numpy(), ref.reshape(-1)))
    seq.drop(h)
    # walk steps and updates of the first frames (fresh grids at their origins)
    stats = [oracle_step(np.zeros(seq.f0.dims[::-1], np.uint8), frames[i], (0, 0, 0),
                         plan[i][1], oracle)[1] for i in range(nc)]
    walk = res["walk_ms"][:nc]
    t = res["timed"]
    return {
        "workload": workload, "frame_pool": len(frames),
        "frames_per_s": round(t["frames_per_s"], 1), "ms_per_step": round(t["ms_per_step"], 5),
        "steps": K, "warmup": W,
        "latency_ms": res["latency_ms"],
        "stage_ms": res["stage_ms"],
        "walk_ms": pct(res["walk_ms"]),
        "voxel_updates_per_frame": round(float(np.mean([s["updates"] for s in stats])), 1),
        "walk_steps_per_frame": round(float(np.mean([s["steps"] for s in stats])), 1),
        "walk_roofline": walk_roofline([s["steps"] for s in stats], walk,
                                       "k_rays_w", None,
                                       f"first {nc} frames of the pool"),
        "bit_exact": same, "oracle_frames": nc,
    }


def run_batched(frames, K, warmup, torch, vg, oracle, autotune, sample_oracle=(),
                walk_steps=None, tune=True, graph=False):
    """Batched vs plain on the same frames, each frame with its own grid: one
    vg_integrate_batch call per step against len(frames) vg_integrate_frame
    calls per step.  graph: the batch call is also captured into a HIP graph
    and replayed (the same frames each replay).  Returns the figures of both
    and whether they agree."""
    n = len(frames)
    dev = [torch.from_numpy(f.depth).cuda() for f in frames]
    sensors = [vg.pinhole_sensor(f.intr) for f in frames]
    poses = [vg.make_pose(f.R, f.t) for f in frames]

    def grids():
        out = []
        for f in frames:
            b = vg.GridBuffers(f.dims, f.vox_inf)
            out.append((b, vg.vg_create_grid(f.dims, f.vox_size, f.origin, f.vox_inf, b.loc,
                                              b.spare, b.scratch)))
        return out

    A, B = grids(), grids()
    ws = torch.empty(vg.vg_batch_workspace_bytes(n), dtype=torch.uint8, device="cuda")
    descs = [vg.frame_image(h, d, s, p) for (_, h), d, s, p in zip(A, dev, sensors, poses)]

    def batch_step():
        vg.vg_integrate_batch(descs, ws)

    def plain_step():
        for (_, h), d, s, p in zip(B, dev, sensors, poses):
            vg.vg_integrate_frame(h, d, s, p)

    def read(h, f):
        out = torch.empty(int(np.prod(f.dims)), dtype=torch.uint8, device="cuda")
        vg.vg_read_grid(h, out)
        return out

    # parity on fresh grids: batch == plain for every frame, sampled frames == oracle
    batch_step()
    plain_step()
    torch.cuda.synchronize()
    same = all(bool(torch.equal(read(ha, f), read(hb, f)))
               for (_, ha), (_, hb), f in zip(A, B, frames))
    for k in sample_oracle:
        f = frames[k]
        ref = np.zeros(f.dims[::-1], np.uint8)
        oracle.integrate_pinhole(ref, f.origin, f.vox_size, f.vox_inf, f.depth, f.intr, f.R, f.t,
                                 want_ms=False)
        same = same and bool(np.array_equal(read(A[k][1], f).cpu().numpy(), ref.reshape(-1)))

    # ray-bundle shapes tuned per fan class: for the plain grids on one frame
    # of the class, for the batch on the batched walk launch
    samples = [(s, f.vox_size, hb, (lambda hb=hb, d=d, s=s, p=p: vg.vg_integrate_frame(hb, d, s, p)))
               for (_, hb), d, s, p, f in zip(B, dev, sensors, poses, frames)]
    table = autotune.tune(samples, vg, torch, reps=3) if tune else {}
    for (_, hb), s, f in zip(B, sensors, frames):
        vg.vg_set_ray_tile(hb, autotune.choose(table, s, f.vox_size, vg))

    S = len(vg.BATCH_STAGES)
    j = vg.BATCH_STAGES.index("rays")

    def batch_rays_ms(reps=1):
        rows = []
        for _ in range(reps):
            row = [None] * (2 * S)
            row[2 * j], row[2 * j + 1] = (torch.cuda.Event(enable_timing=True),
                                          torch.cuda.Event(enable_timing=True))
            vg.vg_integrate_batch_timed(descs, ws, row)
            rows.append(row)
        torch.cuda.synchronize()
        return [r[2 * j].elapsed_time(r[2 * j + 1]) for r in rows]

    classes = {}
    for (_, ha), s, f in zip(A, sensors, frames):
        classes.setdefault(autotune.fan_class(s, f.vox_size, vg), []).append(ha)
    btable = autotune.tune_batch(classes, vg.vg_set_ray_tile,
                                 lambda reps=1: float(np.mean(batch_rays_ms(reps))),
                                 reps=3) if tune else {}

    def timed(step):
        for _ in range(warmup):
            step()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(K)]
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for a, b in ev:
            a.record()
            step()
            b.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        lat = np.array([a.elapsed_time(b) for a, b in ev])
        return wall, lat

    wb, lb = timed(batch_step)
    wp, lp = timed(plain_step)
    graph_res = None
    if graph:
        # the batch call captured into a HIP graph and replayed: a replay
        # repeats the captured frames (same images, poses, shifts, stamps)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            vg.vg_integrate_batch(descs, ws, s)
        torch.cuda.synchronize()
        for _ in range(warmup):
            g.replay()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(K)]
        w0 = time.perf_counter()
        for a, b in ev:
            a.record()
            g.replay()
            b.record()
        torch.cuda.synchronize()
        wg = time.perf_counter() - w0
        lg = np.array([a.elapsed_time(b) for a, b in ev])
        same_g = all(bool(torch.equal(read(ha, f), read(hb, f)))
                     for (_, ha), (_, hb), f in zip(A, B, frames))
        graph_res = {"graph_replay_frames_per_s": round(n * K / wg, 1),
                     "graph_replay_ms_per_step": round(wg * 1e3 / K, 4),
                     "graph_replay_step_latency_ms": pct(lg, 4),
                     "graph_replay_bit_exact": same_g}
        del g

    # the batched walk kernel's live time: events its own launches record
    rays_ms = batch_rays_ms(K)
    for (_, h) in A + B:
        vg.vg_destroy_grid(h)

    def tiles_of(tab):
        return {"x".join(str(v) for v in c): {"best": f"{1 << b}x{64 >> b}",
                                              "rays_ms": {f"{1 << w}x{64 >> w}": round(ms, 4)
                                                          for w, ms in t.items()}}
                for c, (b, t) in tab.items()}
    result = {
        "frames_per_step": n, "steps": K,
        "batched_frames_per_s": round(n * K / wb, 1),
        "plain_frames_per_s": round(n * K / wp, 1),
        "speedup": round(wp / wb, 3),
        "batched_ms_per_step": round(wb * 1e3 / K, 4),
        "plain_ms_per_step": round(wp * 1e3 / K, 4),
        "batched_step_latency_ms": pct(lb, 4),
        "plain_step_latency_ms": pct(lp, 4),
        "bit_exact": same,
        "oracle_sampled_frames": list(sample_oracle),
        "ray_tiles_plain": tiles_of(table),
        "ray_tiles_batched": tiles_of(btable),
        "kb_rays_ms": round(float(np.mean(rays_ms)), 5),
    }
    if graph_res:
        result.update(graph_res)
    if walk_steps is not None:
        result["roofline"] = walk_roofline([float(np.sum(walk_steps))] * len(rays_ms), rays_ms,
                                           "kb_rays",
                                           measured_traffic("kb_rays", TRAFFIC_FILE_BATCHED,
                                                            "batched-x16"),
                                           "one batched walk launch over every frame of the step")
    return result


def run_served(frames, torch, vg, serve, rate_hz=30.0):
    """Continuous-batching server over the fleet's frames: real-time Poisson
    arrivals with room for every grid, the same with a budget of three
    quarters of the grids (evictions), and every frame at once (capacity)."""
    n_robots = len(frames)
    n_frames = len(frames[0])
    f0 = frames[0][0]
    sensor = vg.pinhole_sensor(f0.intr)
    backend = serve.GpuBackend(torch, vg, frames, sensor, streams=2, max_batch=64)
    gbytes = backend.grid_bytes(f0.dims, f0.vox_inf)
    fbytes = f0.depth.nbytes
    fixed = 2 * backend.workspace_bytes(64) + backend.fixed_bytes()
    reserve = backend.frame_reserve_bytes(fbytes)
    out = {}
    for name, grids, speed in [("realtime", n_robots, 1.0),
                               ("realtime, tight budget", (3 * n_robots) // 4, 1.0),
                               ("all at once", n_robots, float("inf"))]:
        robots = [serve.Robot(r, f0.dims, f0.vox_size, frames[r][0].origin, f0.vox_inf)
                  for r in range(n_robots)]
        budget = fixed + grids * gbytes + 16 * reserve
        srv = serve.Server(backend, robots, fbytes, budget, max_batch=64, streams=2)
        arrivals = serve.poisson_arrivals(n_robots, n_frames, rate_hz,
                                          np.random.default_rng([2112131694, n_robots]))
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        done = srv.run(arrivals, speed=speed)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        entry = {"frames": len(done), "wall_s": round(wall, 4),
                 "frames_per_s": round(len(done) / wall, 1),
                 "latency": serve.latency_summary(done),
                 "batches": srv.stats.batches,
                 "mean_batch": round(float(np.mean(srv.stats.batch_sizes)), 2),
                 "max_batch": int(max(srv.stats.batch_sizes)),
                 "evictions": srv.stats.evictions, "restores": srv.stats.restores,
                 "budget_MB": round(budget / 2 ** 20, 1),
                 "peak_MB": round(srv.stats.peak_bytes / 2 ** 20, 1)}
        if name == "realtime, tight budget":
            # two robots' served grids against the same frames alone
            same = True
            for r in (0, n_robots - 1):
                b = vg.GridBuffers(f0.dims, f0.vox_inf)
                h = vg.vg_create_grid(f0.dims, f0.vox_size, frames[r][0].origin, f0.vox_inf,
                                      b.loc, b.spare, b.scratch)
                for f in frames[r]:
                    vg.vg_shift_grid(h, *vg.vg_center_offset(h, f.t))
                    vg.vg_integrate_frame(h, torch.from_numpy(f.depth).cuda(), sensor,
                                          vg.make_pose(f.R, f.t))
                alone = torch.empty(int(np.prod(f0.dims)), dtype=torch.uint8, device="cuda")
                vg.vg_read_grid(h, alone)
                torch.cuda.synchronize()
                same = same and bool(np.array_equal(backend.read(srv.robots[r]),
                                                    alone.cpu().numpy()))
                vg.vg_destroy_grid(h)
            entry["bit_exact_vs_alone"] = same
        for rb in srv.robots.values():
            vg.vg_destroy_grid(rb.handle)
        out[name] = entry
    return out


# The paper's own GPU times for its standard parameters (RTX 2060, Table II):
# populate occupied 7 us, ray-trace to free 44 us, merge 7 us; 58 us of
# kernels per frame in all (Sec. V), next to 0.1 / 2.2 / 0.2 ms on one core of
# an i7-9750H.
PAPER_STANDARD_US = {"populate": 7.0, "raytrace": 44.0, "merge": 7.0, "kernels": 58.0}
PAPER_STANDARD_CPU_MS = {"populate": 0.1, "raytrace": 2.2, "merge": 0.2}


def run_paper_standard(K, warmup, torch, vg, oracle, scenes):
    """The paper's standard parameters on the synthetic scene (its Gazebo world
    is not available): 8 seeded frames of random pose cycled through one grid,
    re-centred each frame, one frame per call; per-stage times from the
    stages' own launches beside the paper's Table II, and the grid after one
    cycle against the oracle."""
    frames = [scenes.make_frame("paper-standard", k) for k in range(8)]
    f0 = frames[0]
    seq = Sequence(frames, torch, vg)
    h = seq.new_grid()
    plan = recentre_plan(frames, oracle)
    ref = np.zeros(f0.dims[::-1], np.uint8)
    for k, f in enumerate(frames):
        ref, _ = oracle_step(ref, f, *plan[k], oracle)
        seq.step(h, k)
    same = bool(np.array_equal(seq.read(h).cpu().numpy(), ref.reshape(-1)))

    # stages timed by their own launches
    E = vg.PROFILE_EVENTS
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(E * K)]
    for k in range(warmup):
        seq.step(h, k)
    vg.vg_set_profile_events(h, evs)
    for k in range(K):
        seq.step(h, k)
    torch.cuda.synchronize()
    vg.vg_set_profile_events(h, [])
    stage_us = {}
    for j, name in enumerate(vg.PROFILE_STAGES):
        if name != "shift":
            stage_us[name] = round(float(np.mean([evs[E * k + 2 * j].elapsed_time(
                evs[E * k + 2 * j + 1]) for k in range(K)])) * 1e3, 2)
    # whole steps, no events
    for k in range(warmup):
        seq.step(h, k)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for k in range(K):
        seq.step(h, k)
    torch.cuda.synchronize()
    us = (time.perf_counter() - w0) * 1e6 / K
    seq.drop(h)
    rays = vg.vg_fan_sizes(seq.sensor, f0.vox_size)[3]
    ours = {"populate": round(stage_us["seed"] + stage_us["dilate"], 2),
            "raytrace": stage_us["rays"], "merge": stage_us["resolve"]}
    return {
        "workload": "the paper's standard parameters: 320x240 depth, 85x101 deg as printed, "
                    "0.3-6.5 m, 100x100x20 voxels of 0.15 m (200 000), vox_inf 2, "
                    f"{rays} rays; synthetic scene (ground + 20 boxes, 2 % invalid pixels) "
                    "for its Gazebo world; each frame re-centres the grid",
        "steps": K,
        "us_per_frame": round(us, 2),
        "frames_per_s": round(1e6 / us, 1),
        "stage_us": ours,
        "stage_us_kernels_sum": round(sum(ours.values()), 2),
        "paper_rtx2060_us": PAPER_STANDARD_US,
        "paper_i7_one_core_ms": PAPER_STANDARD_CPU_MS,
        "note": "stage_us: populate = seed + dilation launches, raytrace = walk launch (it "
                "also runs the re-centring clear), merge = merge launch; each from the "
                "start of its first launch to the end of its last",
        "bit_exact": same,
    }


# ---------------------------------------------------------------------- main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300,
                    help="timed steps (frames) of the headline sequence")
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--only", default=",".join(SECTIONS),
                    help="comma-separated sections to run: " + ", ".join(SECTIONS))
    ap.add_argument("--seq-frames", type=int, default=300,
                    help="frames of the large sequences (pinhole headline, spinning)")
    ap.add_argument("--seq-batch", type=int, default=8, help="frames per sequence batch")
    ap.add_argument("--frames-cache", default=None,
                    help="directory holding (or to receive) the rendered large sequences")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="single-thread oracle sample length (0 skips it)")
    ap.add_argument("--stat-frames", type=int, default=16,
                    help="sampled headline frames run through the oracle on every host thread "
                         "for voxel-update and walk-step counts (0 skips them)")
    ap.add_argument("--host-workers", type=int, default=0,
                    help="processes rendering inputs and threads of the CPU legs (0: the "
                         "host's share, at most 16; 1: render in this process, as under a "
                         "profiler that sets up the GPU first)")
    ap.add_argument("--pool-steps", type=int, default=300,
                    help="timed steps of the medium and small frame pools")
    ap.add_argument("--batch", type=int, default=64,
                    help="frames per batch of the batch recipe (0 skips the recipe)")
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--no-tune", action="store_true",
                    help="the default 8x8 ray tile, no tuning runs")
    ap.add_argument("--ray-tile", type=int, default=None,
                    help="headline ray tile as log2 of its width (0..6), no tuning runs "
                         "(a profiled run then holds only the headline's own walk launches)")
    ap.add_argument("--serve-robots", type=int, default=16)
    ap.add_argument("--serve-frames", type=int, default=300, help="frames per robot")
    ap.add_argument("--paper-steps", type=int, default=200)
    ap.add_argument("--paper-only", action="store_true",
                    help="the paper's standard parameters alone (--only paper), printing "
                         "their section")
    args = ap.parse_args()
    if args.host_workers > 0:
        global _WORKERS
        _WORKERS = args.host_workers

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the voxel-grid path "
                          "has no multi-GPU mode (independent grids shard by robot)",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    only = set(s.strip() for s in ("paper" if args.paper_only else args.only).split(","))
    unknown = only - set(SECTIONS)
    if unknown:
        print(json.dumps({"error": f"unknown sections {sorted(unknown)}"}))
        sys.exit(2)

    # every input is rendered in worker processes before the GPU is touched
    t0 = time.time()
    pin = (sequence_frames("large-pinhole", args.seq_frames, args.frames_cache)
           if "headline" in only else [])
    spin = (sequence_frames("large-spinning", args.seq_frames, args.frames_cache)
            if "spinning" in only else [])
    medium = pool_frames("plain-medium", 16) if ("medium" in only or "batched" in only) else []
    small = pool_frames("plain-small", 64) if "small" in only else []
    recipe = batch_recipe_frames(args.batch) if "batched" in only else []
    fleet = served_frames(args.serve_robots, args.serve_frames) if "served" in only else {}
    log(f"inputs rendered in {time.time() - t0:.1f}s on {host_workers()} workers: "
        f"{len(pin)} + {len(spin)} large, {len(medium)} medium, {len(small)} small, "
        f"{len(recipe)} recipe, {sum(len(v) for v in fleet.values())} served")

    import torch
    from paper_2112_13169_amd import autotune, scenes, serve, vg

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    torch.cuda.set_device(0)
    import oracle

    if args.paper_only:
        out = run_paper_standard(max(args.paper_steps, 1), 20, torch, vg, oracle, scenes)
        calibration_copy(torch)
        print(json.dumps({"paper_standard": out}))
        return

    out = {"metric": METRIC}
    if pin:
        hl = run_headline(pin, args, torch, vg, autotune)
        res = hl["res"]
        t = res["timed"]
        fps = t["frames_per_s"]
        stats = hl.get("stats")
        upd = float(np.mean([s["updates"] for s in stats])) if stats else None
        steps = [s["steps"] for s in stats] if stats else None
        roof = None
        if stats:
            walk_s = res["walk_ms"][hl["stats_idx"]]
            roof = walk_roofline(steps, walk_s, "k_rays_w<false, false, true>",
                                 measured_traffic("k_rays", TRAFFIC_FILE, WORKLOAD),
                                 f"walk launch live time (events its own dispatches record) on "
                                 f"the {len(steps)} sampled frames of a dedicated pass over the "
                                 f"sequence, against their in-grid walk steps counted by the "
                                 f"oracle; the launch also runs the re-centring shift's slab "
                                 f"clear (extra workgroups)")
            roof["kernel_ms_all_frames"] = round(float(np.mean(res["walk_ms"])), 5)
        f0 = pin[0]
        out.update({
            "value": round(fps, 2),
            "unit": "frames/s",
            "n_gpus": 1,
            "steps": t["steps"],
            "warmup": t["warmup"],
            "ms_per_step": round(t["ms_per_step"], 5),
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f32",
            "data": "synthetic",
            "config": {
                "workload": f"{WORKLOAD} sequence: 1280x720 f32 z-depth, 90x60 deg, 0.3-12 m, "
                            "2 m/s walk at 30 Hz through a 30x30x8 m world of 1500 boxes + 500 "
                            "spheres; grid 400x400x200 u8 (32 M voxels) at 0.025 m, vox_inf 3; "
                            "step = re-centre shift + integrate one frame (one call)",
                "sequence_frames": hl["n"], "rays": hl["rays"], "vox_depth": hl["vd"],
                "fan": f"{2 * hl['hw'] + 1}x{2 * hl['hh'] + 1}",
                "path": "plain (one frame per call); 8-frame sequence batches in "
                    "'sequence_batched'",
                "ray_tile": f"{1 << hl['tile']}x{64 >> hl['tile']}"
                            + (" (autotuned)" if not args.no_tune and args.ray_tile is None
                               else ""),
                "stats_sample": (f"voxel updates and walk steps: oracle on {len(steps)} frames "
                                 f"spread over the sequence" if stats else None),
            },
            "voxel_updates_per_s": round(upd * fps, 1) if upd else None,
            "voxel_updates_per_frame": round(upd, 1) if upd else None,
            "walk_steps_per_frame": round(float(np.mean(steps)), 1) if steps else None,
            "walk_steps_per_s": round(float(np.mean(steps)) * fps, 1) if steps else None,
            "memory": frame_memory(pin[0], upd, fps),
            "latency_ms": res["latency_ms"],
            "stage_ms": res["stage_ms"],
            "walk_ms": pct(res["walk_ms"]),
            "plain_sequence": res["plain_sequence"],
            "sequence_batched": res.get("batched"),
            "bit_exact": hl.get("bit_exact"),
            "oracle_frames": hl.get("oracle_frames"),
            "roofline": roof,
            "cpu_baseline": hl.get("cpu_baseline"),
            "cpu_baseline_parallel": hl.get("cpu_baseline_parallel"),
            "with_h2d": hl["with_h2d"],
        })
        del hl, res
        torch.cuda.empty_cache()
    extra = {}
    if spin:
        t0 = time.time()
        seq = Sequence(spin, torch, vg)
        res, _ = run_sequence(seq, 0, 0, args.seq_batch, torch, vg, timed=False)
        extra["large-spinning"] = {
            "workload": "128x2048 spinning range images (vfov 45 deg, 0.3-12 m) of a 2 m/s walk "
                        "through the same world, into the same 400x400x200 grid at 0.025 m, "
                        "vox_inf 3, re-centred before every frame",
            "rays": vg.vg_fan_sizes(seq.sensor, seq.f0.vox_size)[3],
            "plain_sequence": res["plain_sequence"], "latency_ms": res["latency_ms"],
            "stage_ms": res["stage_ms"], "walk_ms": pct(res["walk_ms"]),
            "sequence_batched": res["batched"]}
        del seq
        torch.cuda.empty_cache()
        log(f"spinning sequence in {time.time() - t0:.1f}s")
    if medium and "medium" in only:
        t0 = time.time()
        extra["plain-medium"] = run_pool("640x480 f32, 90x60 deg, 0.3-8 m, 200 boxes + 50 "
                                         "spheres, grid 200x200x100 at 0.05 m, vox_inf 2",
                                         medium, args.pool_steps, 30, torch, vg, oracle)
        extra["plain-medium"]["roofline_traffic_k_rays"] = measured_traffic(
            "k_rays", TRAFFIC_FILE_MEDIUM, "plain-medium")
        log(f"medium pool in {time.time() - t0:.1f}s")
    if small:
        t0 = time.time()
        extra["plain-small"] = run_pool("160x120 f32, 90x60 deg, 0.3-5 m, 20 boxes, grid "
                                        "100x100x50 at 0.1 m, vox_inf 1", small,
                                        max(args.pool_steps, 1000), 30, torch, vg, oracle)
        log(f"small pool in {time.time() - t0:.1f}s")
    if "batched" in only and medium:
        t0 = time.time()
        walk16 = []
        for f in medium[:16]:   # in-grid walk steps do not depend on the grid's content
            _, st = oracle.integrate_pinhole(np.zeros(f.dims[::-1], np.uint8), f.origin,
                                             f.vox_size, f.vox_inf, f.depth, f.intr, f.R, f.t,
                                             want_ms=False)
            walk16.append(st["steps"])
        extra["batched"] = {"plain-medium x16": dict(
            workload="16 plain-medium frames per step, each into its own 200x200x100 grid",
            **run_batched(medium[:16], args.batch_steps * 4, 3, torch, vg, oracle, autotune,
                          walk_steps=walk16, tune=not args.no_tune))}
        if recipe:
            extra["batched"]["batch-recipe"] = dict(
                workload=f"{len(recipe)} independent frames per step: 320x240..1280x720, range "
                         "to U[4,10] m, random 6-DoF poses, own grids of gx=gy in 100..256, gz "
                         "in 100..128 at 0.05-0.1 m, vox_inf 1-3",
                **run_batched(recipe, args.batch_steps, 2, torch, vg, oracle, autotune,
                              sample_oracle=(0, len(recipe) - 1), tune=not args.no_tune,
                              graph=True))
        torch.cuda.empty_cache()
        log(f"batched runs in {time.time() - t0:.1f}s")
    if fleet:
        t0 = time.time()
        extra["served"] = dict(
            workload=f"{args.serve_robots} robots x {args.serve_frames} frames (2 m/s walks at "
                     "30 Hz through a 40x40x10 m world of 800 boxes + 200 spheres), 640x480 "
                     "frames as the medium workload, each robot's 200x200x100 grid at 0.05 m "
                     "re-centred every frame; Poisson arrivals at 30 Hz per robot",
            **run_served(fleet, torch, vg, serve))
        log(f"served runs in {time.time() - t0:.1f}s")
    if "paper" in only and args.paper_steps > 0:
        t0 = time.time()
        extra["paper_standard"] = run_paper_standard(args.paper_steps, 20, torch, vg, oracle,
                                                     scenes)
        log(f"paper-standard runs in {time.time() - t0:.1f}s")
    calibration_copy(torch)
    out.update(extra)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
