#!/usr/bin/env python3
"""Benchmark: frames/s and voxel-updates/s of depth-frame -> voxel-grid
integration on one MI355X, with p50/p99 frame latency, per-kernel times,
the roofline of the dominant kernel and the CPU oracle timed beside it.

Workload (one "step" = one frame through the whole path): a 640x480 float32
z-depth frame (90x60 deg pinhole, 0.3-8 m, 200 boxes + 50 spheres, depth noise
N(0, (0.005 d^2)^2), 5 % invalid pixels in 8x8 blocks), integrated into a
resident 200x200x100 uint8 grid at 0.05 m with vox_inf 2: re-centre the grid
on the camera (vg_shift_grid by vg_center_offset), then vg_integrate_frame
(seed, dilation, free pass, traced pass, occupied marking).  A pool of seeded frames with random
yaw and position is cycled; depth images are resident on the GPU before the
timed region starts.
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
WORKLOAD = "plain-medium"

# Algorithmic operations of one walk step (Alg. 2 inner loop): choose the axis
# with the nearest boundary (2 compares), advance the voxel (1 add), advance
# that axis' boundary parameter (1 fp32 add), update the squared lattice
# distance (2 integer ops), the termination test (1 compare), the in-grid test
# (3 compares), the linear index (2 integer multiply-adds), the occupancy test
# (1 compare) and the free / traced store (1).
OPS_PER_STEP = 14
# MI355X: 256 CUs x 4 SIMDs x 16 lanes, one 32-bit VALU op per lane per clock
# at 2.4 GHz (packed fp32 excluded: the library is built without it).
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
CAL_BYTES = 64 << 20            # calibration copy: 64 MiB read + 64 MiB written
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


STAGE_KERNELS = {"k_dilate": ["k_dilate_x", "k_dilate_yz"],
                 "k_rays": ["k_rays<false>", "k_rays<true>"]}


def measured_traffic(stage):
    """Memory-side bytes per launch of a stage's kernels from the committed
    counter summary, or None if absent or taken on kernel sources that have
    changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    from paper_2112_13169_amd.prof_summary import kernel_source_hash
    if t.get("source_hash") != kernel_source_hash() or t.get("workload") != WORKLOAD:
        return None
    got = [t["kernels"][k]["hbm_bytes_per_launch"] for k in STAGE_KERNELS.get(stage, [stage])
           if k in t.get("kernels", {})]
    return float(sum(got)) if got else None


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return platform.processor() or "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--frames", type=int, default=16, help="size of the seeded frame pool")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="CPU oracle sample length (0 skips the CPU baseline)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the voxel-grid path "
                          "has no multi-GPU mode (independent grids shard by robot)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2112_13169_amd import scenes, vg

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()

    # ---- inputs: seeded frame pool, resident on the GPU
    t0 = time.time()
    frames = [scenes.make_frame(WORKLOAD, i) for i in range(args.frames)]
    print(f"# generated {len(frames)} frames in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    fr0 = frames[0]
    sensor = vg.pinhole_sensor(fr0.intr)
    vd, hw, hh, rays = vg.vg_fan_sizes(sensor, fr0.vox_size)
    depth_dev = [torch.from_numpy(f.depth).cuda() for f in frames]
    poses = [vg.make_pose(f.R, f.t) for f in frames]
    gx, gy, gz = fr0.dims
    nvox = gx * gy * gz

    def new_grid():
        buf = vg.GridBuffers(fr0.dims, fr0.vox_inf)
        h = vg.vg_create_grid(fr0.dims, fr0.vox_size, fr0.origin, fr0.vox_inf, buf.loc, buf.spare,
                              buf.scratch)
        return buf, h

    def step(h, k, origins=None):
        i = k % len(frames)
        d = vg.vg_center_offset(h, frames[i].t)
        vg.vg_shift_grid(h, *d)
        if origins is not None:
            origins.append((i, vg.vg_grid_origin(h).tobytes()))
        vg.vg_integrate_frame(h, depth_dev[i], sensor, poses[i])

    # ---- parity pass: one cycle of the pool on a fresh grid vs the oracle
    import oracle
    buf, h = new_grid()
    par_origins = []
    for k in range(len(frames)):
        step(h, k, par_origins)
    got = torch.empty(nvox, dtype=torch.uint8, device="cuda")
    vg.vg_read_grid(h, got)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    vg.vg_destroy_grid(h)
    del buf

    ref = np.zeros((gz, gy, gx), np.uint8)
    base = fr0.origin.astype(np.float32)
    shift_total = np.zeros(3, np.int32)
    stats_cache = {}
    cpu_times = []

    def oracle_step(k, loc, shift_total):
        i = k % len(frames)
        f = frames[i]
        org = oracle.origin(base, shift_total, f.vox_size)
        d = oracle.center_offset(f.dims, f.vox_size, org, f.t)
        loc = oracle.shift(loc, d)
        shift_total = shift_total + np.asarray(d, np.int32)
        org = oracle.origin(base, shift_total, f.vox_size)
        _, st = oracle.integrate_pinhole(loc, org, f.vox_size, f.vox_inf, f.depth, f.intr, f.R,
                                         f.t, want_ms=False)
        stats_cache.setdefault((i, org.tobytes()), st)
        return loc, shift_total

    for k in range(len(frames)):
        c0 = time.perf_counter()
        ref, shift_total = oracle_step(k, ref, shift_total)
        cpu_times.append(time.perf_counter() - c0)
    bit_exact = bool(np.array_equal(got, ref.reshape(-1)))
    print(f"# parity pass: {len(frames)} frames, bit-exact={bit_exact}", file=sys.stderr,
          flush=True)

    # ---- CPU baseline: keep stepping the oracle until the sample is long enough
    k = len(frames)
    while args.cpu_seconds > 0 and sum(cpu_times) < args.cpu_seconds:
        c0 = time.perf_counter()
        ref, shift_total = oracle_step(k, ref, shift_total)
        cpu_times.append(time.perf_counter() - c0)
        k += 1

    # ---- GPU: warmup; a stage pass (every stage timed by events its kernel
    # dispatches record) picks the dominant kernel; a latency pass (start of the
    # shift to end of the resolve pass); then the timed region, where only the
    # dominant kernel's dispatches record events.
    buf, h = new_grid()
    for k in range(args.warmup):
        step(h, k)
    K = args.steps
    E = vg.PROFILE_EVENTS
    names = ["k_" + n for n in vg.PROFILE_STAGES]

    def run(k0, profile, origins=None):
        vg.vg_set_profile_events(h, profile)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for k in range(K):
            step(h, k0 + k, origins)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        vg.vg_set_profile_events(h, [])
        return wall

    def ev():
        return torch.cuda.Event(enable_timing=True)

    def pair_ms(evs, j):
        return np.array([evs[E * k + 2 * j].elapsed_time(evs[E * k + 2 * j + 1])
                         for k in range(K)])

    # stage pass: every stage timed by its own kernel dispatches
    st_ev = [ev() for _ in range(E * K)]
    run(args.warmup, st_ev)
    stage_ms = {name: pair_ms(st_ev, j) for j, name in enumerate(names)}
    kernels = {k: float(v.mean()) for k, v in stage_ms.items()}
    dominant = max(kernels, key=kernels.get)

    # latency pass: start of the shift .. end of the resolve pass
    lat_start = [ev() for _ in range(K)]
    lat_end = [ev() for _ in range(K)]
    prof = []
    i_shift, i_resolve = names.index("k_shift"), names.index("k_resolve")
    for k in range(K):
        row = [None] * E
        row[2 * i_shift] = lat_start[k]
        row[2 * i_resolve + 1] = lat_end[k]
        prof += row
    run(args.warmup + K, prof)
    lat = np.array([lat_start[k].elapsed_time(lat_end[k]) for k in range(K)])

    # timed region: K steps, only the dominant kernel's dispatches timed
    dom_ev = []
    j = names.index(dominant)
    for k in range(K):
        row = [None] * E
        row[2 * j], row[2 * j + 1] = ev(), ev()
        dom_ev += row
    origins = []
    wall = run(args.warmup + 2 * K, dom_ev, origins)
    kernel_live_ms = float(pair_ms(dom_ev, j).mean())
    ms_per_step = wall * 1e3 / K
    fps = 1e3 / ms_per_step

    # a plain device copy of known size, untimed: under rocprofv3 --pmc its
    # FETCH_SIZE / WRITE_SIZE calibrate the counters of the path's kernels
    # (the source is written first, then 4x its size of other data pushes it
    # out of the L2 caches, so the copy reads it all from beyond the L2)
    cal_src = torch.empty(CAL_BYTES, dtype=torch.uint8, device="cuda").fill_(1)
    cal_evict = torch.empty(4 * CAL_BYTES, dtype=torch.uint8, device="cuda").fill_(2)
    cal_dst = torch.empty_like(cal_src)
    cal_dst.copy_(cal_src)
    torch.cuda.synchronize()
    del cal_src, cal_dst, cal_evict

    # ---- per-frame work, from the oracle on the same (frame, grid origin)
    for i, ob in origins:
        if (i, ob) not in stats_cache:
            f = frames[i]
            tmp = np.zeros((gz, gy, gx), np.uint8)
            _, st = oracle.integrate_pinhole(tmp, np.frombuffer(ob, np.float32), f.vox_size,
                                             f.vox_inf, f.depth, f.intr, f.R, f.t, want_ms=False)
            stats_cache[(i, ob)] = st
    st_steps = [stats_cache[key] for key in origins]
    upd = np.array([s["updates"] for s in st_steps], float)
    walk = np.array([s["steps"] for s in st_steps], float)
    after = np.array([s["steps_after_hit"] for s in st_steps], float)
    before = walk - after

    if dominant == "k_rays":
        units = walk.mean()
        achieved = units * OPS_PER_STEP / (kernel_live_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(ALU_PEAK_TOPS, 1),
                "unit": "TOP/s", "frac": round(achieved / ALU_PEAK_TOPS, 4),
                "traffic": measured_traffic(dominant),
                "kernel": dominant, "units_per_launch": float(units),
                "unit_kind": "in-grid walk steps", "ops_per_unit": OPS_PER_STEP,
                "kernel_ms": round(kernel_live_ms, 5)}
    else:
        # algorithmic HBM bytes of the streaming stages
        nbytes = {"k_shift": 2.0 * nvox,                   # read + write the grid
                  "k_seed": 5.0 * fr0.depth.size,           # depth in, stamp out
                  "k_dilate": nvox / 8.0 * 2 + nvox,        # seeds in, bit planes out
                  "k_resolve": nvox * (1 + 1 / 8.0) + 2.0 * upd.mean()}[dominant]
        achieved = nbytes / (kernel_live_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(dominant),
                "kernel": dominant, "bytes_per_launch": float(nbytes),
                "kernel_ms": round(kernel_live_ms, 5)}

    cpu = None
    if cpu_times:
        n = len(cpu_times)
        cpu = {"value": round(n / sum(cpu_times), 3), "unit": "frames/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{n} steps (re-centre + integrate) of the same workload on the CPU "
                         f"oracle, single thread, {sum(cpu_times):.1f} s",
               "host_cpu": cpu_model()}

    out = {
        "metric": METRIC,
        "value": round(fps, 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{WORKLOAD}: 640x480 f32 depth, 90x60 deg, 0.3-8 m, 200 boxes + 50 "
                        "spheres, grid 200x200x100 u8 at 0.05 m, vox_inf 2; step = re-centre "
                        "shift + integrate",
            "rays": rays, "vox_depth": vd, "fan": f"{2 * hw + 1}x{2 * hh + 1}",
            "frame_pool": len(frames), "path": "plain (one frame per call)",
        },
        "voxel_updates_per_s": round(float(upd.mean()) * fps, 1),
        "voxel_updates_per_frame": round(float(upd.mean()), 1),
        "walk_steps_per_frame": round(float(walk.mean()), 1),
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 5),
                       "p99": round(float(np.percentile(lat, 99)), 5),
                       "mean": round(float(lat.mean()), 5)},
        "stage_ms": {k: round(v, 5) for k, v in kernels.items()},
        "bit_exact": bit_exact,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
