"""Ray-bundle shape autotuner.

The walk kernel gives each wavefront a tile of 64 fan targets, (1 << w) along
the fan's width by (64 >> w) along its height (vg_set_ray_tile).  The grid
does not depend on the shape -- every ray is walked on its own -- but speed
does: the shape decides how alike the 64 walks of a wavefront are (length,
direction, the occupancy words they touch).  The tuner times every shape on
the device for one representative frame per fan class and keeps the fastest.

A fan class is what sets the walk geometry: sensor kind, fan extent (from the
field of view) and vox_depth bucketed by powers of sqrt(2).  Image resolution
does not enter: the fan of Sec. IV-C depends on the field of view, the range
and the voxel size only.
"""
from __future__ import annotations

import json
import math

import numpy as np

SHAPES = tuple(range(7))     # log2 of the tile width: 1x64 ... 64x1


def fan_class(sensor, vox_size, lib_vg):
    """Hashable class of a (sensor, voxel size) pair."""
    vd, hw, hh, rays = lib_vg.vg_fan_sizes(sensor, vox_size)
    bucket = int(round(2.0 * math.log2(max(vd, 1))))
    aspect = 0 if sensor.kind == lib_vg.VG_SPINNING else int(round(4.0 * math.log2(
        (2 * hw + 1) / (2 * hh + 1))))
    return (int(sensor.kind), aspect, bucket)


def time_shapes(grid, run_frame, lib_vg, torch, reps=5):
    """Median k_rays time (ms) of each tile shape for the frame `run_frame()`
    integrates into `grid` (a vg handle); the grid's content changes."""
    E = lib_vg.PROFILE_EVENTS
    j = lib_vg.PROFILE_STAGES.index("rays")
    out = {}
    for w in SHAPES:
        lib_vg.vg_set_ray_tile(grid, w)
        run_frame()                                  # warm
        evs = []
        for _ in range(reps):
            row = [None] * E
            row[2 * j] = torch.cuda.Event(enable_timing=True)
            row[2 * j + 1] = torch.cuda.Event(enable_timing=True)
            evs += row
        lib_vg.vg_set_profile_events(grid, evs)
        for _ in range(reps):
            run_frame()
        torch.cuda.synchronize()
        lib_vg.vg_set_profile_events(grid, [])
        ms = [evs[E * k + 2 * j].elapsed_time(evs[E * k + 2 * j + 1]) for k in range(reps)]
        out[w] = float(np.median(ms))
    return out


def tune(samples, lib_vg, torch, reps=5):
    """samples: list of (sensor, vox_size, grid, run_frame).  Returns
    {class: (best shape, {shape: ms})} with one timing per class (the first
    sample of each class is its representative)."""
    table = {}
    for sensor, vox, grid, run in samples:
        c = fan_class(sensor, vox, lib_vg)
        if c in table:
            continue
        times = time_shapes(grid, run, lib_vg, torch, reps)
        table[c] = (min(times, key=times.get), times)
    return table


def tune_batch(classes, set_tile, time_rays, reps=3):
    """Shapes for the frames of one batch, timed on the batched walk launch
    itself: there many frames' wavefronts share the chip, so the shape that is
    fastest for a lone frame (latency) need not be fastest in the batch
    (throughput, cache footprint).  classes: {class: [grid handles]} of the
    batch's frames; set_tile(handle, shape); time_rays() runs the batch and
    returns its walk launch time (ms).  One coordinate-descent pass over the
    classes, largest first, the others held at their current shape (8 x 8 to
    begin with).  Returns {class: (best shape, {shape: ms})}."""
    for hs in classes.values():
        for h in hs:
            set_tile(h, 3)
    table = {}
    for c in sorted(classes, key=lambda c: -len(classes[c])):
        times = {}
        for w in SHAPES:
            for h in classes[c]:
                set_tile(h, w)
            time_rays()                                  # warm
            times[w] = float(np.median([time_rays() for _ in range(reps)]))
        best = min(times, key=times.get)
        for h in classes[c]:
            set_tile(h, best)
        table[c] = (best, times)
    return table


def choose(table, sensor, vox_size, lib_vg, default=3):
    """Tuned shape of a (sensor, voxel size), or the default (8 x 8)."""
    hit = table.get(fan_class(sensor, vox_size, lib_vg))
    return default if hit is None else hit[0]


def save(table, path):
    with open(path, "w") as fh:
        json.dump([{"class": list(c), "best": b, "ms": {str(k): v for k, v in t.items()}}
                   for c, (b, t) in table.items()], fh, indent=1)


def load(path):
    with open(path) as fh:
        rows = json.load(fh)
    return {tuple(r["class"]): (int(r["best"]), {int(k): v for k, v in r["ms"].items()})
            for r in rows}
