"""Serving loop: depth frames from many robots, integrated as they arrive.

Each robot owns a resident local grid (its ring buffer and scratch) that is
re-centred on the robot before every frame (Sec. IV-E) and integrated with the
frame (Sec. IV-B..D).  The server batches continuously: whenever a stream is
free it forms a batch from the frames that have arrived and can be admitted
(at most one per robot: a robot's next frame is re-centred on the grid its
previous frame leaves), and launches it with vg_integrate_batch -- frames that
arrive while batches are on the GPU join the next batch.  Up to `streams` batches run on the device
at once; frames of one robot stay in order (a batch waits on the event of the
robot's previous batch when that ran on another stream).

Admission is by a device-memory budget: resident grids, the device copies of
admitted frames and the per-stream batch workspaces must fit in it.  A frame
whose robot has no resident grid is admitted once one fits; to make room, the
least recently used idle grid (no frame queued or in flight) is evicted: read
back to host memory and its device buffers released; it is restored
(vg_rebind_grid + vg_write_grid) when its robot's next frame is admitted.
Results do not depend on batching, streams or evictions: every robot's grid is
the one its frames give when applied alone, in order.

The scheduler is device-agnostic; `GpuBackend` runs it on the library.
"""
from __future__ import annotations

import collections
import heapq
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    robot: int
    index: int              # frame number within the robot's sequence
    arrival: float          # seconds on the server clock
    admitted: float = None
    done: float = None
    batch: int = None


@dataclass
class Robot:
    rid: int
    dims: tuple
    vox_size: float
    origin: np.ndarray
    vox_inf: int
    handle: object = None
    buffers: object = None       # device buffers while resident
    checkpoint: object = None    # host copy while evicted
    inflight: int = 0            # admitted frames not yet complete
    last_event: object = None
    last_stream: int = -1
    last_used: int = 0


@dataclass
class Stats:
    batches: int = 0
    evictions: int = 0
    restores: int = 0
    blocked_ticks: int = 0
    batch_sizes: list = field(default_factory=list)
    peak_bytes: int = 0


class Server:
    """Continuous-batching scheduler over a backend (see GpuBackend)."""

    def __init__(self, backend, robots, frame_bytes, budget_bytes, max_batch=64, streams=2):
        self.b = backend
        self.robots = {r.rid: r for r in robots}
        self.frame_bytes = int(frame_bytes)
        self.max_batch = int(max_batch)
        self.n_streams = int(streams)
        self.busy = [None] * self.n_streams       # (event, requests) in flight per stream
        self.ws_bytes = self.b.workspace_bytes(self.max_batch)
        self.budget = int(budget_bytes)
        # memory the backend holds whatever is admitted (e.g. per-stream frame
        # slots), and what each admitted frame adds on top of it
        fixed = getattr(self.b, "fixed_bytes", lambda: 0)()
        self.frame_reserve = getattr(self.b, "frame_reserve_bytes", lambda n: n)(self.frame_bytes)
        self.used = self.n_streams * self.ws_bytes + int(fixed)
        self.grid_bytes = {r.rid: self.b.grid_bytes(r.dims, r.vox_inf) for r in robots}
        if self.used + max(self.grid_bytes.values()) + self.frame_reserve > self.budget:
            raise ValueError("budget below one grid, one frame, the batch workspaces and the "
                             "backend's fixed memory")
        self.queue = collections.deque()           # arrived, not admitted (arrival order)
        self.done = []
        self.tick_no = 0
        self.batch_no = 0
        self.stats = Stats()
        self.stats.peak_bytes = self.used
        self.b.robots = self.robots

    # -------------------------------------------------------------- memory

    def _reserve(self, nbytes):
        if self.used + nbytes > self.budget:
            return False
        self.used += nbytes
        self.stats.peak_bytes = max(self.stats.peak_bytes, self.used)
        return True

    def _release(self, nbytes):
        self.used -= nbytes
        assert self.used >= 0

    def _make_resident(self, r, protected):
        need = self.grid_bytes[r.rid]
        while not self._reserve(need):
            idle = [x for x in self.robots.values()
                    if x.buffers is not None and x.inflight == 0 and x.rid not in protected]
            if not idle:
                return False
            victim = min(idle, key=lambda x: x.last_used)
            victim.checkpoint = self.b.evict(victim)
            victim.buffers = None
            victim.last_event, victim.last_stream = None, -1
            self._release(self.grid_bytes[victim.rid])
            self.stats.evictions += 1
        if r.handle is None:
            ev = self.b.create(r)
        else:
            ev = self.b.restore(r, r.checkpoint)
            r.checkpoint = None
            self.stats.restores += 1
        r.last_event, r.last_stream = ev, -1     # set-up work on the backend's own stream
        return True

    # ------------------------------------------------------------ schedule

    def arrive(self, req):
        self.queue.append(req)

    def poll(self, now):
        """Retire finished batches; returns the number of frames completed."""
        n = 0
        for s, slot in enumerate(self.busy):
            if slot is None or not self.b.query(slot[0]):
                continue
            for q in slot[1]:
                q.done = now
                r = self.robots[q.robot]
                r.inflight -= 1
                self._release(self.frame_reserve)
                self.b.finish_frame(q)
                self.done.append(q)
                n += 1
            self.busy[s] = None
        return n

    def launch(self, now):
        """Form and launch one batch if a stream is free; returns its size."""
        free = [s for s, slot in enumerate(self.busy) if slot is None]
        if not free or not self.queue:
            return 0
        s = free[0]
        self.tick_no += 1
        batch, skipped_robots, in_batch = [], set(), set()
        protected = {q.robot for q in self.queue}   # robots with frames waiting keep their grids
        kept = collections.deque()
        while self.queue:
            if (len(batch) >= self.max_batch or
                    len(in_batch) + len(skipped_robots) >= len(self.robots)):
                # nothing further can join: every robot is in the batch or
                # blocked behind an earlier frame (the rest keeps its order)
                kept.extend(self.queue)
                self.queue.clear()
                break
            q = self.queue.popleft()
            r = self.robots[q.robot]
            # one frame per robot per batch: the next one is re-centred on the
            # grid state this frame leaves, which exists once it is enqueued
            ok = (len(batch) < self.max_batch and q.robot not in skipped_robots
                  and q.robot not in in_batch)
            if ok and r.buffers is None:
                ok = self._make_resident(r, protected)
            if ok and not self._reserve(self.frame_reserve):
                ok = False
            if not ok:
                skipped_robots.add(q.robot)      # keep this robot's later frames behind it
                kept.append(q)
                continue
            in_batch.add(q.robot)
            r.inflight += 1
            r.last_used = self.tick_no
            q.admitted = now
            q.batch = self.batch_no
            batch.append(q)
        self.queue = kept
        if not batch:
            self.stats.blocked_ticks += 1
            return 0
        waits = []
        for q in batch:
            r = self.robots[q.robot]
            if r.last_event is not None and r.last_stream != s:
                waits.append(r.last_event)
        event = self.b.launch(s, batch, waits)
        for q in batch:
            r = self.robots[q.robot]
            r.last_event, r.last_stream = event, s
        self.busy[s] = (event, batch)
        self.batch_no += 1
        self.stats.batches += 1
        self.stats.batch_sizes.append(len(batch))
        return len(batch)

    def idle(self):
        return not self.queue and all(slot is None for slot in self.busy)

    def run(self, arrivals, clock=time.perf_counter, speed=1.0, spin=2e-5, sleep=time.sleep):
        """Serve `arrivals` ([(t, robot, index)] with t in seconds from the
        start, frames of a robot in order) on `clock`, time scaled by 1/speed
        (speed=inf: everything arrives at once).  Returns the completed
        requests."""
        heap = [(t, rid, k) for t, rid, k in arrivals]
        heapq.heapify(heap)
        t0 = clock()
        scale = 0.0 if speed == float("inf") else 1.0 / speed
        while heap or not self.idle():
            now = clock() - t0
            while heap and heap[0][0] * scale <= now:
                t, rid, k = heapq.heappop(heap)
                self.arrive(Request(rid, k, t * scale))
            self.poll(clock() - t0)
            launched = self.launch(clock() - t0)
            if not launched:
                if self.idle() and heap:
                    wait = heap[0][0] * scale - (clock() - t0)
                    if wait > 0:
                        sleep(min(wait, 1e-3))
                elif spin:
                    sleep(spin)
        return self.done


def poisson_arrivals(n_robots, n_frames, rate_hz, rng):
    """Independent Poisson arrivals per robot, frames in order."""
    out = []
    for rid in range(n_robots):
        t = 0.0
        for k in range(n_frames):
            t += rng.exponential(1.0 / rate_hz)
            out.append((t, rid, k))
    return out


def latency_summary(done):
    lat = np.array([q.done - q.arrival for q in done]) * 1e3
    if lat.size == 0:
        return {}
    return {"p50_ms": round(float(np.percentile(lat, 50)), 4),
            "p99_ms": round(float(np.percentile(lat, 99)), 4),
            "mean_ms": round(float(lat.mean()), 4), "max_ms": round(float(lat.max()), 4)}


class GpuBackend:
    """Runs the server on the library: grids and frames in device memory (torch
    allocations), batches through vg_integrate_batch on `streams` torch
    streams.  `frames[rid][k]` is robot rid's k-th frame (a scenes.Frame whose
    depth is pinned host memory or numpy)."""

    def __init__(self, torch, vg, frames, sensor, streams=2, max_batch=64, tile=None):
        self.torch, self.vg = torch, vg
        self.frames = frames
        self.sensor = sensor
        self.tile = tile
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.aux = torch.cuda.Stream()     # grid set-up, eviction and restore
        self.ws = [torch.empty(vg.vg_batch_workspace_bytes(max_batch), dtype=torch.uint8,
                               device="cuda") for _ in range(streams)]
        # frames in pinned host memory, so that uploads are asynchronous, and
        # their poses, built once
        self.host = {rid: [torch.from_numpy(np.ascontiguousarray(f.depth)).pin_memory()
                           for f in seq] for rid, seq in frames.items()}
        self.poses = {rid: [vg.make_pose(f.R, f.t) for f in seq] for rid, seq in frames.items()}
        # device slots of each stream's batch: a stream's next batch starts only
        # after its previous one has completed, so the slots are reused as is
        shapes = {f.depth.shape for seq in frames.values() for f in seq}
        self.slots = None
        if len(shapes) == 1:
            shape = shapes.pop()
            self.slots = [torch.empty((max_batch,) + tuple(shape), dtype=torch.float32,
                                      device="cuda") for _ in range(streams)]
        self.dev = {}          # (rid, k) -> device depth of an admitted frame
        self.robots = {}

    def workspace_bytes(self, max_batch):
        return self.vg.vg_batch_workspace_bytes(max_batch)

    def grid_bytes(self, dims, vox_inf):
        return self.vg.vg_grid_bytes(*dims) + self.vg.vg_scratch_bytes(*dims, vox_inf)

    def fixed_bytes(self):
        """Device memory held whatever is admitted: the per-stream frame slots."""
        if self.slots is None:
            return 0
        return sum(t.numel() * t.element_size() for t in self.slots)

    def frame_reserve_bytes(self, frame_bytes):
        """Device memory an admitted frame adds: none with slots (they are
        charged once, in fixed_bytes), else its own device copy."""
        return 0 if self.slots is not None else frame_bytes

    def _event(self):
        ev = self.torch.cuda.Event()
        ev.record(self.aux)
        return ev

    def create(self, r):
        torch, vg = self.torch, self.vg
        with torch.cuda.stream(self.aux):
            r.buffers = vg.GridBuffers(r.dims, r.vox_inf)
            r.handle = vg.vg_create_grid(r.dims, r.vox_size, r.origin, r.vox_inf, r.buffers.loc,
                                         r.buffers.spare, r.buffers.scratch, self.aux)
            if self.tile is not None:
                vg.vg_set_ray_tile(r.handle, self.tile)
            return self._event()

    def evict(self, r):
        torch = self.torch
        host = torch.empty(int(np.prod(r.dims)), dtype=torch.uint8, pin_memory=True)
        with torch.cuda.stream(self.aux):
            self.vg.vg_read_grid(r.handle, host, self.aux)
        self.aux.synchronize()
        r.buffers = None
        return host

    def restore(self, r, host):
        torch, vg = self.torch, self.vg
        with torch.cuda.stream(self.aux):
            r.buffers = vg.GridBuffers(r.dims, r.vox_inf)
            vg.vg_rebind_grid(r.handle, r.buffers.loc, r.buffers.spare, r.buffers.scratch,
                              self.aux)
            vg.vg_write_grid(r.handle, host, self.aux)
            ev = self._event()
        self.aux.synchronize()        # the copy reads `host`, which is released on return
        return ev

    def launch(self, s, batch, waits):
        torch, vg = self.torch, self.vg
        st = self.streams[s]
        with torch.cuda.stream(st):
            # the uploads depend on no grid: they go first, so that they overlap
            # the other stream's batch; the integration then waits for the
            # robots' previous frames
            devs = []
            for j, q in enumerate(batch):
                fr = self.frames[q.robot][q.index]
                if self.slots is not None:
                    d = self.slots[s][j]
                else:
                    d = torch.empty(fr.depth.shape, dtype=torch.float32, device="cuda")
                    self.dev[(q.robot, q.index)] = d
                d.copy_(self.host[q.robot][q.index], non_blocking=True)
                devs.append(d)
            for e in waits:
                st.wait_event(e)
            descs = []
            for q, d in zip(batch, devs):
                fr = self.frames[q.robot][q.index]
                r = self.robots[q.robot]
                shift = vg.vg_center_offset(r.handle, fr.t)
                descs.append(vg.frame_image(r.handle, d, self.sensor,
                                            self.poses[q.robot][q.index], shift))
            vg.vg_integrate_batch(descs, self.ws[s], st)
            ev = torch.cuda.Event()
            ev.record(st)
        return ev

    def query(self, ev):
        return ev.query()

    def read(self, r):
        """Host copy (numpy, linear layout) of a robot's grid once its work is
        done: from the device while resident, else the eviction copy."""
        if r.buffers is None:
            return r.checkpoint.numpy().copy()
        self.torch.cuda.synchronize()
        host = self.torch.empty(int(np.prod(r.dims)), dtype=self.torch.uint8, pin_memory=True)
        with self.torch.cuda.stream(self.aux):
            self.vg.vg_read_grid(r.handle, host, self.aux)
        self.aux.synchronize()
        return host.numpy().copy()

    def finish_frame(self, q):
        self.dev.pop((q.robot, q.index), None)
