"""The serving scheduler on a simulated device (no GPU): frames of each robot
are applied in order exactly once, the memory budget is never exceeded,
admission waits for room and evicts idle grids (restored with their content
before the robot's next frame), and batches that share a robot are ordered
across streams."""
import numpy as np
import pytest

from paper_2112_13169_amd import serve


class FakeEvent:
    """Completes a few device ticks after it is recorded, once every event it
    waits on has completed."""

    def __init__(self, be, waits=()):
        self.be = be
        self.ready_at = be.clock + int(be.rng.integers(0, 4))
        self.waits = list(waits)

    def done(self):
        if self.waits is not None:
            if self.be.clock < self.ready_at or not all(w.done() for w in self.waits):
                return False
            self.waits = None        # done for good
        return True


class FakeBackend:
    """Applies a batch's frames when it is launched, in launch order, and
    checks what the real backend relies on."""

    def __init__(self, rng, grid_bytes=1000, ws=100):
        self.rng = rng
        self._grid = grid_bytes
        self._ws = ws
        self.applied = {}          # rid -> frame indices applied to its grid
        self.stream_last = {}      # stream -> last event launched on it
        self.robots = {}
        self.creates = 0
        self.clock = 0             # device time, one tick per query

    def workspace_bytes(self, max_batch):
        return self._ws

    def grid_bytes(self, dims, vox_inf):
        return self._grid

    def create(self, r):
        assert r.rid not in self.applied
        self.applied[r.rid] = []
        r.handle = ("grid", r.rid)
        r.buffers = object()
        self.creates += 1
        return FakeEvent(self)

    def evict(self, r):
        assert r.inflight == 0 and r.buffers is not None
        r.buffers = None
        return ("ckpt", r.rid, tuple(self.applied[r.rid]))

    def restore(self, r, ckpt):
        assert ckpt == ("ckpt", r.rid, tuple(self.applied[r.rid]))
        r.buffers = object()
        return FakeEvent(self)

    def launch(self, s, batch, waits):
        prev = self.stream_last.get(s)
        ev = FakeEvent(self, list(waits) + ([prev] if prev is not None else []))
        assert len({q.robot for q in batch}) == len(batch), "two frames of one robot in a batch"
        for q in batch:
            r = self.robots[q.robot]
            assert r.buffers is not None, "frame admitted for a robot without a resident grid"
            got = self.applied[q.robot]
            assert q.index == len(got), (q.robot, q.index, got)
            got.append(q.index)
            # the robot's previous batch on another stream must be waited on
            if r.last_event is not None and r.last_stream != s and not r.last_event.done():
                assert any(w is r.last_event for w in waits)
        self.stream_last[s] = ev
        return ev

    def query(self, ev):
        self.clock += 1
        return ev.done()

    def finish_frame(self, q):
        pass


def _robots(n):
    return [serve.Robot(rid, (8, 8, 8), 0.1, np.zeros(3, np.float32), 1) for rid in range(n)]


class FakeClock:
    def __init__(self, dt):
        self.t, self.dt = 0.0, dt

    def __call__(self):
        self.t += self.dt
        return self.t


@pytest.mark.parametrize("budget_grids,streams,max_batch,speed", [
    (16, 2, 64, float("inf")), (5, 2, 8, float("inf")), (2, 3, 4, float("inf")),
    (1, 1, 3, float("inf")), (16, 2, 64, 1.0), (5, 2, 8, 1.0), (2, 3, 4, 1.0), (1, 1, 3, 1.0)])
def test_every_frame_once_in_order_within_budget(budget_grids, streams, max_batch, speed):
    rng = np.random.default_rng(budget_grids * 10 + streams)
    be = FakeBackend(rng)
    n_robots, n_frames = 9, 25
    frame_bytes = 10
    budget = streams * be._ws + budget_grids * be._grid + 3 * frame_bytes
    srv = serve.Server(be, _robots(n_robots), frame_bytes, budget, max_batch=max_batch,
                       streams=streams)
    arrivals = serve.poisson_arrivals(n_robots, n_frames, 30.0, rng)
    # paced arrivals on a simulated clock (0.2 ms per reading), or all at once
    done = srv.run(arrivals, clock=FakeClock(2e-4), speed=speed, spin=0, sleep=lambda s: None)
    assert len(done) == n_robots * n_frames
    for rid in range(n_robots):
        assert be.applied[rid] == list(range(n_frames))
    assert srv.stats.peak_bytes <= budget
    assert srv.used == streams * be._ws + sum(
        be._grid for r in srv.robots.values() if r.buffers is not None)
    assert max(srv.stats.batch_sizes) <= max_batch
    assert be.creates == n_robots
    if budget_grids < n_robots:
        assert srv.stats.evictions > 0
        if speed != float("inf"):      # robots come back after eviction
            assert srv.stats.restores > 0
    else:
        assert srv.stats.evictions == 0
    assert all(q.done >= q.admitted >= q.arrival for q in done)


def test_frames_arriving_during_a_batch_join_the_next_one():
    rng = np.random.default_rng(3)
    be = FakeBackend(rng)
    srv = serve.Server(be, _robots(4), 10, 10 ** 6, max_batch=64, streams=1)
    for rid in range(4):
        srv.arrive(serve.Request(rid, 0, 0.0))
    assert srv.launch(0.0) == 4                    # one batch with every waiting frame
    for rid in range(4):
        srv.arrive(serve.Request(rid, 1, 0.001))
    assert srv.launch(0.001) == 0                  # the only stream is busy
    while not srv.poll(0.002):
        pass
    assert srv.launch(0.002) == 4                  # the late arrivals, all together
    assert srv.stats.batch_sizes == [4, 4]


def test_budget_below_one_grid_is_refused():
    be = FakeBackend(np.random.default_rng(0))
    with pytest.raises(ValueError):
        serve.Server(be, _robots(2), 10, 2 * be._ws + be._grid, streams=2)


def test_latency_summary_and_arrivals():
    rng = np.random.default_rng(1)
    arr = serve.poisson_arrivals(3, 200, 30.0, rng)
    assert len(arr) == 600
    for rid in range(3):
        ts = [t for t, r, k in arr if r == rid]
        assert ts == sorted(ts)
        assert abs(len(ts) / ts[-1] - 30.0) < 6.0
    reqs = [serve.Request(0, k, 0.0, 0.0, 0.001 * (k + 1)) for k in range(100)]
    s = serve.latency_summary(reqs)
    assert abs(s["p50_ms"] - 50.5) < 1e-6 and abs(s["max_ms"] - 100.0) < 1e-9


class CountingDeque(__import__("collections").deque):
    pops = 0

    def popleft(self):
        CountingDeque.pops += 1
        return super().popleft()


def test_admission_stops_scanning_once_no_frame_can_join():
    """With every robot's frames queued at once, forming a batch looks at one
    frame per robot (plus those blocked behind it), not the whole queue, and
    leaves the rest in order."""
    be = FakeBackend(np.random.default_rng(4))
    srv = serve.Server(be, _robots(4), 10, 10 ** 6, max_batch=64, streams=1)
    for k in range(200):
        for rid in range(4):
            srv.arrive(serve.Request(rid, k, 0.0))
    srv.queue = CountingDeque(srv.queue)
    CountingDeque.pops = 0
    assert srv.launch(0.0) == 4
    assert CountingDeque.pops <= 8
    # the frames left keep their arrival order, robot by robot
    rest = list(srv.queue)
    assert len(rest) == 4 * 199
    for rid in range(4):
        assert [q.index for q in rest if q.robot == rid] == list(range(1, 200))


class SlotBackend(FakeBackend):
    """A backend that holds per-stream frame slots: fixed memory charged once,
    nothing per admitted frame."""

    def __init__(self, rng, slot_bytes):
        super().__init__(rng)
        self.slot_bytes = slot_bytes

    def fixed_bytes(self):
        return self.slot_bytes

    def frame_reserve_bytes(self, frame_bytes):
        return 0


def test_backend_fixed_memory_counts_against_the_budget():
    """Fixed device memory of the backend (frame slots) is charged at start-up
    and per-frame reservations follow the backend: the budget covers what is
    really resident, and a budget without room for the slots is refused."""
    rng = np.random.default_rng(5)
    be = SlotBackend(rng, slot_bytes=700)
    streams, frame_bytes = 2, 10
    budget = streams * be._ws + 700 + 3 * be._grid
    srv = serve.Server(be, _robots(6), frame_bytes, budget, max_batch=4, streams=streams)
    assert srv.used == streams * be._ws + 700
    done = srv.run(serve.poisson_arrivals(6, 12, 30.0, rng), clock=FakeClock(2e-4),
                   speed=float("inf"), spin=0, sleep=lambda s: None)
    assert len(done) == 6 * 12 and srv.stats.peak_bytes <= budget
    assert srv.stats.evictions > 0
    assert srv.used == streams * be._ws + 700 + sum(
        be._grid for r in srv.robots.values() if r.buffers is not None)
    with pytest.raises(ValueError):
        serve.Server(SlotBackend(rng, slot_bytes=5000), _robots(2), frame_bytes, budget,
                     max_batch=4, streams=streams)
