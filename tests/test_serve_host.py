"""The serving engine's host logic, on the CPU: streams, events and buffers are
stand-ins and the library calls are replaced by recorders, so the tests see
what the engine asks for and in which stream context.

Checked: latest wins (a superseded scan is dropped and counted) and one update
per robot in flight; the memory budget; a robot's particle set and buffers are
made inside the context of the stream its tick then runs on; uploads run on
the copy stream after it waited for the tick's stream, and the tick's stream
waits for them through an event; a tick refused as busy is retried, on
another stream only after the admission's initialisation; the two request
orders; the resampling draw (seed, tick) of each update.
"""

import time

import pytest

from paper_2310_04172_amd import serve


class FakeTensor:
    def __init__(self, shape, tag=""):
        self.shape = tuple(shape)
        self.tag = tag
        self.copies = []

    def numel(self):
        n = 1
        for d in self.shape:
            n *= d
        return n

    @property
    def device(self):
        return "fake"

    def copy_(self, src, non_blocking=False):
        self.copies.append((src, FakeTorch.current[-1], non_blocking))
        return self


class FakeStream:
    count = 0

    def __init__(self):
        FakeStream.count += 1
        self.name = f"s{FakeStream.count}"
        self.log = []

    def wait_stream(self, other):
        self.log.append(("wait_stream", other.name))

    def wait_event(self, ev):
        self.log.append(("wait_event", ev.stream.name if ev.stream else None, ev.serial))

    def __repr__(self):
        return self.name


class FakeEvent:
    serials = 0
    lag = 0                     # queries an event answers "not yet" before it completes

    def __init__(self, enable_timing=False):
        self.stream = None
        self.t = None
        FakeEvent.serials += 1
        self.serial = FakeEvent.serials
        self.queries_left = FakeEvent.lag

    def record(self, stream=None):
        self.stream = stream if stream is not None else FakeTorch.current[-1]
        self.t = time.perf_counter()
        if self.stream is not None:
            self.stream.log.append(("record", self.serial))

    def query(self):
        if self.queries_left:
            self.queries_left -= 1
            return False
        return True

    def synchronize(self):
        pass

    def elapsed_time(self, other):
        return (other.t - self.t) * 1e3


class _StreamCtx:
    def __init__(self, s):
        self.s = s

    def __enter__(self):
        FakeTorch.current.append(self.s)

    def __exit__(self, *a):
        FakeTorch.current.pop()


class FakeCuda:
    Stream = FakeStream
    Event = FakeEvent

    @staticmethod
    def synchronize():
        pass

    @staticmethod
    def stream(s):
        return _StreamCtx(s)


class FakeTorch:
    cuda = FakeCuda
    float32 = "float32"
    current = [None]            # stream contexts entered (None: the default stream)

    @staticmethod
    def empty_like(t):
        return FakeTensor(t.shape, "empty_like@" + str(FakeTorch.current[-1]))

    @staticmethod
    def empty(shape, dtype=None, device=None):
        return FakeTensor(shape, "empty@" + str(FakeTorch.current[-1]))


class FakeFilter:
    def __init__(self, m, points, poses, sigma, seed, tick=0, want_w=True, **kw):
        self.map, self.points, self.poses, self.sigma, self.seed, self.tick = m, points, poses, sigma, seed, tick
        self.made_in = FakeTorch.current[-1]
        self.poses_out = None
        self.logw = self.wq = self.log_z = self.idx = None

    @property
    def N(self):
        return self.poses.shape[1]


class Recorder:
    """Stands in for the library calls the engine makes."""

    def __init__(self, busy_first=0):
        self.ticks = []         # (stream, [(rid, seed, tick)])
        self.plain = []
        self.busy_left = busy_first
        self.busy_calls = set()  # indices of tick calls to refuse (0 = the first call)
        self.calls = 0

    def tick(self, filters, graph=False, stream=None, nowait=False):
        assert FakeTorch.current[-1] is stream, "tick enqueued outside its stream's context"
        call, self.calls = self.calls, self.calls + 1
        if self.busy_left or call in self.busy_calls:
            self.busy_left = max(0, self.busy_left - 1)
            return False
        # a robot's resampling seed is engine seed * 2^32 + robot id
        self.ticks.append((stream, [(f.seed & 0xFFFFFFFF, f.seed, f.tick) for f in filters]))
        return True

    def sensor_update(self, m, points, poses, sigma, logw, stream):
        self.plain.append(stream)

    def normalize(self, *a, **k):
        pass

    def resample(self, *a, **k):
        pass


@pytest.fixture
def lib(monkeypatch):
    rec = Recorder()
    monkeypatch.setattr(serve.mcl, "Filter", FakeFilter)
    monkeypatch.setattr(serve.mcl, "tick", rec.tick)
    monkeypatch.setattr(serve.mcl, "sensor_update", rec.sensor_update)
    monkeypatch.setattr(serve.mcl, "normalize", rec.normalize)
    monkeypatch.setattr(serve.mcl, "resample", rec.resample)
    monkeypatch.setattr(serve.mcl, "job_bytes", lambda N, K: 1000 * N + K)
    FakeTorch.current = [None]
    FakeEvent.lag = 0
    return rec


def make(n_robots, lib, phases=((None, "track"),), N=10, K=5):
    made = []

    def init(r, phase, stream, probe=False):
        if probe:
            return N
        made.append((r.rid, phase, stream, FakeTorch.current[-1]))
        return FakeTensor((12, N), "init")

    robots = [serve.Robot(i, "map", FakeTensor((3, K), "host"), 0.1, list(phases)) for i in range(n_robots)]
    return robots, init, made


def run(engine, trace):
    return engine.run(trace)


def test_latest_wins_and_one_update_in_flight(lib):
    robots, init, made = make(1, lib)
    eng = serve.Engine(robots, init, n_streams=1, torch_module=FakeTorch, seed=3)
    st = run(eng, [(0.0, 0), (0.0, 0), (0.0, 0)])
    assert st.arrived == 3 and st.dropped == 2 and st.completed == 1
    assert len(lib.ticks) == 1 and lib.ticks[0][1] == [(0, serve.robot_seed(3, 0), 0)]


def test_budget_admission_and_phase_release(lib):
    robots, init, made = make(3, lib, phases=((1, "global"), (None, "track")))
    budget = 1000 * 10 + 5          # one robot's job bytes
    eng = serve.Engine(robots, init, budget_bytes=budget, n_streams=1, torch_module=FakeTorch)
    st = run(eng, [(0.0, 0), (0.0, 1), (0.0, 2)])
    assert st.completed == 3 and st.max_resident_bytes <= budget
    assert [t[1][0][0] for t in lib.ticks] == [0, 1, 2]     # one at a time, as the budget frees
    assert all(r.phase == "track" and r.filt is None for r in robots)


def test_particles_and_buffers_made_on_the_ticks_stream(lib):
    """The advisor's race: a robot's particle set, its buffers and its filter are
    made inside the context of the stream its tick runs on."""
    robots, init, made = make(4, lib)
    eng = serve.Engine(robots, init, n_streams=2, max_evals_per_tick=2 * 10 * 5, torch_module=FakeTorch)
    st = run(eng, [(0.0, i) for i in range(4)])
    assert st.completed == 4
    tick_stream = {}
    for s, jobs in lib.ticks:
        for rid, _, _ in jobs:
            tick_stream[rid] = s
    for rid, phase, stream_arg, ctx in made:
        assert stream_arg is tick_stream[rid] and ctx is tick_stream[rid], (rid, stream_arg, ctx)
    for r in robots:
        assert r.filt.made_in is tick_stream[r.rid]
        assert r.poses.tag == "init" or r.poses.tag.startswith("empty_like@" + tick_stream[r.rid].name)


def test_uploads_are_ordered_around_the_tick(lib):
    robots, init, made = make(2, lib)
    eng = serve.Engine(robots, init, n_streams=1, torch_module=FakeTorch)
    run(eng, [(0.0, 0), (0.0, 1)])
    s, cs = eng.streams[0], eng.copy_stream
    # the copy stream waited for the tick's stream, copied, recorded an event; the
    # tick's stream waited for that event
    assert ("wait_stream", s.name) in cs.log
    rec = [e for e in cs.log if e[0] == "record"]
    assert rec and ("wait_event", cs.name, rec[0][1]) in s.log
    for r in robots:
        assert r.points is None or all(c[1] is cs and c[2] for c in r.points.copies)
    assert eng.stats.uploaded_bytes == 2 * 3 * 5 * 4


def test_busy_tick_is_retried(lib):
    lib.busy_left = 2
    robots, init, made = make(2, lib)
    eng = serve.Engine(robots, init, n_streams=1, torch_module=FakeTorch)
    st = run(eng, [(0.0, 0), (0.0, 1)])
    assert st.busy == 2 and st.completed == 2 and st.dropped == 0


def test_busy_retry_on_another_stream_waits_for_the_initialisation(lib):
    """Robot 0's tick runs on stream 1; robot 1 is admitted while its tick is
    built for stream 2, that tick is refused as busy, and once robot 0's tick
    has completed the retry runs on stream 1: the copy stream must have waited
    for the event recorded on stream 2 after robot 1's particle set was made,
    and stream 1 for the copy."""
    lib.busy_calls = {1}
    FakeEvent.lag = 1
    robots, init, made = make(2, lib)
    eng = serve.Engine(robots, init, n_streams=2, max_evals_per_tick=10 * 5, torch_module=FakeTorch)
    st = run(eng, [(0.0, 0), (0.0, 1)])
    s1, s2, cs = eng.streams[0], eng.streams[1], eng.copy_stream
    assert st.busy == 1 and st.completed == 2
    assert [(t[0], t[1][0][0]) for t in lib.ticks] == [(s1, 0), (s1, 1)]
    (rid, phase, stream_arg, ctx), = [m for m in made if m[0] == 1]
    assert stream_arg is s2 and ctx is s2
    ready = [e for e in s2.log if e[0] == "record"]
    assert ready, s2.log
    ready_serial = ready[0][1]
    i_wait = cs.log.index(("wait_event", s2.name, ready_serial))
    # the copy event recorded after that wait is one stream 1 waited for
    later = [e[1] for e in cs.log[i_wait:] if e[0] == "record"]
    assert any(("wait_event", cs.name, serial) in s1.log for serial in later)
    assert all(r.ready is None for r in robots)


@pytest.mark.parametrize("order", ["fifo", "stale"])
def test_request_order(lib, order):
    """Robot 0 completes an update first; then both robots wait, robot 0's scan
    the older one: fifo serves robot 0 first, stale serves robot 1 (never
    updated) first."""
    robots, init, made = make(2, lib)
    eng = serve.Engine(robots, init, plain=True, torch_module=FakeTorch, order=order)
    robots[0].last_done = 0.5              # robot 0 was updated recently
    robots[0].pending, robots[1].pending = 0.01, 0.02
    robots[0].in_flight = robots[1].in_flight = None
    eng.stats.arrived = 2
    st = run(eng, [])
    assert st.completed == 2
    # one request at a time: the robot whose particle set was made first went first
    assert made[0][0] == (0 if order == "fifo" else 1)


def test_request_log_lines(lib):
    """One JSON line per completed update, with the robot, map, phase, sizes,
    tick and stream, and times ordered arrival <= enqueue <= completion; the
    time the particle set became resident precedes the enqueue, and precedes
    the arrival too once a tracking robot stays resident."""
    import io
    import json

    robots, init, made = make(3, lib, phases=((1, "global"), (None, "track")), N=10, K=5)
    for i, r in enumerate(robots):
        r.map_id = i % 2
    buf = io.StringIO()
    eng = serve.Engine(robots, init, n_streams=2, max_evals_per_tick=2 * 10 * 5, torch_module=FakeTorch, log=buf)
    st = run(eng, [(0.0, 0), (0.0, 1), (0.0, 2), (0.02, 0), (0.04, 0)])
    lines = [json.loads(x) for x in buf.getvalue().splitlines()]
    assert len(lines) == st.completed == 5 and st.dropped == 0
    for x in lines:
        assert x["map"] == x["robot"] % 2
        assert x["N"] == 10 and x["K"] == 5 and x["evals"] == 50
        assert x["arrival_s"] <= x["enqueued_s"] <= x["done_s"]
        assert x["resident_s"] <= x["enqueued_s"]
        assert abs(x["latency_ms"] - (x["done_s"] - x["arrival_s"]) * 1e3) < 1e-9
        assert 0 <= x["tick"] < st.ticks and x["stream"] in (0, 1)
    r0 = [x for x in lines if x["robot"] == 0]
    assert [x["phase"] for x in r0] == ["global", "track", "track"]
    # the global phase's set was released; the tracking set stayed resident
    assert r0[0]["resident_s"] < r0[1]["resident_s"] == r0[2]["resident_s"] < r0[2]["arrival_s"]
    # the statistics split each latency into the wait for a stream and the service
    for lat, w, sv in zip(st.latencies_ms, st.waits_ms, st.service_ms):
        assert w >= 0 and sv >= 0 and abs(lat - (w + sv)) < 1e-9
    bp = st.by_phase()
    assert set(bp) == {"global", "track"} and bp["global"]["completed"] == 3
    assert all(k in bp["track"] for k in ("p99_ms", "wait_p50_ms", "wait_p99_ms", "service_p50_ms", "service_p99_ms"))


def test_small_request_lane(lib):
    """With a small-request lane, stream 0 takes only requests of at most the
    lane's evaluations and the other stream any: the large request (robot 0,
    1000 particles) runs on stream 1 while the small ones (robots 1 and 2, 10
    particles) run together on stream 0 in the same pass; a lone large request
    leaves stream 0 idle.  Without the lane the first free stream takes the
    oldest request, large or small."""
    K = 5
    sizes = {0: 1000, 1: 10, 2: 10}

    def init(r, phase, stream, probe=False):
        return sizes[r.rid] if probe else FakeTensor((12, sizes[r.rid]), "init")

    def robots():
        return [serve.Robot(i, "map", FakeTensor((3, K), "host"), 0.1, [(None, "track")]) for i in range(3)]

    eng = serve.Engine(robots(), init, n_streams=2, max_evals_per_tick=1e9, torch_module=FakeTorch,
                       small_lane_evals=100)
    st = eng.run([(0.0, 0), (0.0, 1), (0.0, 2)])
    assert st.completed == 3
    on = {rid: s for s, jobs in lib.ticks for rid, _, _ in jobs}
    assert on[0] is eng.streams[1] and on[1] is eng.streams[0] and on[2] is eng.streams[0]
    assert len(lib.ticks) == 2
    # a lone large request: stream 0 never runs it
    lib.ticks.clear()
    eng = serve.Engine(robots(), init, n_streams=2, torch_module=FakeTorch, small_lane_evals=100)
    eng.run([(0.0, 0), (0.01, 0), (0.02, 0)])
    assert lib.ticks and all(s is eng.streams[1] for s, _ in lib.ticks)
    # without the lane: oldest first on the first free stream, one stream per pass
    lib.ticks.clear()
    eng = serve.Engine(robots(), init, n_streams=2, max_evals_per_tick=1e9, torch_module=FakeTorch)
    eng.run([(0.0, 0), (0.0, 1), (0.0, 2)])
    assert lib.ticks[0][0] is eng.streams[0] and lib.ticks[0][1][0][0] == 0
    with pytest.raises(ValueError):
        serve.Engine(robots(), init, n_streams=1, torch_module=FakeTorch, small_lane_evals=100)
