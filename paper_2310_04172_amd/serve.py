"""Serving: continuous batching of sensor updates from many robots.

Requests (a robot's new scan) arrive over time.  The engine keeps every
admitted robot's particle set resident in device memory and, whenever one of
its streams is free, gathers the waiting requests of robots that are not
already on the GPU into one batched tick (``mcl_tick``: sensor update,
normalisation and resampling of every filter in one launch per stage).  Up to
``n_streams * depth`` ticks are in flight: with two streams a new tick runs
beside the previous one on the device; with one stream and depth 2 the next
tick is queued behind the running one.

* Each request carries its scan in pinned host memory.  When the request is
  taken, the scan is copied to the robot's device buffer on a copy stream and
  the tick's stream waits for that copy (an event), so uploads overlap the
  ticks already running; the latency includes the upload.
* Latest wins: a robot keeps at most one waiting request; a newer scan replaces
  an older one that has not started (counted as dropped, as a localiser drops
  stale scans).  A robot has at most one update in flight.
* Order: waiting requests are taken oldest scan first (``order="fifo"``), or
  the robot whose last completed update is oldest first (``order="stale"``:
  every robot's pose is kept as fresh as the device allows; under overload the
  scan served is then one that arrived recently, not one that waited longest).
* Admission: a robot becomes resident when its device state (``mcl_job_bytes``)
  fits the memory budget; until then its request waits.  Its particle set is
  made by the library's initialisation calls on the stream of the tick being
  built, and an event recorded there after them orders the robot's first
  upload (and so its first tick) after them, also when that tick is refused
  as busy and the robot is then served on another stream.
* Resampling draws: robot r's n-th completed update uses seed
  ``seed * 2^32 + r`` and tick n (the library's draw), so results do not depend
  on batching or timing.
* Latency is measured from a request's arrival to the GPU completion of its
  tick, read from device events against a reference event.

The robots' initial particle sets (global or round a pose, per phase) come from
a caller-supplied function of (robot, phase, stream) that calls the library.
"""

from __future__ import annotations

import collections
import json
import time
from dataclasses import dataclass, field

import numpy as np

from . import mcl


def robot_seed(seed: int, rid: int) -> int:
    """Resampling seed of robot `rid` in an engine seeded with `seed`."""
    return ((int(seed) << 32) + int(rid)) & (2 ** 64 - 1)


class LibraryInit:
    """Initial particle sets made by the library, for Engine's init_particles:
    a 'global' phase uniform over the map's free voxels (mcl_init_uniform,
    roll and pitch within max_tilt), a 'track' phase round the robot's pose
    estimate (mcl_init_gaussian).  counts[rid][phase] is the particle count,
    means[rid] the estimate (12 floats, R row-major and t).  The random numbers
    of robot r's phase p are fixed by (seed, r, p)."""

    PHASES = ("global", "track")

    def __init__(self, counts, means, max_tilt: float, sigma_t: float, sigma_r: float, seed: int = 0):
        self.counts, self.means = counts, means
        self.max_tilt, self.sigma_t, self.sigma_r = float(max_tilt), float(sigma_t), float(sigma_r)
        self.seed = int(seed)

    def __call__(self, r, phase: str, stream, probe: bool = False):
        n = int(self.counts[r.rid][phase])
        if probe:
            return n
        key = robot_seed(self.seed, r.rid)
        step = self.PHASES.index(phase)
        if phase == "global":
            return mcl.init_uniform(r.map, n, self.max_tilt, key ^ (step << 62), stream=stream)
        return mcl.init_gaussian(self.means[r.rid], n, self.sigma_t, self.sigma_r, key, step, stream=stream)


@dataclass
class Robot:
    rid: int
    map: "mcl.Map"
    host_points: object         # pinned host [3, K] float32: the scan every request carries
    sigma: float
    phases: list                # [(n_updates or None for the rest, phase name)]
    completed: int = 0
    phase_i: int = 0
    points: object = None       # device [3, K] upload target (while resident)
    poses: object = None        # device [12, N] current particle set
    spare: object = None        # device [12, N] resample target
    filt: object = None
    bytes: int = 0
    pending: float | None = None
    in_flight: float | None = None
    evals_done: int = 0
    last_done: float = -1.0     # completion time of the last update (-1: none yet)
    ready: object = None        # event after the initialisation, until the first update is enqueued
    map_id: int = -1            # which resident map (for the request log)
    resident: float | None = None   # when the robot's current particle set was made resident
    started: float | None = None    # when its update in flight was enqueued
    tick_no: int = -1               # the tick that carries it

    @property
    def K(self):
        return self.host_points.shape[1]

    @property
    def phase(self):
        return self.phases[self.phase_i][1]


@dataclass
class ServeStats:
    latencies_ms: list = field(default_factory=list)
    waits_ms: list = field(default_factory=list)    # arrival to enqueue (waiting for a stream / admission)
    service_ms: list = field(default_factory=list)  # enqueue to completion (its tick, and ticks queued before it)
    phases: list = field(default_factory=list)      # the robot's phase of each completed update
    completed: int = 0
    dropped: int = 0
    arrived: int = 0
    evals: int = 0
    ticks: int = 0
    busy: int = 0               # ticks refused by the library (MCL_EBUSY) and retried later
    uploaded_bytes: int = 0
    max_resident_bytes: int = 0
    wall_s: float = 0.0

    def summary(self) -> dict:
        lat = np.asarray(self.latencies_ms) if self.latencies_ms else np.zeros(1)
        return {"p10_ms": float(np.percentile(lat, 10)), "p50_ms": float(np.percentile(lat, 50)),
                "p90_ms": float(np.percentile(lat, 90)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()), "completed": self.completed, "arrived": self.arrived,
                "dropped": self.dropped, "drop_rate": self.dropped / max(1, self.arrived),
                "evals_per_s": self.evals / max(self.wall_s, 1e-9), "ticks": self.ticks, "busy": self.busy,
                "uploaded_MB": self.uploaded_bytes / 1e6,
                "max_resident_GiB": self.max_resident_bytes / 2 ** 30, "wall_s": self.wall_s,
                "by_phase": self.by_phase()}

    def by_phase(self) -> dict:
        """Completed updates per robot phase: p50 / p99 of the latency and of its
        two parts, the wait for a stream and the service once enqueued."""
        out = {}
        ph = np.asarray(self.phases)
        parts = {"": np.asarray(self.latencies_ms), "wait_": np.asarray(self.waits_ms),
                 "service_": np.asarray(self.service_ms)}
        for name in sorted(set(self.phases)):
            sel = ph == name
            d = {"completed": int(sel.sum())}
            for pre, a in parts.items():
                if a.size == ph.size:
                    d[f"{pre}p50_ms"] = float(np.percentile(a[sel], 50))
                    d[f"{pre}p99_ms"] = float(np.percentile(a[sel], 99))
            out[name] = d
        return out


class Engine:
    """Continuous-batching server over mcl_tick (or, with plain=True, the same
    trace served one request at a time with the single-filter calls).

    init_particles(robot, phase, stream, probe=False): with probe, the particle
    count of the robot's set for that phase; else the set itself, a device
    [12, N] tensor made on `stream` by the library's initialisation calls.
    on_complete(robot, filter): optional, called when an update has completed,
    before the resampled set becomes the robot's particle set (tests read the
    update's inputs and outputs there).
    torch_module: the torch module the engine takes streams, events and buffers
    from (default: torch itself; tests of the host logic pass a stand-in).
    log: optional text stream; one JSON line per completed update (robot, map,
    phase, N, K, evaluations, tick, stream, and in seconds from the start of the
    run the request's arrival, enqueue and completion and the time the robot's
    particle set was made resident, which precedes the arrival for a robot that
    stays resident between updates).
    small_lane_evals: optional; with two or more streams, stream 0 takes only
    requests of at most this many particle-point evaluations (the other streams
    take any), so small updates (tracking) never queue behind large ones (global
    localisation) for a stream; it stays idle while no small request waits."""

    def __init__(self, robots, init_particles, budget_bytes: int = 64 << 30, max_evals_per_tick: float = 1.2e11,
                 n_streams: int = 2, plain: bool = False, graph: bool = False, seed: int = 0, depth: int = 1,
                 order: str = "fifo", on_complete=None, torch_module=None, log=None, small_lane_evals=None):
        if torch_module is None:
            import torch as torch_module
        torch = self.torch = torch_module
        self.robots = robots
        self.init_particles = init_particles
        self.budget = int(budget_bytes)
        self.max_evals = float(max_evals_per_tick)
        self.plain = plain
        self.graph = graph and not plain
        self.seed = seed
        self.on_complete = on_complete
        self.log = log
        self._t0 = time.perf_counter()
        self.streams = [torch.cuda.Stream() for _ in range(1 if plain else n_streams)]
        self.copy_stream = torch.cuda.Stream()
        self.depth = 1 if plain else max(1, int(depth))    # ticks in flight per stream
        if order not in ("fifo", "stale"):
            raise ValueError("order must be 'fifo' or 'stale'")
        self.order = order
        if small_lane_evals is not None and len(self.streams) < 2:
            raise ValueError("a small-request lane needs two or more streams")
        self.small_lane = None if small_lane_evals is None else float(small_lane_evals)
        self.used = 0
        self.stats = ServeStats()

    # -------------------------------------------------------------- state
    def _admit(self, r: Robot, stream) -> bool:
        """Make r resident: its buffers and initial particle set, on `stream`."""
        if r.filt is not None:
            return True
        torch = self.torch
        N = self.init_particles(r, r.phase, stream, probe=True)
        need = mcl.job_bytes(N, r.K)
        if self.used + need > self.budget:
            return False
        with torch.cuda.stream(stream):
            r.poses = self.init_particles(r, r.phase, stream)
            r.spare = torch.empty_like(r.poses)
            r.points = torch.empty((3, r.K), dtype=torch.float32, device=r.poses.device)
            r.filt = mcl.Filter(r.map, r.points, r.poses, r.sigma, robot_seed(self.seed, r.rid), want_w=False)
        r.ready = torch.cuda.Event()
        r.ready.record(stream)
        r.resident = time.perf_counter() - self._t0
        r.filt.poses_out = r.spare
        r.bytes = need
        self.used += need
        self.stats.max_resident_bytes = max(self.stats.max_resident_bytes, self.used)
        return True

    def _release(self, r: Robot):
        r.filt = r.ready = None
        r.poses = r.spare = r.points = None
        self.used -= r.bytes
        r.bytes = 0

    def _finish(self, r: Robot, t_done: float, si: int):
        if self.on_complete is not None:
            self.on_complete(r, r.filt)
        self.stats.latencies_ms.append((t_done - r.in_flight) * 1e3)
        self.stats.waits_ms.append((r.started - r.in_flight) * 1e3)
        self.stats.service_ms.append((t_done - r.started) * 1e3)
        self.stats.phases.append(r.phase)
        self.stats.completed += 1
        n_evals = r.poses.shape[1] * r.K
        if self.log is not None:
            self.log.write(json.dumps({
                "robot": r.rid, "map": r.map_id, "phase": r.phase, "N": int(r.poses.shape[1]), "K": int(r.K),
                "evals": int(n_evals), "tick": r.tick_no, "stream": si, "arrival_s": r.in_flight,
                "resident_s": r.resident, "enqueued_s": r.started, "done_s": t_done,
                "latency_ms": (t_done - r.in_flight) * 1e3}) + "\n")
        self.stats.evals += n_evals
        r.evals_done += n_evals
        r.in_flight = None
        r.last_done = t_done
        r.completed += 1
        r.poses, r.spare = r.spare, r.poses          # the resampled set is the new particle set
        r.filt.poses, r.filt.poses_out = r.poses, r.spare
        limit = self.phases_limit(r)
        if limit is not None and r.completed >= limit:
            self._release(r)
            r.phase_i += 1

    @staticmethod
    def phases_limit(r: Robot):
        n = 0
        for i, (count, _) in enumerate(r.phases):
            if count is None:
                return None
            n += count
            if i == r.phase_i:
                return n
        return None

    def _upload(self, batch, s):
        """Copy the batch's scans from pinned host memory on the copy stream; the
        tick's stream `s` waits for them.  The copies wait for s and for the
        initialisation of robots admitted on any stream and not yet served."""
        torch = self.torch
        cs = self.copy_stream
        cs.wait_stream(s)
        for r in batch:
            if r.ready is not None:
                cs.wait_event(r.ready)
        with torch.cuda.stream(cs):
            for r in batch:
                r.points.copy_(r.host_points, non_blocking=True)
                self.stats.uploaded_bytes += r.host_points.numel() * 4
        ev = torch.cuda.Event()
        ev.record(cs)
        s.wait_event(ev)

    def _submit(self, batch, s) -> bool:
        """Enqueue one update of every robot in `batch` on stream s; False if
        the library reports the stream's staging buffer busy (nothing enqueued)."""
        torch = self.torch
        for r in batch:
            r.filt.tick = r.completed
        with torch.cuda.stream(s):
            if self.plain:
                f = batch[0].filt
                mcl.sensor_update(f.map, f.points, f.poses, f.sigma, f.logw, s)
                mcl.normalize(f.logw, None, f.wq, f.log_z, want_w=False, stream=s)
                mcl.resample(f.wq, f.seed, f.tick, f.poses, f.poses_out, f.idx, s)
                return True
            return mcl.tick([r.filt for r in batch], graph=self.graph, stream=s, nowait=True)

    # ---------------------------------------------------------------- run
    def run(self, trace, drain: bool = True) -> ServeStats:
        torch = self.torch
        st = self.stats
        ref = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = self._t0 = time.perf_counter()
        ref.record()
        ref.synchronize()
        t_ref = time.perf_counter() - t0
        inflight = collections.deque()        # (event, robots, stream index)
        busy = [0] * len(self.streams)        # ticks in flight per stream
        ptr = 0
        while True:
            now = time.perf_counter() - t0
            progressed = False
            while ptr < len(trace) and trace[ptr][0] <= now:
                t, rid = trace[ptr]
                r = self.robots[rid]
                if r.pending is not None:
                    st.dropped += 1
                r.pending = t
                st.arrived += 1
                ptr += 1
                progressed = True
            for item in list(inflight):
                ev, rs, si = item
                if ev.query():
                    t_done = t_ref + ref.elapsed_time(ev) * 1e-3
                    for r in rs:
                        self._finish(r, t_done, si)
                    inflight.remove(item)
                    busy[si] -= 1
                    progressed = True
            free = [i for i, b in enumerate(busy) if b < self.depth]
            key = (lambda r: r.pending) if self.order == "fifo" else (lambda r: (r.last_done, r.pending))
            cands = sorted((r for r in self.robots if r.pending is not None and r.in_flight is None), key=key) \
                if free else []
            # the small-request lane (stream 0) is tried first, then the other free streams
            for si in free:
                s = self.streams[si]
                lane = self.small_lane is not None and si == 0
                batch, evals = [], 0.0
                for r in cands:
                    if r.in_flight is not None:      # taken by the other stream in this pass
                        continue
                    e = self.init_particles(r, r.phase, s, probe=True) * r.K if r.filt is None else \
                        r.poses.shape[1] * r.K
                    if lane and e > self.small_lane:
                        continue
                    if batch and (self.plain or evals + e > self.max_evals):
                        break
                    if not self._admit(r, s):
                        continue
                    batch.append(r)
                    evals += e
                if batch:
                    self._upload(batch, s)
                    if self._submit(batch, s):
                        t_sub = time.perf_counter() - t0
                        for r in batch:
                            r.in_flight, r.pending, r.ready = r.pending, None, None
                            r.started, r.tick_no = t_sub, st.ticks
                        ev = torch.cuda.Event(enable_timing=True)
                        ev.record(s)
                        inflight.append((ev, batch, si))
                        busy[si] += 1
                        st.ticks += 1
                        progressed = True
                    else:
                        st.busy += 1
                if self.small_lane is None:
                    break                            # one stream per pass, as before the lane existed
            if ptr >= len(trace) and not inflight and (not drain or not any(
                    r.pending is not None for r in self.robots)):
                break
            if not progressed:
                time.sleep(0.0002)
        torch.cuda.synchronize()
        st.wall_s = time.perf_counter() - t0
        return st
