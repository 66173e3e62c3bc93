"""The served workload: many robots localising in several resident maps.

Four int16 warehouse maps (512x512x64, 1024x1024x128 and 2048x2048x128 at
0.05 m; 1024x1024x256 at 0.1 m), object counts scaled to floor area; 256
robots, 64 per map, each with a ground-truth pose and a VLP-16-shaped or
OS0-64-shaped scan (a few distinct scans per map, shared by its robots);
requests form a Poisson process at 10 Hz per robot, first arrivals staggered
over 10 s; a robot's first five accepted updates use a global particle set
(N log-uniform in [262144, 1048576], uniform over free voxels), later ones a
tracking set (N log-uniform in [4096, 32768], spread round the true pose at
0.5 m and 5 degrees).  Only the counts and the true poses are generated here:
the particle sets themselves are made on the device by the library's
initialisation calls.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .configs import (DEG, OS0_64, VLP16, beam_dirs, ground_truth_pose, pose_matrix, raycast_scan, rng,
                      warehouse_scene)
from .tsdf import build_map, f32

CFG = 5
MAP_SPECS = [  # dims, voxel, tau
    ((512, 512, 64), 0.05, 0.15),
    ((1024, 1024, 128), 0.05, 0.15),
    ((2048, 2048, 128), 0.05, 0.15),
    ((1024, 1024, 256), 0.1, 0.3),
]


@dataclass
class RobotSpec:
    rid: int
    map_idx: int
    scan_idx: int
    gt: tuple           # (xyz float64[3], rpy float64[3])
    n_global: int
    n_track: int


@dataclass
class ServedWorkload:
    tmaps: list          # TsdfMap per map
    scans: list          # per map: list of [3, K] float32
    robots: list         # RobotSpec
    trace: list          # (arrival_s, robot_id), sorted
    global_updates: int = 5


def build(n_robots: int = 256, trace_s: float = 30.0, rate_hz: float = 10.0, scans_per_map: int = 4,
          map_subset=None, stagger_s: float = 10.0) -> ServedWorkload:
    """The served workload; robots' first requests arrive uniformly within
    stagger_s seconds, then at `rate_hz` (Poisson) until trace_s."""
    tmaps, scans, scenes = [], [], []
    specs = MAP_SPECS if map_subset is None else [MAP_SPECS[i] for i in map_subset]
    for mi, (dims, v, tau) in enumerate(specs):
        ext = (dims[0] * v, dims[1] * v, dims[2] * v)
        area = ext[0] * ext[1] / (51.2 * 51.2)
        sc = warehouse_scene(rng(CFG, 0, mi), extent=ext, n_boxes=int(round(300 * area)), n_cyl=int(round(80 * area)))
        tm = build_map(sc, dims, v, (0.0, 0.0, 0.0), tau, "i16")
        lst = []
        for s in range(scans_per_map):
            gxyz, grpy = ground_truth_pose(rng(CFG, 1, 1000 * mi + s), sc, (1.0, 1.0), (ext[0] - 1.0, ext[1] - 1.0),
                                           sc.floor_z)
            R, t = pose_matrix(gxyz, grpy)
            if s % 2 == 0:
                pts = raycast_scan(sc, tm, R, t, beam_dirs(azimuths=1800, **VLP16), 100.0, 0.03, rng(CFG, 2, 1000 * mi + s))
            else:
                pts = raycast_scan(sc, tm, R, t, beam_dirs(azimuths=1024, **OS0_64), 50.0, 0.02, rng(CFG, 2, 1000 * mi + s))
            lst.append((pts, (gxyz, grpy)))
        tmaps.append(tm)
        scans.append([p for p, _ in lst])
        scenes.append(lst)
    r = rng(CFG, 3)
    robots = []
    for rid in range(n_robots):
        mi = rid % len(tmaps)
        si = (rid // len(tmaps)) % scans_per_map
        ng = int(round(math.exp(r.uniform(math.log(262144), math.log(1048576)))))
        nt = int(round(math.exp(r.uniform(math.log(4096), math.log(32768)))))
        robots.append(RobotSpec(rid, mi, si, scenes[mi][si][1], ng, nt))
    tr = rng(CFG, 4)
    trace = []
    for rid in range(n_robots):
        t = tr.uniform(0.0, stagger_s)
        while t < trace_s:
            trace.append((t, rid))
            t += tr.exponential(1.0 / rate_hz)
    trace.sort()
    return ServedWorkload(tmaps, scans, robots, trace)


def pose12(gt) -> np.ndarray:
    """A ground-truth pose (xyz, roll/pitch/yaw) as 12 float32 values: R row-major, t."""
    R, t = pose_matrix(gt[0], gt[1])
    return np.concatenate([np.asarray(R, np.float64).ravel(), np.asarray(t, np.float64)]).astype(np.float32)


TRACK_SIGMA_T = 0.5            # metres
TRACK_SIGMA_R = 5.0 * DEG      # radians
MAX_TILT = 5.0 * DEG           # global phase: |roll|, |pitch| bound


def sigma_for(tmap) -> float:
    return f32(tmap.tau / 2)
