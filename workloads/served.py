"""The served workload: many robots localising in several resident maps.

Four int16 warehouse maps (512x512x64, 1024x1024x128 and 2048x2048x128 at
0.05 m; 1024x1024x256 at 0.1 m), object counts scaled to floor area; 256
robots, 64 per map, each with a ground-truth pose and a VLP-16-shaped or
OS0-64-shaped scan (a few distinct scans per map, shared by its robots);
requests form a Poisson process at 10 Hz per robot, first arrivals staggered
over 10 s; a robot's first five accepted updates use a global particle set
(N log-uniform in [262144, 1048576], uniform over free voxels), later ones a
tracking set (N log-uniform in [4096, 32768], Gaussian around the true pose).

Particle sets are sampled on the device with torch's seeded generator (input
generation only: none of the sensor model's arithmetic).
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
          map_subset=None) -> ServedWorkload:
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
        t = tr.uniform(0.0, 10.0)
        while t < trace_s:
            trace.append((t, rid))
            t += tr.exponential(1.0 / rate_hz)
    trace.sort()
    return ServedWorkload(tmaps, scans, robots, trace)


def device_particles(torch, tmap, map_values_dev, n: int, kind: str, gt, seed: int, device):
    """[12, n] float32 poses on the device: 'global' uniform over free voxels (stored
    value > 0) with jitter, yaw uniform, roll/pitch within 5 degrees; 'track'
    Gaussian around gt (0.5 m, 5 degrees)."""
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    f64 = torch.float64
    if kind == "global":
        flat = map_values_dev.reshape(-1)
        nx, ny, _ = tmap.dims
        chunks, need = [], n
        while need > 0:
            lin = torch.randint(0, flat.numel(), (int(need * 1.4) + 64,), generator=g, device=device)
            lin = lin[flat[lin] > 0][:need]
            chunks.append(lin)
            need -= lin.numel()
        lin = torch.cat(chunks)
        k = lin // (nx * ny)
        rem = lin - k * (nx * ny)
        j = rem // nx
        i = rem - j * nx
        ijk = torch.stack([i, j, k], 1).to(f64)
        xyz = torch.tensor(tmap.origin, dtype=f64, device=device) + \
            (ijk + torch.rand((n, 3), generator=g, device=device, dtype=f64)) * float(tmap.voxel)
        u = torch.rand((n, 3), generator=g, device=device, dtype=f64)
        roll = (u[:, 0] * 10 - 5) * DEG
        pitch = (u[:, 1] * 10 - 5) * DEG
        yaw = (u[:, 2] * 2 - 1) * math.pi
    else:
        gxyz, grpy = gt
        xyz = torch.tensor(gxyz, dtype=f64, device=device) + 0.5 * torch.randn((n, 3), generator=g, device=device, dtype=f64)
        e = torch.tensor(grpy, dtype=f64, device=device) + 5 * DEG * torch.randn((n, 3), generator=g, device=device, dtype=f64)
        roll, pitch, yaw = e[:, 0], e[:, 1], e[:, 2]
    cr, sr, cp, sp, cy, sy = (torch.cos(roll), torch.sin(roll), torch.cos(pitch), torch.sin(pitch),
                              torch.cos(yaw), torch.sin(yaw))
    rows = [cy * cp, cy * sp * sr - sy * cr, cy * sp * cr + sy * sr,
            sy * cp, sy * sp * sr + cy * cr, sy * sp * cr - cy * sr,
            -sp, cp * sr, cp * cr,
            xyz[:, 0], xyz[:, 1], xyz[:, 2]]
    return torch.stack(rows, 0).to(torch.float32).contiguous()


def sigma_for(tmap) -> float:
    return f32(tmap.tau / 2)
