"""The five synthetic workloads, built from seeds.

They stand in for the paper's missing data: the simulated office with a virtual
VLP-16 and the HILTI drone arena recorded with an OS0-64 (§VI).  Beam geometry
follows those sensors; scenes are procedural (floor, boxes, walls, cylinders).

Seeds: numpy ``default_rng((cfg, component, index))`` with components
0 scene, 1 ground-truth pose, 2 range noise, 3 particles, 4 subset choice; the
resampling seed of filter f of config c is c * 2^32 + f (its first update is
tick 0).

Poses are handed to the library as 12 float32 rows (structure of arrays):
r00 r01 r02 r10 r11 r12 r20 r21 r22 tx ty tz, the rotation row-major and the
translation of the sensor in the world frame.  Points are float32 rows x, y, z in
the sensor frame, ring-major (all azimuths of ring 0, then ring 1, ...), misses
dropped.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .scene import Scene, euler_zyx_to_matrix
from .tsdf import TsdfMap, build_map, f32

DEG = math.pi / 180.0


def rng(cfg: int, component: int, index: int = 0) -> np.random.Generator:
    return np.random.default_rng((cfg, component, index))


# --------------------------------------------------------------------- scenes
def office_scene(r: np.random.Generator, extent=(12.8, 12.8), floor_z=1.0, n_boxes=20,
                 side=(0.5, 4.0)) -> Scene:
    """Floor plus boxes resting on it, sides uniform per axis, centres uniform in xy."""
    s = Scene(floor_z=floor_z)
    sides = r.uniform(side[0], side[1], size=(n_boxes, 3))
    cxy = r.uniform(0.0, 1.0, size=(n_boxes, 2)) * np.asarray(extent)
    lo = np.column_stack([cxy - sides[:, :2] / 2, np.full(n_boxes, floor_z)])
    hi = np.column_stack([cxy + sides[:, :2] / 2, floor_z + sides[:, 2]])
    s.boxes = np.hstack([lo, hi])
    return s


def warehouse_scene(r: np.random.Generator, extent=(51.2, 51.2, 6.4), floor_z=0.3,
                    n_boxes=300, n_cyl=80, wall=0.3, inset=0.7) -> Scene:
    """Floor, four perimeter walls, boxes and full-height vertical cylinders."""
    ex, ey, ez = extent
    top = ez + 1.0
    s = Scene(floor_z=floor_z)
    a0, a1 = inset, inset + wall
    walls = np.array([
        [a0, a0, floor_z, ex - a0, a1, top],
        [a0, ey - a1, floor_z, ex - a0, ey - a0, top],
        [a0, a0, floor_z, a1, ey - a0, top],
        [ex - a1, a0, floor_z, ex - a0, ey - a0, top],
    ])
    lo_in, hi_in = np.array([a1, a1]), np.array([ex - a1, ey - a1])
    sxy = r.uniform(0.5, 3.0, size=(n_boxes, 2))
    h = r.uniform(0.5, 4.0, size=n_boxes)
    c = lo_in + r.uniform(0.0, 1.0, size=(n_boxes, 2)) * (hi_in - lo_in)
    boxes = np.column_stack([c - sxy / 2, np.full(n_boxes, floor_z), c + sxy / 2, floor_z + h])
    s.boxes = np.vstack([walls, boxes])
    rad = r.uniform(0.2, 0.6, size=n_cyl)
    cc = lo_in + r.uniform(0.0, 1.0, size=(n_cyl, 2)) * (hi_in - lo_in)
    s.cylinders = np.column_stack([cc, rad, np.full(n_cyl, floor_z), np.full(n_cyl, top)])
    return s


# ---------------------------------------------------------------------- beams
def beam_dirs(rings: int, azimuths: int, el_lo_deg: float, el_hi_deg: float) -> np.ndarray:
    """Unit beam directions in the sensor frame, ring-major, float64 [rings*azimuths, 3]."""
    el = np.deg2rad(np.linspace(el_lo_deg, el_hi_deg, rings))
    az = np.arange(azimuths) * (2 * math.pi / azimuths)
    E, A = np.meshgrid(el, az, indexing="ij")
    d = np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], axis=-1)
    return d.reshape(-1, 3)


VLP16 = dict(rings=16, el_lo_deg=-15.0, el_hi_deg=15.0)
OS0_64 = dict(rings=64, el_lo_deg=-45.0, el_hi_deg=45.0)


def raycast_scan(scene: Scene, tmap: TsdfMap, R: np.ndarray, t: np.ndarray, dirs_s: np.ndarray,
                 max_range: float, sigma_r: float, r: np.random.Generator) -> np.ndarray:
    """Points [3, K] float32 in the sensor frame; a beam is a miss (dropped) when it hits
    nothing within max_range or its hit lies outside the map box."""
    dirs_w = dirs_s @ R.T
    rng_hit = scene.raycast(t, dirs_w)
    lo = np.asarray(tmap.origin, np.float64)
    hi = lo + np.array(tmap.dims, np.float64) * float(tmap.voxel)
    hit = np.isfinite(rng_hit) & (rng_hit <= max_range)
    pw = t[None, :] + np.where(hit, rng_hit, 0.0)[:, None] * dirs_w
    hit &= np.all((pw >= lo) & (pw < hi), axis=1)
    noise = r.normal(0.0, sigma_r, size=rng_hit.shape)
    rr = (rng_hit + noise)[hit]
    p = dirs_s[hit] * rr[:, None]
    return np.ascontiguousarray(p.T.astype(np.float32))


# ------------------------------------------------------------------ particles
def poses_soa(xyz: np.ndarray, rpy: np.ndarray) -> np.ndarray:
    """[12, N] float32: rotation rows (ZYX Euler -> matrix in float64, then rounded) and t."""
    R = euler_zyx_to_matrix(rpy[:, 0], rpy[:, 1], rpy[:, 2])
    out = np.empty((12, xyz.shape[0]), np.float32)
    out[:9] = R.reshape(-1, 9).T
    out[9:] = xyz.T
    return out


def pose_matrix(xyz, rpy):
    return euler_zyx_to_matrix(rpy[0], rpy[1], rpy[2]), np.asarray(xyz, np.float64)


def gaussian_particles(r, gt_xyz, gt_rpy, n, s_xyz=0.5, s_rpy_deg=5.0):
    xyz = np.asarray(gt_xyz) + r.normal(0.0, s_xyz, size=(n, 3))
    rpy = np.asarray(gt_rpy) + r.normal(0.0, s_rpy_deg * DEG, size=(n, 3))
    return xyz, rpy


def free_voxel_particles(r, tmap: TsdfMap, n, rp_deg=5.0):
    """Positions uniform over free voxels (stored value > 0) with uniform jitter inside
    the voxel (rejection sampling over the grid); yaw uniform, roll/pitch uniform."""
    nx, ny, nz = tmap.dims
    flat = tmap.values.reshape(-1)
    got = []
    need = n
    while need > 0:
        m = int(need * 1.3) + 64
        lin = r.integers(0, flat.size, size=m)
        lin = lin[flat[lin] > 0][:need]
        got.append(lin)
        need -= lin.size
    lin = np.concatenate(got)
    k, rem = np.divmod(lin, nx * ny)
    j, i = np.divmod(rem, nx)
    ijk = np.column_stack([i, j, k]).astype(np.float64)
    xyz = np.asarray(tmap.origin, np.float64) + (ijk + r.uniform(0.0, 1.0, size=(n, 3))) * float(tmap.voxel)
    rpy = np.column_stack([r.uniform(-rp_deg, rp_deg, size=n) * DEG,
                           r.uniform(-rp_deg, rp_deg, size=n) * DEG,
                           r.uniform(-math.pi, math.pi, size=n)])
    return xyz, rpy


def ground_truth_pose(r, scene: Scene, lo_xy, hi_xy, floor_z, clearance=0.5):
    for _ in range(10000):
        x, y = r.uniform(lo_xy[0], hi_xy[0]), r.uniform(lo_xy[1], hi_xy[1])
        z = floor_z + r.uniform(0.5, 2.0)
        if scene.sdf(np.array([[x, y, z]]))[0] > clearance:
            rpy = np.array([r.uniform(-5, 5) * DEG, r.uniform(-5, 5) * DEG, r.uniform(-math.pi, math.pi)])
            return np.array([x, y, z]), rpy
    raise RuntimeError("no free ground-truth pose found")


# ------------------------------------------------------------------ workloads
@dataclass
class Workload:
    name: str
    tmap: TsdfMap
    points: np.ndarray            # [3, K] float32
    poses: np.ndarray             # [12, N] float32
    sigma: float                  # Eq. (3) sigma, float32 value
    seed: int                     # resampling seed (the draw of update `tick` is fixed by both)
    gt: tuple = field(default=None)
    extra: dict = field(default_factory=dict)

    @property
    def N(self):
        return self.poses.shape[1]

    @property
    def K(self):
        return self.points.shape[1]


def resample_seed(cfg: int, index: int = 0) -> int:
    return (cfg << 32) + index


def config1(n_particles=1000) -> Workload:
    sc = office_scene(rng(1, 0))
    tmap = build_map(sc, (128, 128, 64), 0.1, (0.0, 0.0, 0.0), 0.3, "i16")
    gxyz, grpy = ground_truth_pose(rng(1, 1), sc, (0.5, 0.5), (12.3, 12.3), 1.0)
    R, t = pose_matrix(gxyz, grpy)
    pts = raycast_scan(sc, tmap, R, t, beam_dirs(azimuths=360, **VLP16), 30.0, 0.02, rng(1, 2))
    xyz, rpy = gaussian_particles(rng(1, 3), gxyz, grpy, n_particles)
    return Workload("plain-small: 128x128x64@0.1m int16, VLP-16 16x360, N=1000", tmap, pts,
                    poses_soa(xyz, rpy), f32(tmap.tau / 2), resample_seed(1), (gxyz, grpy))


_WAREHOUSE_CACHE = {}


def warehouse_map(cfg_seed=2, keep_d64=False) -> tuple[Scene, TsdfMap]:
    key = (cfg_seed, keep_d64)
    if key not in _WAREHOUSE_CACHE:
        sc = warehouse_scene(rng(cfg_seed, 0))
        tmap = build_map(sc, (1024, 1024, 128), 0.05, (0.0, 0.0, 0.0), 0.15, "i16", keep_d64=keep_d64)
        _WAREHOUSE_CACHE[key] = (sc, tmap)
    return _WAREHOUSE_CACHE[key]


def config2(n_particles=1_000_000) -> Workload:
    sc, tmap = warehouse_map(2)
    gxyz, grpy = ground_truth_pose(rng(2, 1), sc, (1.0, 1.0), (50.2, 50.2), sc.floor_z)
    R, t = pose_matrix(gxyz, grpy)
    pts = raycast_scan(sc, tmap, R, t, beam_dirs(azimuths=1800, **VLP16), 100.0, 0.03, rng(2, 2))
    xyz, rpy = free_voxel_particles(rng(2, 3), tmap, n_particles)
    return Workload("plain-global: 1024x1024x128@0.05m int16 warehouse, VLP-16 16x1800, N=1e6",
                    tmap, pts, poses_soa(xyz, rpy), f32(tmap.tau / 2), resample_seed(2), (gxyz, grpy))


def config2_converged(n_particles=1_000_000) -> Workload:
    """The global-localisation map and scan with the particles converged: Gaussian
    round the true pose (0.05 m, 1 degree), the steady state of tracking."""
    sc, tmap = warehouse_map(2)
    gxyz, grpy = ground_truth_pose(rng(2, 1), sc, (1.0, 1.0), (50.2, 50.2), sc.floor_z)
    R, t = pose_matrix(gxyz, grpy)
    pts = raycast_scan(sc, tmap, R, t, beam_dirs(azimuths=1800, **VLP16), 100.0, 0.03, rng(2, 2))
    xyz, rpy = gaussian_particles(rng(2, 9), gxyz, grpy, n_particles, s_xyz=0.05, s_rpy_deg=1.0)
    return Workload("plain-converged: 1024x1024x128@0.05m int16 warehouse, VLP-16 16x1800, N=1e6 "
                    "Gaussian round the true pose (0.05 m, 1 deg)",
                    tmap, pts, poses_soa(xyz, rpy), f32(tmap.tau / 2), resample_seed(2), (gxyz, grpy))


def config2_local(n_particles: int, s_xyz: float = 0.5, s_rpy_deg: float = 5.0) -> Workload:
    """The global-localisation map and scan with the particles normally
    distributed round the true pose (s_xyz metres, s_rpy_deg degrees per axis),
    as the clouds the paper times its sensor update on against the particle count."""
    sc, tmap = warehouse_map(2)
    gxyz, grpy = ground_truth_pose(rng(2, 1), sc, (1.0, 1.0), (50.2, 50.2), sc.floor_z)
    R, t = pose_matrix(gxyz, grpy)
    pts = raycast_scan(sc, tmap, R, t, beam_dirs(azimuths=1800, **VLP16), 100.0, 0.03, rng(2, 2))
    xyz, rpy = gaussian_particles(rng(2, 10, n_particles), gxyz, grpy, n_particles, s_xyz=s_xyz, s_rpy_deg=s_rpy_deg)
    return Workload(f"plain-local: 1024x1024x128@0.05m int16 warehouse, VLP-16 16x1800, N={n_particles} "
                    f"Gaussian round the true pose ({s_xyz} m, {s_rpy_deg} deg)",
                    tmap, pts, poses_soa(xyz, rpy), f32(tmap.tau / 2), resample_seed(2), (gxyz, grpy))


def config3(n_particles=262_144, dtype="i16") -> Workload:
    sc, tmap = warehouse_map(2, keep_d64=True)
    if dtype != "i16":
        tmap = tmap.with_dtype(dtype)
    gxyz, grpy = ground_truth_pose(rng(3, 1), sc, (1.0, 1.0), (50.2, 50.2), sc.floor_z)
    R, t = pose_matrix(gxyz, grpy)
    pts = raycast_scan(sc, tmap, R, t, beam_dirs(azimuths=1024, **OS0_64), 50.0, 0.02, rng(3, 2))
    half = n_particles // 2
    xg, rg = free_voxel_particles(rng(3, 3, 0), tmap if dtype == "i16" else warehouse_map(2, True)[1], half)
    xl, rl = gaussian_particles(rng(3, 3, 1), gxyz, grpy, n_particles - half)
    poses = poses_soa(np.vstack([xg, xl]), np.vstack([rg, rl]))
    return Workload(f"precision: warehouse {dtype}, OS0-64 64x1024, N=262144", tmap, pts, poses,
                    f32(tmap.tau / 2), resample_seed(3), (gxyz, grpy))


def subset_indices(cfg: int, n_total: int, n_sub: int = 4096) -> np.ndarray:
    """Seeded, sorted particle subset the oracle checks at full size."""
    return np.sort(rng(cfg, 4).choice(n_total, size=min(n_sub, n_total), replace=False))


@dataclass
class FilterSpec:
    points: np.ndarray            # [3, K] float32
    poses: np.ndarray             # [12, N] float32
    sigma: float
    seed: int
    gt: tuple

    @property
    def N(self):
        return self.poses.shape[1]

    @property
    def K(self):
        return self.points.shape[1]


def config4(n_filters: int = 64, n_scale: float = 1.0):
    """64 filters on the warehouse map: particle counts log-uniform in
    [2048, 524288] (scaled by n_scale), even filters VLP-16 16x1800 scans, odd
    ones OS0-64 64x1024, each from its own ground-truth pose; Gaussian particles
    below 65,536, uniform over free space above."""
    sc, tmap = warehouse_map(2)
    Ns = np.round(np.exp(rng(4, 3).uniform(math.log(2048), math.log(524288), size=n_filters)) * n_scale)
    Ns = np.maximum(Ns.astype(int), 1)
    out = []
    for f in range(n_filters):
        gxyz, grpy = ground_truth_pose(rng(4, 1, f), sc, (1.0, 1.0), (50.2, 50.2), sc.floor_z)
        R, t = pose_matrix(gxyz, grpy)
        if f % 2 == 0:
            pts = raycast_scan(sc, tmap, R, t, beam_dirs(azimuths=1800, **VLP16), 100.0, 0.03, rng(4, 2, f))
        else:
            pts = raycast_scan(sc, tmap, R, t, beam_dirs(azimuths=1024, **OS0_64), 50.0, 0.02, rng(4, 2, f))
        N = int(Ns[f])
        if N < 65536:
            xyz, rpy = gaussian_particles(rng(4, 5, f), gxyz, grpy, N)
        else:
            xyz, rpy = free_voxel_particles(rng(4, 5, f), tmap, N)
        out.append(FilterSpec(pts, poses_soa(xyz, rpy), f32(tmap.tau / 2), resample_seed(4, f), (gxyz, grpy)))
    return tmap, out
