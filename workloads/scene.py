"""Analytic scenes: exact signed distance functions and exact ray casts.

A scene is a union of solids: a floor half-space, axis-aligned boxes, vertical
capped cylinders and spheres.  Its signed distance is positive in free space and
negative inside a solid, the sign convention of the paper's TSDF figure (§III).
The union's distance is the minimum over the primitives, which keeps it
1-Lipschitz; the pins that bound voxelisation error rely on that.

Everything here is float64 and vectorised over query points / rays.  This module
generates inputs only; it holds none of the sensor model's arithmetic.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Scene:
    floor_z: float | None = None                 # solid below z = floor_z
    boxes: np.ndarray = field(default_factory=lambda: np.zeros((0, 6)))      # [xmin ymin zmin xmax ymax zmax]
    cylinders: np.ndarray = field(default_factory=lambda: np.zeros((0, 5)))  # [cx cy r z0 z1]
    spheres: np.ndarray = field(default_factory=lambda: np.zeros((0, 4)))    # [cx cy cz r]

    # ------------------------------------------------------------------ SDF
    def sdf(self, p: np.ndarray) -> np.ndarray:
        """Signed distance at points p[..., 3] (float64)."""
        p = np.asarray(p, dtype=np.float64)
        d = np.full(p.shape[:-1], np.inf)
        if self.floor_z is not None:
            d = np.minimum(d, p[..., 2] - self.floor_z)
        for b in self.boxes:
            d = np.minimum(d, box_sdf(p, b))
        for c in self.cylinders:
            d = np.minimum(d, cylinder_sdf(p, c))
        for s in self.spheres:
            d = np.minimum(d, sphere_sdf(p, s))
        return d

    def primitives(self):
        """Yield (kind, params, aabb_min, aabb_max); the floor has an infinite box."""
        if self.floor_z is not None:
            yield "floor", self.floor_z, None, None
        for b in self.boxes:
            yield "box", b, b[:3], b[3:]
        for c in self.cylinders:
            yield "cyl", c, np.array([c[0] - c[2], c[1] - c[2], c[3]]), \
                np.array([c[0] + c[2], c[1] + c[2], c[4]])
        for s in self.spheres:
            yield "sph", s, s[:3] - s[3], s[:3] + s[3]

    # ------------------------------------------------------------- raycast
    def raycast(self, origin: np.ndarray, dirs: np.ndarray) -> np.ndarray:
        """Distance along unit rays dirs[R, 3] from origin[3] to the first surface.

        Returns +inf where a ray hits nothing.  The origin must lie in free space.
        Exact (closed-form) intersections, float64.
        """
        o = np.asarray(origin, np.float64)
        d = np.asarray(dirs, np.float64)
        best = np.full(d.shape[0], np.inf)
        if self.floor_z is not None:
            with np.errstate(divide="ignore", invalid="ignore"):
                t = (self.floor_z - o[2]) / d[:, 2]
            t = np.where((d[:, 2] < 0) & (t >= 0), t, np.inf)
            best = np.minimum(best, t)
        if len(self.boxes):
            best = np.minimum(best, _ray_boxes(o, d, self.boxes))
        if len(self.cylinders):
            best = np.minimum(best, _ray_cylinders(o, d, self.cylinders))
        if len(self.spheres):
            best = np.minimum(best, _ray_spheres(o, d, self.spheres))
        return best


def box_sdf(p: np.ndarray, b: np.ndarray) -> np.ndarray:
    lo, hi = b[:3], b[3:]
    q = np.maximum(lo - p, p - hi)                       # per-axis outside distance
    outside = np.sqrt(np.sum(np.maximum(q, 0.0) ** 2, axis=-1))
    inside = np.minimum(np.max(q, axis=-1), 0.0)
    return outside + inside


def cylinder_sdf(p: np.ndarray, c: np.ndarray) -> np.ndarray:
    cx, cy, r, z0, z1 = c
    dr = np.hypot(p[..., 0] - cx, p[..., 1] - cy) - r
    dz = np.maximum(z0 - p[..., 2], p[..., 2] - z1)
    outside = np.hypot(np.maximum(dr, 0.0), np.maximum(dz, 0.0))
    inside = np.minimum(np.maximum(dr, dz), 0.0)
    return outside + inside


def sphere_sdf(p: np.ndarray, s: np.ndarray) -> np.ndarray:
    return np.sqrt(np.sum((p - s[:3]) ** 2, axis=-1)) - s[3]


def _ray_boxes(o, d, boxes, chunk=8192):
    """Slab test of every ray against every box (float64, torch CPU threads)."""
    import torch
    O = torch.as_tensor(o, dtype=torch.float64)
    B = torch.as_tensor(boxes, dtype=torch.float64)
    lo, hi = B[:, :3] - O, B[:, 3:] - O                     # [nb, 3]
    out = np.empty(d.shape[0])
    for s in range(0, d.shape[0], chunk):
        D = torch.as_tensor(d[s:s + chunk], dtype=torch.float64)
        inv = 1.0 / D                                          # +-inf on axis-parallel rays
        t1 = lo[None] * inv[:, None]                           # [r, nb, 3]
        t2 = hi[None] * inv[:, None]
        bad = torch.isnan(t1) | torch.isnan(t2)                # 0*inf: axis-parallel ray outside a slab
        tmin = torch.where(bad, torch.inf, torch.minimum(t1, t2)).amax(dim=2)
        tmax = torch.where(bad, -torch.inf, torch.maximum(t1, t2)).amin(dim=2)
        hit = (tmin <= tmax) & (tmin >= 0)
        out[s:s + chunk] = torch.where(hit, tmin, torch.inf).amin(dim=1).numpy()
    return out


def _ray_cylinders(o, d, cyl, chunk=16384):
    """Side and cap intersections of every ray with every vertical cylinder."""
    import torch
    C = torch.as_tensor(cyl, dtype=torch.float64)
    cx, cy, r, z0, z1 = (C[:, i][None, :] for i in range(5))
    ox, oy, oz = float(o[0]), float(o[1]), float(o[2])
    out = np.empty(d.shape[0])
    for s in range(0, d.shape[0], chunk):
        D = torch.as_tensor(d[s:s + chunk], dtype=torch.float64)
        dx, dy, dz = D[:, 0:1], D[:, 1:2], D[:, 2:3]
        px, py = ox - cx, oy - cy
        a = dx * dx + dy * dy
        b = 2.0 * (px * dx + py * dy)
        c = px * px + py * py - r * r
        disc = b * b - 4 * a * c
        t = (-b - torch.sqrt(disc)) / (2 * a)
        z = oz + t * dz
        ok = (disc >= 0) & (a > 0) & (t >= 0) & (z >= z0) & (z <= z1)
        best = torch.where(ok, t, torch.inf).amin(dim=1)
        # caps: a ray leaving the side range can enter through the top or bottom disc
        for zc in (z0, z1):
            tc = (zc - oz) / dz
            qx, qy = px + tc * dx, py + tc * dy
            okc = (tc >= 0) & (qx * qx + qy * qy <= r * r)
            best = torch.minimum(best, torch.where(okc, tc, torch.inf).amin(dim=1))
        out[s:s + chunk] = best.numpy()
    return out


def _ray_spheres(o, d, sph):
    oc = o[None, :] - sph[:, :3]                          # [S, 3]
    b = d @ oc.T                                          # [R, S]
    c = np.sum(oc * oc, axis=1)[None, :] - sph[:, 3][None, :] ** 2
    disc = b * b - c
    t = -b - np.sqrt(np.maximum(disc, 0.0))
    ok = (disc >= 0) & (t >= 0)
    return np.where(ok, t, np.inf).min(axis=1)


def euler_zyx_to_matrix(roll, pitch, yaw) -> np.ndarray:
    """R = Rz(yaw) Ry(pitch) Rx(roll) in float64; arrays broadcast, result [..., 3, 3].

    This is the reading of the paper's (phi, psi, theta) of Eq. (2): roll about x,
    pitch about y, yaw about z, composed as z-y-x.
    """
    roll, pitch, yaw = (np.asarray(v, np.float64) for v in (roll, pitch, yaw))
    cr, sr = np.cos(roll), np.sin(roll)
    cp, sp = np.cos(pitch), np.sin(pitch)
    cy, sy = np.cos(yaw), np.sin(yaw)
    R = np.empty(np.broadcast(roll, pitch, yaw).shape + (3, 3))
    R[..., 0, 0] = cy * cp
    R[..., 0, 1] = cy * sp * sr - sy * cr
    R[..., 0, 2] = cy * sp * cr + sy * sr
    R[..., 1, 0] = sy * cp
    R[..., 1, 1] = sy * sp * sr + cy * cr
    R[..., 1, 2] = sy * sp * cr - cy * sr
    R[..., 2, 0] = -sp
    R[..., 2, 1] = cp * sr
    R[..., 2, 2] = cp * cr
    return R
