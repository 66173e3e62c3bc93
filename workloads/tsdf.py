"""Dense TSDF maps voxelised from an analytic scene.

Voxel (i, j, k) covers [o + i v, o + (i+1) v) per axis and stores the scene's
signed distance at its centre o + (i + 1/2, j + 1/2, k + 1/2) v, clamped to the
truncation band [-tau, +tau] (the paper clamps every cell beyond the truncation
distance to the truncation value, §III).  Arrays are C-ordered (nz, ny, nx), so
x is the fastest-varying index: linear index i + nx (j + ny k).

Storage types: int16 and int8 fixed point store q = rint(d / tau * Q) with
Q = 32767 or 127 (round half to even, float64); float32 stores d in metres.
The library converts this dense x-fastest array to its own device layout.
"""

from __future__ import annotations

import os
from dataclasses import dataclass

import numpy as np

from .scene import Scene, box_sdf, cylinder_sdf, sphere_sdf

QSCALE = {"i16": 32767, "i8": 127, "f32": 1, "f64": 1}
NP_DTYPE = {"i16": np.int16, "i8": np.int8, "f32": np.float32, "f64": np.float64}
DTYPE_CODE = {"i16": 0, "i8": 1, "f32": 2}


@dataclass
class TsdfMap:
    nx: int
    ny: int
    nz: int
    voxel: float          # float32 value (held as a Python float)
    origin: tuple         # three float32 values
    tau: float            # float32 value
    dtype: str            # "i16" | "i8" | "f32"
    values: np.ndarray    # (nz, ny, nx) of NP_DTYPE[dtype]
    d64: np.ndarray | None = None   # (nz, ny, nx) float64 clamped distances, if kept

    @property
    def Q(self) -> int:
        return QSCALE[self.dtype]

    @property
    def scale(self) -> float:
        """Metres per stored unit, s = tau / Q (1 for float maps), float64."""
        return 1.0 if self.dtype in ("f32", "f64") else float(self.tau) / self.Q

    @property
    def dims(self):
        return (self.nx, self.ny, self.nz)

    def with_dtype(self, dtype: str) -> "TsdfMap":
        if self.d64 is None:
            raise ValueError("re-quantising needs the float64 distances (keep_d64=True)")
        vals = self.d64 if dtype == "f64" else quantise(self.d64, self.tau, dtype)
        return TsdfMap(self.nx, self.ny, self.nz, self.voxel, self.origin, self.tau, dtype, vals, self.d64)


def f32(x) -> float:
    return float(np.float32(x))


def voxelise(scene: Scene, dims, voxel: float, origin, tau: float, dtype: str = "f64",
             keep_d64: bool = False, slab: int = 8):
    """Voxelise a scene: clamped signed distance at every voxel centre.

    Returns (values, d64): values are the stored values of ``dtype`` ("f64" keeps the
    float64 distances themselves), d64 the float64 distances when keep_d64 is set.
    Works through z-slabs with one reused float64 buffer; each primitive is evaluated
    only inside its bounding box grown by tau plus a voxel, beyond which its distance
    exceeds tau and the clamp makes it irrelevant.
    """
    nx, ny, nz = dims
    v = float(voxel)
    o = np.asarray(origin, np.float64)
    tau = float(tau)
    out = np.empty((nz, ny, nx), dtype=np.float64 if dtype == "f64" else NP_DTYPE[dtype])
    d64 = out if dtype == "f64" else (np.empty((nz, ny, nx)) if keep_d64 else None)
    centres = [o[a] + (np.arange(n, dtype=np.float64) + 0.5) * v for a, n in enumerate((nx, ny, nz))]
    prims = []
    for kind, prm, lo, hi in scene.primitives():
        if kind == "floor":
            prims.append((kind, prm, None))
            continue
        sl = []
        for a, n in enumerate((nx, ny, nz)):
            i0 = int(np.floor((lo[a] - tau - v - o[a]) / v - 0.5))
            i1 = int(np.ceil((hi[a] + tau + v - o[a]) / v - 0.5)) + 1
            sl.append((max(0, i0), min(n, i1)))
        if all(b > a for a, b in sl):
            prims.append((kind, prm, sl))
    def do_slab(zs):
        ze = min(nz, zs + slab)
        d = np.empty((ze - zs, ny, nx), dtype=np.float64)
        d.fill(tau)
        for kind, prm, sl in prims:
            if kind == "floor":
                dz = np.clip(centres[2][zs:ze] - prm, -tau, tau)
                np.minimum(d, dz[:, None, None], out=d)
                continue
            (x0, x1), (y0, y1), (z0, z1) = sl
            z0, z1 = max(z0, zs), min(z1, ze)
            if z1 <= z0:
                continue
            P = np.empty((z1 - z0, y1 - y0, x1 - x0, 3))
            P[..., 0] = centres[0][None, None, x0:x1]
            P[..., 1] = centres[1][None, y0:y1, None]
            P[..., 2] = centres[2][z0:z1, None, None]
            if kind == "box":
                dd = box_sdf(P, prm)
            elif kind == "cyl":
                dd = cylinder_sdf(P, prm)
            else:
                dd = sphere_sdf(P, prm)
            np.clip(dd, -tau, tau, out=dd)
            blk = d[z0 - zs:z1 - zs, y0:y1, x0:x1]
            np.minimum(blk, dd, out=blk)
        if d64 is not None and d64 is not out:
            d64[zs:ze] = d
        if dtype == "f64":
            out[zs:ze] = d
        else:
            _quantise_inplace(d, tau, dtype)
            out[zs:ze] = d

    # slabs are independent (disjoint z ranges of the outputs); numpy releases
    # the interpreter lock in its array loops, so threads share the work
    from concurrent.futures import ThreadPoolExecutor
    workers = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else 4))
    with ThreadPoolExecutor(workers) as ex:
        list(ex.map(do_slab, range(0, nz, slab)))
    return out, d64


def _quantise_inplace(d: np.ndarray, tau: float, dtype: str) -> None:
    if dtype == "f32":
        return
    d /= float(tau)
    d *= QSCALE[dtype]
    np.rint(d, out=d)


def quantise(d64: np.ndarray, tau: float, dtype: str, slab: int = 8) -> np.ndarray:
    """Stored values from clamped float64 distances (see module docstring)."""
    out = np.empty(d64.shape, NP_DTYPE[dtype])
    buf = np.empty((min(slab, d64.shape[0]),) + d64.shape[1:])
    for zs in range(0, d64.shape[0], slab):
        b = buf[: min(slab, d64.shape[0] - zs)]
        b[...] = d64[zs:zs + slab]
        _quantise_inplace(b, tau, dtype)
        out[zs:zs + slab] = b
    return out


def build_map(scene: Scene, dims, voxel, origin, tau, dtype="i16", keep_d64=False) -> TsdfMap:
    v, t = f32(voxel), f32(tau)
    o = tuple(f32(x) for x in origin)
    vals, d64 = voxelise(scene, dims, v, o, t, dtype, keep_d64)
    return TsdfMap(dims[0], dims[1], dims[2], v, o, t, dtype, vals, d64)


def to_bricks(tmap: "TsdfMap", band_only: bool = True):
    """A dense map as a sparse coarse/fine map: (coords int32 [M, 3] (bx, by, bz),
    values [M, 64] of the storage type, in-brick index x + 4 y + 16 z).  With
    band_only, only bricks with a value strictly inside the truncation band are
    listed (the others are all +-Q and read +Q when unlisted, the same q^2);
    voxels beyond the map edge are filled with Q."""
    Qv = {"i16": 32767, "i8": 127}.get(tmap.dtype, None)
    q = np.asarray(Qv if Qv is not None else np.float32(tmap.tau), tmap.values.dtype)
    nz, ny, nx = tmap.values.shape
    pz, py, px = -(-nz // 4) * 4, -(-ny // 4) * 4, -(-nx // 4) * 4
    padded = np.full((pz, py, px), q, tmap.values.dtype)
    padded[:nz, :ny, :nx] = tmap.values
    # [bz, z, by, y, bx, x] -> [by, bx, bz, z, y, x]
    b = padded.reshape(pz // 4, 4, py // 4, 4, px // 4, 4).transpose(2, 4, 0, 1, 3, 5)
    flat = b.reshape(py // 4, px // 4, pz // 4, 64)
    if band_only:
        keep = (np.abs(flat.astype(np.float64)) < float(q)).any(axis=3)
    else:
        keep = np.ones(flat.shape[:3], bool)
    by, bx, bz = np.nonzero(keep)
    coords = np.stack([bx, by, bz], 1).astype(np.int32)
    return coords, np.ascontiguousarray(flat[keep])

