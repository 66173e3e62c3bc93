"""Small shared helpers for the tests (no method arithmetic here)."""

from __future__ import annotations

import numpy as np

from workloads.tsdf import TsdfMap, f32


def make_map(values: np.ndarray, voxel: float, origin=(0.0, 0.0, 0.0), tau: float = 0.3,
             dtype: str = "i16") -> TsdfMap:
    nz, ny, nx = values.shape
    return TsdfMap(nx, ny, nz, f32(voxel), tuple(f32(x) for x in origin), f32(tau), dtype, values)


def identity_poses(n: int, t=(0.0, 0.0, 0.0)) -> np.ndarray:
    p = np.zeros((12, n), np.float32)
    p[0] = p[4] = p[8] = 1.0
    p[9:] = np.asarray(t, np.float32)[:, None]
    return p


def random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """[n, 3, 3] float64 rotations from normalised Gaussian quaternions."""
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((n, 3, 3))
    R[:, 0] = np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], 1)
    R[:, 1] = np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], 1)
    R[:, 2] = np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], 1)
    return R


def poses_from(R: np.ndarray, t: np.ndarray) -> np.ndarray:
    p = np.empty((12, R.shape[0]), np.float32)
    p[:9] = R.reshape(-1, 9).T
    p[9:] = np.asarray(t).T
    return p
