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


def score_const(dtype: str, tau: float, sigma: float) -> float:
    """The library's c = s^2 / (2 sigma^2) (float64, rounded to float32), with
    s = tau / Q metres per stored unit (1 for float32 maps), as its header
    states: tests that need the exact float32 constant recompute it here."""
    Q = {"i16": 32767, "i8": 127, "f32": 1}[dtype]
    s = 1.0 if dtype == "f32" else float(np.float32(tau)) / Q
    sg = float(np.float32(sigma))
    return float(np.float32((s * s) / (2.0 * sg * sg)))


_M64 = 2 ** 64 - 1


def _unxorshift(y: int, s: int) -> int:
    x = y
    for _ in range(64 // s + 1):
        x = y ^ (x >> s)
    return x & _M64


def splitmix64_state_for(u: int) -> int:
    """The state whose SplitMix64 output is u (the output map is a bijection)."""
    z = _unxorshift(u & _M64, 31)
    z = (z * pow(0x94D049BB133111EB, -1, 2 ** 64)) & _M64
    z = _unxorshift(z, 27)
    z = (z * pow(0xBF58476D1CE4E5B9, -1, 2 ** 64)) & _M64
    z = _unxorshift(z, 30)
    return (z - 0x9E3779B97F4A7C15) & _M64


def seed_for_draw(oracle, u: int, tick: int = 0) -> int:
    """A filter seed whose resampling draw at `tick` is u (so that tests can pick
    an edge-case offset); checked against the oracle's draw."""
    seed = splitmix64_state_for(u) ^ oracle.splitmix64(tick)
    assert oracle.resample_draw(seed, tick) == u & _M64
    return seed
