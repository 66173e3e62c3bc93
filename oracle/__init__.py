"""CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path never routes through it.

Thin ctypes wrapper over ``mcl_oracle.c`` and ``mcl_oracle_motion.c`` (the
definitions and readings are in their header comments) plus their build step;
``estimate.py`` holds the pose-estimate oracle.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "mcl_oracle.c"), os.path.join(HERE, "mcl_oracle_motion.c")]
LIB = os.path.join(HERE, "libmcl_oracle.so")

DTYPE_CODE = {"i16": 0, "i8": 1, "f32": 2, "f64": 3}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O2, no contraction, no fast-math."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-pthread", "-Wall", "-o", tmp, *SRCS, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.oracle_voxel_indices.argtypes = [P, C.c_float, P, P, C.c_int32, P, C.c_int32, P]
        L.oracle_sensor_update.argtypes = [P, C.c_float, P, C.c_float, C.c_int32, P, P, C.c_int32,
                                           P, C.c_int32, C.c_float, P, P, C.c_int32]
        L.oracle_sensor_update_trilinear.argtypes = [P, C.c_float, P, C.c_float, C.c_int32, P, P, C.c_int32,
                                                     P, C.c_int32, C.c_float, P, P, P, C.c_int32]
        L.oracle_sensor_update_sum.argtypes = [P, C.c_float, P, C.c_float, C.c_int32, P, P, C.c_int32,
                                               P, C.c_int32, C.c_float, P, P, C.c_int32]
        L.oracle_normalize.argtypes = [P, C.c_int32, P, P, P]
        L.oracle_sensor_update_bricks.argtypes = [P, C.c_float, P, C.c_float, C.c_int32, C.c_int64, P, P, P, C.c_int32,
                                                  P, C.c_int32, C.c_float, P, P, C.c_int32]
        L.oracle_sensor_update_bricks.restype = C.c_int
        L.oracle_philox4x32.argtypes = [P, P, P]
        L.oracle_philox4x32.restype = None
        L.oracle_motion_update.argtypes = [P, P, C.c_int32, P, C.c_float, C.c_float, C.c_uint64, C.c_uint64, P]
        L.oracle_motion_update.restype = C.c_int
        L.oracle_init_uniform.argtypes = [P, C.c_float, P, C.c_int32, P, C.c_int32, C.c_float, C.c_uint64, P, P]
        L.oracle_init_uniform.restype = C.c_int
        L.oracle_resample.argtypes = [P, C.c_int32, C.c_uint64, P]
        L.oracle_splitmix64.argtypes = [C.c_uint64]
        L.oracle_splitmix64.restype = C.c_uint64
        L.oracle_resample_draw.argtypes = [C.c_uint64, C.c_uint64]
        L.oracle_resample_draw.restype = C.c_uint64
        for f in (L.oracle_voxel_indices, L.oracle_sensor_update, L.oracle_sensor_update_trilinear,
                  L.oracle_sensor_update_sum, L.oracle_normalize, L.oracle_resample):
            f.restype = C.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _map_args(tmap):
    dims = np.array([tmap.nx, tmap.ny, tmap.nz], np.int32)
    origin = np.array(tmap.origin, np.float32)
    vals = np.ascontiguousarray(tmap.values)
    want = {"i16": np.int16, "i8": np.int8, "f32": np.float32, "f64": np.float64}[tmap.dtype]
    assert vals.dtype == want, (vals.dtype, tmap.dtype)
    return dims, origin, vals


def voxel_indices(tmap, points: np.ndarray, poses: np.ndarray) -> np.ndarray:
    """int64 [N, K]: linear voxel index i + nx (j + ny k) or -1 outside the map."""
    dims, origin, _ = _map_args(tmap)
    pts = np.ascontiguousarray(points, np.float32)
    ps = np.ascontiguousarray(poses, np.float32)
    K, N = pts.shape[1], ps.shape[1]
    out = np.empty((N, K), np.int64)
    rc = lib().oracle_voxel_indices(_p(dims), tmap.voxel, _p(origin), _p(pts), K, _p(ps), N, _p(out))
    assert rc == 0
    return out


def sensor_update(tmap, points: np.ndarray, poses: np.ndarray, sigma: float, nthreads: int = 1,
                  return_sum: bool = False):
    """float64 log-weights l_n (and optionally the sums of squared stored values)."""
    dims, origin, vals = _map_args(tmap)
    pts = np.ascontiguousarray(points, np.float32)
    ps = np.ascontiguousarray(poses, np.float32)
    K, N = pts.shape[1], ps.shape[1]
    logw = np.empty(N, np.float64)
    ssum = np.empty(N, np.float64)
    rc = lib().oracle_sensor_update(_p(dims), tmap.voxel, _p(origin), tmap.tau, DTYPE_CODE[tmap.dtype],
                                    _p(vals), _p(pts), K, _p(ps), N, sigma, _p(logw), _p(ssum), nthreads)
    assert rc == 0
    return (logw, ssum) if return_sum else logw


def sensor_update_sum(tmap, points: np.ndarray, poses: np.ndarray, sigma: float, nthreads: int = 1,
                      return_sum: bool = False):
    """float64 log-weights under the sum reading, l_n = log sum_k exp(-c q_k^2)
    (and optionally the sums themselves)."""
    dims, origin, vals = _map_args(tmap)
    pts = np.ascontiguousarray(points, np.float32)
    ps = np.ascontiguousarray(poses, np.float32)
    K, N = pts.shape[1], ps.shape[1]
    logw = np.empty(N, np.float64)
    ssum = np.empty(N, np.float64)
    rc = lib().oracle_sensor_update_sum(_p(dims), tmap.voxel, _p(origin), tmap.tau, DTYPE_CODE[tmap.dtype],
                                        _p(vals), _p(pts), K, _p(ps), N, sigma, _p(logw), _p(ssum), nthreads)
    assert rc == 0
    return (logw, ssum) if return_sum else logw


def sensor_update_bricks(dims, voxel: float, origin, tau: float, dtype: str, coords: np.ndarray, values: np.ndarray,
                         points: np.ndarray, poses: np.ndarray, sigma: float, nthreads: int = 1):
    """float64 log-weights on a sparse map given as bricks (unlisted bricks read +Q)."""
    d = np.asarray(dims, np.int32)
    o = np.asarray(origin, np.float32)
    co = np.ascontiguousarray(coords, np.int32).reshape(-1, 3)
    va = np.ascontiguousarray(values, {"i16": np.int16, "i8": np.int8, "f32": np.float32}[dtype]).reshape(-1, 64)
    pts = np.ascontiguousarray(points, np.float32)
    ps = np.ascontiguousarray(poses, np.float32)
    K, N = pts.shape[1], ps.shape[1]
    logw = np.empty(N, np.float64)
    rc = lib().oracle_sensor_update_bricks(_p(d), voxel, _p(o), tau, DTYPE_CODE[dtype], co.shape[0], _p(co), _p(va),
                                           _p(pts), K, _p(ps), N, sigma, _p(logw), None, nthreads)
    assert rc == 0
    return logw


def sensor_update_trilinear(tmap, points: np.ndarray, poses: np.ndarray, sigma: float, nthreads: int = 1,
                            return_sums: bool = False):
    """float64 log-weights with the trilinear lookup (and optionally sum m^2, sum |m|)."""
    dims, origin, vals = _map_args(tmap)
    pts = np.ascontiguousarray(points, np.float32)
    ps = np.ascontiguousarray(poses, np.float32)
    K, N = pts.shape[1], ps.shape[1]
    logw = np.empty(N, np.float64)
    ssum = np.empty(N, np.float64)
    sabs = np.empty(N, np.float64)
    rc = lib().oracle_sensor_update_trilinear(_p(dims), tmap.voxel, _p(origin), tmap.tau, DTYPE_CODE[tmap.dtype],
                                              _p(vals), _p(pts), K, _p(ps), N, sigma, _p(logw), _p(ssum),
                                              _p(sabs), nthreads)
    assert rc == 0
    return (logw, ssum, sabs) if return_sums else logw


def philox4x32(counter, key) -> np.ndarray:
    """Philox4x32-10 of a 4-word counter and a 2-word key: 4 uint32 words."""
    c = np.ascontiguousarray(counter, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.empty(4, np.uint32)
    lib().oracle_philox4x32(_p(c), _p(k), _p(out))
    return out


def motion_update(poses: np.ndarray, delta: np.ndarray, sigma_t: float, sigma_r: float, seed: int, step: int,
                  return_normals: bool = False):
    """float64 [12, N] poses after the motion update (and the [6, N] normals drawn)."""
    ps = np.ascontiguousarray(poses, np.float32)
    N = ps.shape[1]
    d = np.ascontiguousarray(delta, np.float32).reshape(12)
    out = np.empty((12, N), np.float64)
    nrm = np.empty((6, N), np.float64)
    rc = lib().oracle_motion_update(_p(ps), _p(out), N, _p(d), sigma_t, sigma_r, C.c_uint64(seed & (2**64 - 1)),
                                    C.c_uint64(step & (2**64 - 1)), _p(nrm))
    assert rc == 0
    return (out, nrm) if return_normals else out


def init_uniform(tmap, N: int, max_tilt: float, seed: int):
    """(float64 [12, N] poses, int64 [N] chosen voxels) uniform over free voxels."""
    dims, origin, vals = _map_args(tmap)
    out = np.empty((12, N), np.float64)
    vox = np.empty(N, np.int64)
    rc = lib().oracle_init_uniform(_p(dims), tmap.voxel, _p(origin), DTYPE_CODE[tmap.dtype], _p(vals), N, max_tilt,
                                   C.c_uint64(seed & (2**64 - 1)), _p(out), _p(vox))
    if rc == -3:
        raise ValueError("the map has no free voxel")
    assert rc == 0
    return out, vox


def normalize(logw: np.ndarray):
    """(w float64 [N], wq uint64 [N], log_z float)."""
    lw = np.ascontiguousarray(logw, np.float64)
    N = lw.shape[0]
    w = np.empty(N, np.float64)
    wq = np.empty(N, np.uint64)
    lz = np.empty(1, np.float64)
    rc = lib().oracle_normalize(_p(lw), N, _p(w), _p(wq), _p(lz))
    assert rc == 0
    return w, wq, float(lz[0])


def splitmix64(x: int) -> int:
    """SplitMix64 output from state x."""
    return int(lib().oracle_splitmix64(C.c_uint64(int(x) & (2**64 - 1))))


def resample_draw(seed: int, tick: int) -> int:
    """The uniform 64-bit draw of update `tick` of a filter seeded with `seed`."""
    return int(lib().oracle_resample_draw(C.c_uint64(int(seed) & (2**64 - 1)), C.c_uint64(int(tick) & (2**64 - 1))))


def resample_seeded(wq: np.ndarray, seed: int, tick: int) -> np.ndarray:
    """Ancestor indices of update `tick` of a filter seeded with `seed`."""
    return resample(wq, resample_draw(seed, tick))


def resample(wq: np.ndarray, u: int) -> np.ndarray:
    """int32 [N] ancestor indices (non-decreasing) for the draw u."""
    W = np.ascontiguousarray(wq, np.uint64)
    N = W.shape[0]
    idx = np.empty(N, np.int32)
    rc = lib().oracle_resample(_p(W), N, C.c_uint64(int(u) & (2**64 - 1)), _p(idx))
    assert rc == 0
    return idx
