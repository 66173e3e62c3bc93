"""Python binding of libmcl.so: argument marshalling only.

Every step of the sensor update, normalisation, pose estimate, resampling,
motion update and initialisation runs in the HIP kernels behind the C ABI
(include/mcl.h).  torch supplies device memory and streams.  If the built
library is missing this module raises at import: there is no fallback.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np
# torch before the library: the library then binds to the HIP runtime torch has
# loaded, so one runtime serves both (loading the library first would make torch
# share a runtime it was not built against)
import torch  # noqa: F401

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MCL_LIBRARY") or os.path.join(PKG, "libmcl.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2310_04172_amd.build`")

_lib = C.CDLL(LIB_PATH)
_P = C.c_void_p
_I = C.c_int32

MCL_OK, MCL_EINVAL, MCL_ENOMEM, MCL_EDEVICE, MCL_ERANGE, MCL_EBUSY = 0, -1, -2, -3, -4, -5
MAX_JOBS = 4096
TICK_GRAPH, TICK_NOWAIT = 1, 2
LOOKUP_NEAREST, LOOKUP_TRILINEAR = 0, 1
SCORE_PRODUCT, SCORE_SUM = 0, 1
MAX_PARTICLES = 1 << 21
MAX_POINTS = 1 << 20
NOALLOC_SCRATCH_BYTES = 64 << 20
WQ_SHIFT = 42
DTYPE_CODE = {"i16": 0, "i8": 1, "f32": 2}


class MapDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("voxel", C.c_float),
                ("origin", C.c_float * 3), ("tau", C.c_float), ("dtype", C.c_int32)]


class FilterJob(C.Structure):
    _fields_ = [("map", _P), ("points", _P), ("K", C.c_int32), ("poses", _P), ("N", C.c_int32),
                ("sigma", C.c_float), ("logw", _P), ("w", _P), ("wq", _P), ("log_z", _P), ("seed", C.c_uint64),
                ("tick", C.c_uint64),
                ("idx", _P), ("poses_out", _P), ("est_mean", _P), ("est_idx", _P), ("est_pose", _P),
                ("lookup", C.c_int32), ("score", C.c_int32)]


class LaunchConfig(C.Structure):
    _fields_ = [("waves_per_block", C.c_int32), ("blocks_per_cu", C.c_int32), ("coarse", C.c_int32),
                ("runs", C.c_int32), ("lds_threshold", C.c_int32)]


_lib.mcl_map_upload.argtypes = [C.POINTER(MapDesc), _P, _P, C.POINTER(_P)]
_lib.mcl_map_free.argtypes = [_P]
_lib.mcl_map_upload_bricks.argtypes = [C.POINTER(MapDesc), C.c_int64, _P, _P, _P, C.POINTER(_P)]
_lib.mcl_sensor_update.argtypes = [_P, _P, _I, _P, _I, C.c_float, _P, _P]
_lib.mcl_sensor_update_trilinear.argtypes = [_P, _P, _I, _P, _I, C.c_float, _P, _P]
_lib.mcl_sensor_update_noalloc.argtypes = [_P, _P, _I, _P, _I, C.c_float, _P, _P]
_lib.mcl_sensor_update_sum.argtypes = [_P, _P, _I, _P, _I, C.c_float, _P, _P]
_lib.mcl_normalize.argtypes = [_P, _I, _P, _P, _P, _P]
_lib.mcl_resample.argtypes = [_P, _I, C.c_uint64, C.c_uint64, _P, _P, _P, _P]
_lib.mcl_debug_voxel_indices.argtypes = [_P, _P, _I, _P, _I, _P, _P]
_lib.mcl_pose_estimate.argtypes = [_P, _P, _I, _P, _P, _P, _P]
_lib.mcl_motion_update.argtypes = [_P, _P, _I, _P, C.c_float, C.c_float, C.c_uint64, C.c_uint64, _P]
_lib.mcl_init_uniform.argtypes = [_P, _P, _I, C.c_float, C.c_uint64, _P]
_lib.mcl_init_gaussian.argtypes = [_P, _I, _P, C.c_float, C.c_float, C.c_uint64, C.c_uint64, _P]
_lib.mcl_debug_philox.argtypes = [_P, _P]
_lib.mcl_tick.argtypes = [C.POINTER(FilterJob), _I, _I, _P]
_lib.mcl_job_bytes.argtypes = [_I, _I]
_lib.mcl_job_bytes.restype = C.c_size_t
_lib.mcl_map_bytes.argtypes = [_P]
_lib.mcl_map_bytes.restype = C.c_size_t
_lib.mcl_autotune.argtypes = [_P, _P, _I, _P, _I, C.c_float, _P, _P, C.POINTER(LaunchConfig)]
_lib.mcl_set_launch_config.argtypes = [_I, _I, _I, C.POINTER(LaunchConfig)]
_lib.mcl_get_launch_config.argtypes = [_I, _I, _I, C.POINTER(LaunchConfig)]
_lib.mcl_set_weights_fused_max.argtypes = [_I]
_lib.mcl_get_weights_fused_max.argtypes = []
_lib.mcl_get_weights_fused_max.restype = C.c_int32
_lib.mcl_set_spatial_order_min.argtypes = [C.c_int64]
_lib.mcl_get_spatial_order_min.argtypes = []
_lib.mcl_get_spatial_order_min.restype = C.c_int64
_lib.mcl_bench_gather_offsets.argtypes = [_P, _P, _I, _P, _I, _I, _P, _P]
_lib.mcl_bench_gather_replay.argtypes = [_P, _P, _I, _I, _I, _I, _I, _P, C.c_size_t, _P]
_lib.mcl_bench_line_gather.argtypes = [_P, C.c_size_t, _I, _I, _I, _I, C.c_uint32, _I, _P, C.c_size_t, _P]
_lib.mcl_bench_stream_read.argtypes = [_P, C.c_size_t, _I, _P, C.c_size_t, _P]
_lib.mcl_bench_l1_gather.argtypes = [_P, C.c_size_t, _I, _I, _I, _I, _P, C.c_size_t, _P]
_lib.mcl_last_error.restype = C.c_char_p
for _f in ("mcl_map_upload", "mcl_map_upload_bricks", "mcl_map_free", "mcl_sensor_update", "mcl_sensor_update_trilinear",
           "mcl_sensor_update_noalloc", "mcl_sensor_update_sum", "mcl_normalize",
           "mcl_resample",
           "mcl_debug_voxel_indices", "mcl_tick", "mcl_autotune", "mcl_set_launch_config", "mcl_get_launch_config",
           "mcl_set_weights_fused_max", "mcl_set_spatial_order_min",
           "mcl_pose_estimate", "mcl_motion_update",
           "mcl_init_uniform", "mcl_init_gaussian", "mcl_debug_philox", "mcl_bench_gather_offsets",
           "mcl_bench_gather_replay", "mcl_bench_line_gather", "mcl_bench_stream_read", "mcl_bench_l1_gather"):
    getattr(_lib, _f).restype = C.c_int32


class MclError(RuntimeError):
    def __init__(self, status: int, what: str):
        msg = _lib.mcl_last_error().decode()
        super().__init__(f"{what} failed with status {status}: {msg}")
        self.status = status


def _check(status: int, what: str):
    if status != MCL_OK:
        raise MclError(status, what)


def lib():
    return _lib


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev(t, dtype, shape=None, name="tensor"):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


class Map:
    """A TSDF map resident in device memory (library-owned brick layout)."""

    def __init__(self, values: np.ndarray, voxel: float, origin, tau: float, dtype: str, stream=None):
        vals = np.ascontiguousarray(values)
        nz, ny, nx = vals.shape
        d = MapDesc(nx, ny, nz, float(voxel), (C.c_float * 3)(*[float(o) for o in origin]), float(tau),
                    DTYPE_CODE[dtype])
        h = _P()
        _check(_lib.mcl_map_upload(C.byref(d), vals.ctypes.data_as(_P), _stream(stream), C.byref(h)),
               "mcl_map_upload")
        self._h = h
        self.dims = (nx, ny, nz)
        self.dtype = dtype
        self.voxel, self.tau = float(voxel), float(tau)

    @classmethod
    def from_tsdf(cls, tmap, stream=None) -> "Map":
        return cls(tmap.values, tmap.voxel, tmap.origin, tmap.tau, tmap.dtype, stream)

    @classmethod
    def from_bricks(cls, dims, voxel: float, origin, tau: float, dtype: str, coords: np.ndarray,
                    values: np.ndarray, stream=None) -> "Map":
        """Sparse coarse/fine map: coords [M, 3] int32 (bx, by, bz), values [M, 64] of the
        storage type (in-brick index x + 4 y + 16 z); unlisted bricks read +Q."""
        nx, ny, nz = dims
        d = MapDesc(nx, ny, nz, float(voxel), (C.c_float * 3)(*[float(o) for o in origin]), float(tau),
                    DTYPE_CODE[dtype])
        co = np.ascontiguousarray(coords, np.int32).reshape(-1, 3)
        want = {"i16": np.int16, "i8": np.int8, "f32": np.float32}[dtype]
        va = np.ascontiguousarray(values, want).reshape(-1, 64)
        if co.shape[0] != va.shape[0]:
            raise ValueError("coords and values must list the same bricks")
        h = _P()
        _check(_lib.mcl_map_upload_bricks(C.byref(d), co.shape[0], co.ctypes.data_as(_P), va.ctypes.data_as(_P),
                                          _stream(stream), C.byref(h)), "mcl_map_upload_bricks")
        self = cls.__new__(cls)
        self._h = h
        self.dims = (nx, ny, nz)
        self.dtype = dtype
        self.voxel, self.tau = float(voxel), float(tau)
        return self

    @property
    def handle(self):
        return self._h

    @property
    def device_bytes(self) -> int:
        return int(_lib.mcl_map_bytes(self._h))

    def close(self):
        if getattr(self, "_h", None):
            _lib.mcl_map_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sensor_update(m: Map, points, poses, sigma: float, logw=None, stream=None):
    """logw [N] float32 = -(1/(2 sigma^2)) sum_k m(x_n, z_k)^2 (see include/mcl.h)."""
    import torch
    K = points.shape[1] if points is not None else 0
    N = poses.shape[1]
    _dev(poses, torch.float32, (12, N), "poses")
    if K:
        _dev(points, torch.float32, (3, K), "points")
    if logw is None:
        logw = torch.empty(N, dtype=torch.float32, device=poses.device)
    _dev(logw, torch.float32, (N,), "logw")
    _check(_lib.mcl_sensor_update(m.handle, _ptr(points) if K else None, K, _ptr(poses), N,
                                  float(sigma), _ptr(logw), _stream(stream)), "mcl_sensor_update")
    return logw


def sensor_update_noalloc(m: Map, points, poses, sigma: float, logw, stream=None):
    """mcl_sensor_update's result, computed with the library's fixed scratch
    array instead of a workspace (no device allocation; for graph capture).
    logw must be given, since allocating it would defeat the purpose."""
    import torch
    K = points.shape[1] if points is not None else 0
    N = poses.shape[1]
    _dev(poses, torch.float32, (12, N), "poses")
    if K:
        _dev(points, torch.float32, (3, K), "points")
    _dev(logw, torch.float32, (N,), "logw")
    _check(_lib.mcl_sensor_update_noalloc(m.handle, _ptr(points) if K else None, K, _ptr(poses), N,
                                          float(sigma), _ptr(logw), _stream(stream)), "mcl_sensor_update_noalloc")
    return logw


def sensor_update_sum(m: Map, points, poses, sigma: float, logw=None, stream=None):
    """logw [N] float32 = log sum_k exp(-(1/(2 sigma^2)) m(x_n, z_k)^2), the sum
    reading of the sensor model (see include/mcl.h)."""
    import torch
    K = points.shape[1] if points is not None else 0
    N = poses.shape[1]
    _dev(poses, torch.float32, (12, N), "poses")
    if K:
        _dev(points, torch.float32, (3, K), "points")
    if logw is None:
        logw = torch.empty(N, dtype=torch.float32, device=poses.device)
    _dev(logw, torch.float32, (N,), "logw")
    _check(_lib.mcl_sensor_update_sum(m.handle, _ptr(points) if K else None, K, _ptr(poses), N,
                                      float(sigma), _ptr(logw), _stream(stream)), "mcl_sensor_update_sum")
    return logw


def sensor_update_trilinear(m: Map, points, poses, sigma: float, logw=None, stream=None):
    """logw [N] float32 with the trilinear lookup (see include/mcl.h)."""
    import torch
    K = points.shape[1] if points is not None else 0
    N = poses.shape[1]
    _dev(poses, torch.float32, (12, N), "poses")
    if K:
        _dev(points, torch.float32, (3, K), "points")
    if logw is None:
        logw = torch.empty(N, dtype=torch.float32, device=poses.device)
    _dev(logw, torch.float32, (N,), "logw")
    _check(_lib.mcl_sensor_update_trilinear(m.handle, _ptr(points) if K else None, K, _ptr(poses), N,
                                            float(sigma), _ptr(logw), _stream(stream)), "mcl_sensor_update_trilinear")
    return logw


def normalize(logw, w=None, wq=None, log_z=None, want_w=True, stream=None):
    """(w float64 [N] or None, wq uint64 [N], log_z float64 [1])."""
    import torch
    N = logw.shape[0]
    _dev(logw, torch.float32, (N,), "logw")
    dev = logw.device
    if w is None and want_w:
        w = torch.empty(N, dtype=torch.float64, device=dev)
    if wq is None:
        wq = torch.empty(N, dtype=torch.uint64, device=dev)
    if log_z is None:
        log_z = torch.empty(1, dtype=torch.float64, device=dev)
    _check(_lib.mcl_normalize(_ptr(logw), N, _ptr(w), _ptr(wq), _ptr(log_z), _stream(stream)), "mcl_normalize")
    return w, wq, log_z


def resample(wq, seed: int, tick: int, poses_in=None, poses_out=None, idx=None, stream=None):
    """(idx int32 [N], poses_out [12, N] or None); the draw is selected by (seed, tick)."""
    import torch
    N = wq.shape[0]
    _dev(wq, torch.uint64, (N,), "wq")
    if idx is None:
        idx = torch.empty(N, dtype=torch.int32, device=wq.device)
    if poses_in is not None and poses_out is None:
        poses_out = torch.empty_like(poses_in)
    _check(_lib.mcl_resample(_ptr(wq), N, C.c_uint64(int(seed) & (2 ** 64 - 1)), C.c_uint64(int(tick) & (2 ** 64 - 1)),
                             _ptr(idx), _ptr(poses_in), _ptr(poses_out), _stream(stream)), "mcl_resample")
    return idx, poses_out


def pose_estimate(w, poses, mean=None, best_idx=None, best_pose=None, stream=None):
    """(mean float64 [12], best_idx int32 [1], best_pose float32 [12]) on the device."""
    import torch
    N = poses.shape[1]
    _dev(w, torch.float64, (N,), "w")
    _dev(poses, torch.float32, (12, N), "poses")
    if mean is None:
        mean = torch.empty(12, dtype=torch.float64, device=poses.device)
    if best_idx is None:
        best_idx = torch.empty(1, dtype=torch.int32, device=poses.device)
    if best_pose is None:
        best_pose = torch.empty(12, dtype=torch.float32, device=poses.device)
    _check(_lib.mcl_pose_estimate(_ptr(w), _ptr(poses), N, _ptr(mean), _ptr(best_idx), _ptr(best_pose),
                                  _stream(stream)), "mcl_pose_estimate")
    return mean, best_idx, best_pose


def motion_update(poses_in, delta, sigma_t: float, sigma_r: float, seed: int, step: int, poses_out=None,
                  stream=None):
    """Poses [12, N] after the motion update (in place if poses_out is poses_in)."""
    import torch
    N = poses_in.shape[1]
    _dev(poses_in, torch.float32, (12, N), "poses_in")
    if poses_out is None:
        poses_out = torch.empty_like(poses_in)
    _dev(poses_out, torch.float32, (12, N), "poses_out")
    d = np.ascontiguousarray(np.asarray(delta, np.float32).reshape(12))
    _check(_lib.mcl_motion_update(_ptr(poses_in), _ptr(poses_out), N, d.ctypes.data_as(C.c_void_p), float(sigma_t),
                                  float(sigma_r), C.c_uint64(int(seed) & (2 ** 64 - 1)),
                                  C.c_uint64(int(step) & (2 ** 64 - 1)), _stream(stream)), "mcl_motion_update")
    return poses_out


def init_uniform(m: Map, N: int, max_tilt: float, seed: int, poses=None, device=None, stream=None):
    """[12, N] poses uniform over the map's free voxels (see include/mcl.h)."""
    import torch
    if poses is None:
        poses = torch.empty((12, N), dtype=torch.float32, device=device or "cuda")
    _dev(poses, torch.float32, (12, N), "poses")
    _check(_lib.mcl_init_uniform(m.handle, _ptr(poses), N, float(max_tilt), C.c_uint64(int(seed) & (2 ** 64 - 1)),
                                 _stream(stream)), "mcl_init_uniform")
    return poses


def init_gaussian(mean, N: int, sigma_t: float, sigma_r: float, seed: int, step: int = 0, poses=None, device=None,
                  stream=None):
    """[12, N] poses spread round the pose `mean` (12 floats: R row-major, t), see include/mcl.h."""
    import torch
    if poses is None:
        poses = torch.empty((12, N), dtype=torch.float32, device=device or "cuda")
    _dev(poses, torch.float32, (12, N), "poses")
    mv = np.ascontiguousarray(np.asarray(mean, np.float32).reshape(12))
    _check(_lib.mcl_init_gaussian(_ptr(poses), N, mv.ctypes.data_as(C.c_void_p), float(sigma_t), float(sigma_r),
                                  C.c_uint64(int(seed) & (2 ** 64 - 1)), C.c_uint64(int(step) & (2 ** 64 - 1)),
                                  _stream(stream)), "mcl_init_gaussian")
    return poses


def debug_philox(counter, key) -> np.ndarray:
    """Philox4x32-10 on the device (test support): 4 uint32 words."""
    ck = np.ascontiguousarray(list(counter) + list(key), np.uint32)
    out = np.empty(4, np.uint32)
    _check(_lib.mcl_debug_philox(ck.ctypes.data_as(C.c_void_p), out.ctypes.data_as(C.c_void_p)), "mcl_debug_philox")
    return out


def debug_voxel_indices(m: Map, points, poses, out=None, stream=None):
    import torch
    K, N = points.shape[1], poses.shape[1]
    if out is None:
        out = torch.empty((N, K), dtype=torch.int64, device=poses.device)
    _check(_lib.mcl_debug_voxel_indices(m.handle, _ptr(points), K, _ptr(poses), N, _ptr(out), _stream(stream)),
           "mcl_debug_voxel_indices")
    return out


class Filter:
    """Device buffers of one filter for a batched tick (see include/mcl.h, mcl_tick).

    poses, poses_out: [12, N] float32; points: [3, K] float32 or None.  Output
    buffers are allocated here unless given.
    """

    def __init__(self, m: Map, points, poses, sigma: float, seed: int, tick: int = 0, want_w: bool = True,
                 resample_poses: bool = True, want_estimate: bool = False, trilinear: bool = False,
                 score: str = "product"):
        import torch
        self.map = m
        self.points = points
        self.poses = poses
        self.sigma = float(sigma)
        self.seed = int(seed)        # resampling draw of this update: (seed, tick)
        self.tick = int(tick)
        self.trilinear = bool(trilinear)   # the sensor update as mcl_sensor_update_trilinear
        if score not in ("product", "sum"):
            raise ValueError("score must be 'product' or 'sum'")
        self.score = score                  # "sum": the sensor update as mcl_sensor_update_sum
        N = poses.shape[1]
        dev = poses.device
        self.logw = torch.empty(N, dtype=torch.float32, device=dev)
        self.w = torch.empty(N, dtype=torch.float64, device=dev) if want_w else None
        self.wq = torch.empty(N, dtype=torch.uint64, device=dev)
        self.log_z = torch.empty(1, dtype=torch.float64, device=dev)
        self.idx = torch.empty(N, dtype=torch.int32, device=dev)
        self.poses_out = torch.empty_like(poses) if resample_poses else None
        if want_estimate and self.w is None:
            raise ValueError("a pose estimate needs the weights (want_w=True)")
        self.est_mean = torch.empty(12, dtype=torch.float64, device=dev) if want_estimate else None
        self.est_idx = torch.empty(1, dtype=torch.int32, device=dev) if want_estimate else None
        self.est_pose = torch.empty(12, dtype=torch.float32, device=dev) if want_estimate else None

    @property
    def N(self):
        return self.poses.shape[1]

    @property
    def K(self):
        return 0 if self.points is None else self.points.shape[1]

    # ------------------------------------------------------ checkpoint / resume
    def state_dict(self) -> dict:
        """The filter's state as host copies: the particle set the next update
        reads, and (seed, tick), which fix that update's resampling draw.  The
        copy runs on the current stream: work that writes the poses on another
        stream must have completed."""
        return {"poses": self.poses.cpu().numpy(), "sigma": self.sigma, "seed": self.seed, "tick": self.tick,
                "score": self.score, "trilinear": self.trilinear}

    def load_state_dict(self, state: dict):
        """Restores a state_dict() into this filter's buffers (same N; the copy
        runs on the current stream); the next update then draws exactly as the
        saved filter's would have."""
        import torch
        poses = np.ascontiguousarray(state["poses"], np.float32)
        if poses.shape != tuple(self.poses.shape):
            raise ValueError(f"poses of shape {poses.shape} for a filter of shape {tuple(self.poses.shape)}")
        self.poses.copy_(torch.from_numpy(poses))
        self.sigma, self.seed, self.tick = float(state["sigma"]), int(state["seed"]), int(state["tick"])
        self.score, self.trilinear = str(state["score"]), bool(state["trilinear"])

    def save(self, path: str):
        """state_dict() to a .npz file (plain arrays, no pickled objects)."""
        st = self.state_dict()
        np.savez(path, poses=st["poses"], sigma=np.float64(st["sigma"]), seed=np.uint64(st["seed"]),
                 tick=np.uint64(st["tick"]), score=np.str_(st["score"]), trilinear=np.bool_(st["trilinear"]))

    def load(self, path: str):
        """Restores a file written by save()."""
        with np.load(path, allow_pickle=False) as z:
            self.load_state_dict({"poses": z["poses"], "sigma": float(z["sigma"]), "seed": int(z["seed"]),
                                  "tick": int(z["tick"]), "score": str(z["score"]),
                                  "trilinear": bool(z["trilinear"])})

    def job(self) -> FilterJob:
        import torch
        _dev(self.poses, torch.float32, (12, self.N), "poses")
        if self.K:
            _dev(self.points, torch.float32, (3, self.K), "points")
        return FilterJob(self.map.handle, _ptr(self.points) if self.K else None, self.K, _ptr(self.poses), self.N,
                         self.sigma, _ptr(self.logw), _ptr(self.w), _ptr(self.wq), _ptr(self.log_z),
                         self.seed & (2 ** 64 - 1), self.tick & (2 ** 64 - 1), _ptr(self.idx), _ptr(self.poses_out),
                         _ptr(self.est_mean),
                         _ptr(self.est_idx), _ptr(self.est_pose), LOOKUP_TRILINEAR if self.trilinear else LOOKUP_NEAREST,
                         SCORE_SUM if self.score == "sum" else SCORE_PRODUCT)


def tick(filters, graph: bool = False, stream=None, nowait: bool = False) -> bool:
    """One batched update (sensor, normalise, pose estimate if asked, resample) of every filter.
    nowait: return False (nothing enqueued) instead of blocking while the stream's
    previous tick still holds the table staging buffer (MCL_EBUSY)."""
    arr = (FilterJob * len(filters))(*[f.job() for f in filters])
    flags = (TICK_GRAPH if graph else 0) | (TICK_NOWAIT if nowait else 0)
    st = _lib.mcl_tick(arr, len(filters), flags, _stream(stream))
    if st == MCL_EBUSY and nowait:
        return False
    _check(st, "mcl_tick")
    return True


def job_bytes(N: int, K: int) -> int:
    return int(_lib.mcl_job_bytes(N, K))


def autotune(m: Map, points, poses, sigma: float, stream=None):
    """Tune the sensor kernel's launch settings on this filter; returns
    (waves_per_block, blocks_per_cu, coarse, runs, lds_threshold)."""
    import torch
    N, K = poses.shape[1], points.shape[1]
    scratch = torch.empty(N, dtype=torch.float32, device=poses.device)
    best = LaunchConfig()
    _check(_lib.mcl_autotune(m.handle, _ptr(points), K, _ptr(poses), N, float(sigma), _ptr(scratch),
                             _stream(stream), C.byref(best)), "mcl_autotune")
    return best.waves_per_block, best.blocks_per_cu, best.coarse, best.runs, best.lds_threshold


def get_launch_config(dtype: str, K: int, N: int):
    """(waves_per_block, blocks_per_cu, coarse, runs, lds_threshold) the sensor update would use."""
    c = LaunchConfig()
    _check(_lib.mcl_get_launch_config(DTYPE_CODE[dtype], K, N, C.byref(c)), "mcl_get_launch_config")
    return c.waves_per_block, c.blocks_per_cu, c.coarse, c.runs, c.lds_threshold


def set_launch_config(dtype: str, K: int, N: int, cfg=None):
    """cfg = (waves_per_block, blocks_per_cu[, coarse[, runs[, lds_threshold]]]), or None to clear;
    coarse: 0 auto, 1 global bytes, 2 LDS bits; runs: 0 automatic or a power of two <= 64."""
    c = None if cfg is None else C.byref(LaunchConfig(*cfg))
    _check(_lib.mcl_set_launch_config(DTYPE_CODE[dtype], K, N, c), "mcl_set_launch_config")


def set_weights_fused_max(max_n: int):
    """Filters of at most max_n particles normalise and resample with one
    workgroup each in one launch (0: never); the results are the same bits
    either way.  Returns the previous value."""
    prev = int(_lib.mcl_get_weights_fused_max())
    _check(_lib.mcl_set_weights_fused_max(int(max_n)), "mcl_set_weights_fused_max")
    return prev


def get_weights_fused_max() -> int:
    return int(_lib.mcl_get_weights_fused_max())


def set_spatial_order_min(min_evals: int):
    """Dense-map sensor updates of at least min_evals particle-point evaluations
    visit the particles sorted by their x-y cell (negative: never); the results
    are the same bits either way.  Returns the previous value."""
    prev = int(_lib.mcl_get_spatial_order_min())
    _check(_lib.mcl_set_spatial_order_min(int(min_evals)), "mcl_set_spatial_order_min")
    return prev


def get_spatial_order_min() -> int:
    return int(_lib.mcl_get_spatial_order_min())


# ------------------------------------------------------------ measurement support
def bench_gather_offsets(m: Map, points, poses, masked: bool, out=None, stream=None):
    """[N, K] uint32 byte offsets the nearest lookup reads (see include/mcl.h)."""
    import torch
    K, N = points.shape[1], poses.shape[1]
    if out is None:
        out = torch.empty((N, K), dtype=torch.uint32, device=poses.device)
    _check(_lib.mcl_bench_gather_offsets(m.handle, _ptr(points), K, _ptr(poses), N, int(masked), _ptr(out),
                                         _stream(stream)), "mcl_bench_gather_offsets")
    return out


def bench_gather_replay(m: Map, offs, reps: int, two_gathers: bool, blocks: int, sink, stream=None):
    S, K = offs.shape
    _check(_lib.mcl_bench_gather_replay(m.handle, _ptr(offs), S, K, int(reps), int(two_gathers), int(blocks),
                                        _ptr(sink), sink.numel(), _stream(stream)), "mcl_bench_gather_replay")


def bench_line_gather(region, log2_lines: int, lines: int, steps: int, seed: int, blocks: int, sink, stream=None,
                      bytes_per_lane: int = 4):
    _check(_lib.mcl_bench_line_gather(_ptr(region), region.numel() * region.element_size(), int(log2_lines),
                                      int(lines), int(bytes_per_lane), int(steps), int(seed) & 0xFFFFFFFF, int(blocks),
                                      _ptr(sink), sink.numel(), _stream(stream)), "mcl_bench_line_gather")


def bench_l1_gather(block, lines: int, bytes_per_lane: int, steps: int, blocks: int, sink, stream=None):
    _check(_lib.mcl_bench_l1_gather(_ptr(block), block.numel() * block.element_size(), int(lines), int(bytes_per_lane),
                                    int(steps), int(blocks), _ptr(sink), sink.numel(), _stream(stream)),
           "mcl_bench_l1_gather")


def bench_stream_read(src, blocks: int, sink, stream=None):
    _check(_lib.mcl_bench_stream_read(_ptr(src), src.numel() * src.element_size(), int(blocks), _ptr(sink),
                                      sink.numel(), _stream(stream)), "mcl_bench_stream_read")
