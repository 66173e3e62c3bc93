"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

Scenes, TSDF maps, LiDAR scans and particle sets only: this package holds none
of the sensor model's arithmetic (no transform-and-lookup, no scoring, no
normalisation, no resampling).
"""

from .scene import Scene, euler_zyx_to_matrix  # noqa: F401
from .tsdf import TsdfMap, build_map, quantise, voxelise, QSCALE, DTYPE_CODE, f32  # noqa: F401
from . import configs  # noqa: F401
