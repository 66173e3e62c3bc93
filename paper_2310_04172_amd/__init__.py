"""6-DoF Monte Carlo localisation sensor update in TSDF maps for MI355X (gfx950).

The HIP library behind ``include/mcl.h`` is loaded by ``paper_2310_04172_amd.mcl``;
importing this package itself loads nothing, so the build step can run without it.
"""

__all__ = ["mcl"]
