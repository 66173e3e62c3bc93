"""Pins for the oracle's sparse coarse/fine map (§III, after Akai et al.): the
same score as the dense definition when the listed bricks carry the map's
values, with bricks built here by explicit loops over the layout."""

import numpy as np
import pytest

from tests.helpers import make_map, poses_from, random_rotations
from workloads.tsdf import f32, to_bricks


def bricks_by_loops(vals, Q, keep=None):
    nz, ny, nx = vals.shape
    coords, bricks = [], []
    for by in range((ny + 3) // 4):
        for bx in range((nx + 3) // 4):
            for bz in range((nz + 3) // 4):
                blk = np.full(64, Q, vals.dtype)
                for z in range(4):
                    for y in range(4):
                        for x in range(4):
                            k, j, i = 4 * bz + z, 4 * by + y, 4 * bx + x
                            if k < nz and j < ny and i < nx:
                                blk[x + 4 * y + 16 * z] = vals[k, j, i]
                if keep is None or keep(blk):
                    coords.append((bx, by, bz))
                    bricks.append(blk)
    return np.array(coords, np.int32).reshape(-1, 3), np.array(bricks).reshape(-1, 64)


def case(seed, dims, dtype):
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    Q = {"i16": 32767, "i8": 127, "f32": np.float32(0.3)}[dtype]
    if dtype == "f32":
        vals = rng.uniform(-0.3, 0.3, (nz, ny, nx)).astype(np.float32)
    else:
        vals = rng.integers(-Q, Q + 1, (nz, ny, nx)).astype(np.int16 if dtype == "i16" else np.int8)
    # whole bricks at +-Q, so that the band-only listing differs from the full one
    m = rng.random(((nz + 3) // 4, (ny + 3) // 4, (nx + 3) // 4)) < 0.5
    sgn = np.where(rng.random(m.shape) < 0.5, Q, -Q)
    for bz, by, bx in zip(*np.nonzero(m)):
        vals[4 * bz:4 * bz + 4, 4 * by:4 * by + 4, 4 * bx:4 * bx + 4] = sgn[bz, by, bx]
    tmap = make_map(vals, 0.1, origin=(-0.3, 0.2, -0.1), tau=0.3, dtype=dtype)
    ext = np.array(dims) * 0.1
    N, K = 20, 3000
    poses = poses_from(random_rotations(rng, N), rng.uniform(0, 1, (N, 3)) * ext)
    pts = rng.normal(0, 0.4 * ext.mean(), (3, K)).astype(np.float32)
    return tmap, Q, pts, poses


@pytest.mark.parametrize("dtype", ["i16", "i8", "f32"])
def test_all_bricks_equal_dense(oracle_lib, dtype):
    tmap, Q, pts, poses = case(1, (13, 10, 7), dtype)
    co, va = bricks_by_loops(tmap.values, Q)
    got = oracle_lib.sensor_update_bricks(tmap.dims, tmap.voxel, tmap.origin, tmap.tau, dtype, co, va, pts, poses,
                                          f32(0.15))
    ref = oracle_lib.sensor_update(tmap, pts, poses, f32(0.15))
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("dtype", ["i16", "i8", "f32"])
def test_band_bricks_equal_dense(oracle_lib, dtype):
    """Unlisted bricks read +Q; bricks of +-Q score Q^2 either way."""
    tmap, Q, pts, poses = case(2, (17, 9, 11), dtype)
    co, va = bricks_by_loops(tmap.values, Q, keep=lambda b: bool((np.abs(b.astype(np.float64)) < float(Q)).any()))
    assert 0 < co.shape[0] < ((17 + 3) // 4) * ((9 + 3) // 4) * ((11 + 3) // 4)
    got = oracle_lib.sensor_update_bricks(tmap.dims, tmap.voxel, tmap.origin, tmap.tau, dtype, co, va, pts, poses,
                                          f32(0.15))
    ref = oracle_lib.sensor_update(tmap, pts, poses, f32(0.15))
    assert np.array_equal(got, ref)
    # the input helper lists the same bricks with the same values
    co2, va2 = to_bricks(tmap)
    o1 = np.lexsort(co.T[::-1])
    o2 = np.lexsort(co2.T[::-1])
    assert np.array_equal(co[o1], co2[o2]) and np.array_equal(va[o1], va2[o2])


def test_missing_brick_reads_q(oracle_lib):
    """Dropping a brick with values inside the band changes the score to Q^2 on
    its voxels (closed form on a lattice)."""
    vals = np.full((4, 4, 8), 100, np.int16)          # two bricks along x
    tmap = make_map(vals, 0.125)
    co, va = bricks_by_loops(vals, 32767)
    pts = (np.array([[0.5, 4.5], [0.5, 0.5], [0.5, 0.5]]) * 0.125).astype(np.float32)
    poses = poses_from(np.eye(3)[None], np.zeros((1, 3)))
    c = (float(np.float32(0.3)) / 32767) ** 2 / (2 * float(np.float32(0.1)) ** 2)
    full = oracle_lib.sensor_update_bricks(tmap.dims, tmap.voxel, tmap.origin, tmap.tau, "i16", co, va, pts, poses,
                                           f32(0.1))
    np.testing.assert_allclose(full[0], -c * 2 * 100.0 ** 2, rtol=1e-15)
    keep = co[:, 0] == 0
    part = oracle_lib.sensor_update_bricks(tmap.dims, tmap.voxel, tmap.origin, tmap.tau, "i16", co[keep], va[keep],
                                           pts, poses, f32(0.1))
    np.testing.assert_allclose(part[0], -c * (100.0 ** 2 + 32767.0 ** 2), rtol=1e-15)
