"""Pins for the oracle's trilinear lookup (§III: a pseudo-continuous map value by
interpolation): closed forms on inputs where every float32 step is exact."""

import numpy as np
import pytest

from tests.helpers import identity_poses, make_map

V = 0.125  # a power of two: points on a 1/64 lattice give exact grid coordinates


def affine_map(dims, coef, dtype):
    nx, ny, nz = dims
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d = coef[0] * i + coef[1] * j + coef[2] * k + coef[3]
    np_t = {"i16": np.int16, "i8": np.int8, "f32": np.float32, "f64": np.float64}[dtype]
    return make_map(d.astype(np_t), V, tau=0.3 if dtype in ("i16", "i8") else float(np.abs(d).max()) + 1.0,
                    dtype=dtype)


@pytest.mark.parametrize("dtype,coef", [("i16", (100, -50, 30, 7)), ("i8", (3, -2, 5, -20)),
                                        ("f32", (0.015625, -0.03125, 0.0078125, 0.046875)), ("f64", (0.25, 0.5, -0.125, 1.0))])
def test_affine_field_is_reproduced(oracle_lib, dtype, coef):
    """Trilinear interpolation reproduces an affine field exactly where all 8
    centres are inside: m = a h_x + b h_y + c h_z + e with h = g - 1/2.  A wrong
    half-voxel offset, corner or weight breaks the identity."""
    dims = (9, 7, 6)
    tmap = affine_map(dims, coef, dtype)
    rng = np.random.default_rng(4)
    # g in [0.5, n - 0.5]: every centre around the point is inside
    g = np.stack([rng.integers(32, 64 * d - 32, 300) / 64.0 for d in dims])
    pts = (g * V).astype(np.float32)
    t = np.array([0.0, 0.0, 0.0])
    poses = identity_poses(1, t)
    _, S, A = oracle_lib.sensor_update_trilinear(tmap, pts, poses, 0.1, return_sums=True)
    h = g - 0.5
    m = coef[0] * h[0] + coef[1] * h[1] + coef[2] * h[2] + coef[3]
    np.testing.assert_allclose(S[0], np.sum(m * m), rtol=1e-13)
    np.testing.assert_allclose(A[0], np.sum(np.abs(m)), rtol=1e-13)


def test_translation_and_axis_permutation(oracle_lib):
    """The same affine field seen through a pose that swaps x and y and shifts by
    whole lattice steps (all float32 steps exact)."""
    dims = (8, 8, 5)
    coef = (120, 40, -90, 11)
    tmap = affine_map(dims, coef, "i16")
    rng = np.random.default_rng(5)
    g = np.stack([rng.integers(32, 64 * 8 - 32, 200) / 64.0, rng.integers(32, 64 * 8 - 32, 200) / 64.0,
                  rng.integers(32, 64 * 5 - 32, 200) / 64.0])
    # world point = R p + t with R swapping x and y; choose p so that R p + t = g V
    t = np.array([0.25, -0.5, 0.125])
    R = np.array([[0.0, 1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    xw = g * V
    p = R.T @ (xw - t[:, None])
    poses = np.zeros((12, 1), np.float32)
    poses[:9, 0] = R.reshape(9)
    poses[9:, 0] = t
    _, S, _ = oracle_lib.sensor_update_trilinear(tmap, p.astype(np.float32), poses, 0.1, return_sums=True)
    h = g - 0.5
    m = coef[0] * h[0] + coef[1] * h[1] + coef[2] * h[2] + coef[3]
    np.testing.assert_allclose(S[0], np.sum(m * m), rtol=1e-13)


def test_centres_read_the_stored_value(oracle_lib):
    """At a voxel centre the interpolation is the voxel's own value: the sum
    equals the nearest lookup's, for any map contents."""
    rng = np.random.default_rng(6)
    dims = (6, 5, 4)
    vals = rng.integers(-32767, 32768, (dims[2], dims[1], dims[0])).astype(np.int16)
    tmap = make_map(vals, V)
    k, j, i = np.meshgrid(np.arange(4), np.arange(5), np.arange(6), indexing="ij")
    pts = ((np.stack([i.ravel(), j.ravel(), k.ravel()]) + 0.5) * V).astype(np.float32)
    _, S, _ = oracle_lib.sensor_update_trilinear(tmap, pts, identity_poses(1), 0.1, return_sums=True)
    assert S[0] == float(np.sum(vals.astype(np.int64) ** 2))


def test_boundary_blend_outside_and_nan(oracle_lib):
    """Near the map's low x face the missing centre reads +Q; far outside and NaN
    read +Q on all 8 centres."""
    dims = (4, 4, 4)
    vals = np.full((4, 4, 4), 1000, np.int16)
    tmap = make_map(vals, V)
    Q = 32767
    # g_x = 0.25: h_x = -0.25, i_x = -1, f_x = 0.75: m = 0.25 Q + 0.75 * 1000
    # (y, z at centres 1.5, 2.5 so only x blends)
    pts = np.array([[0.25 * V, 1e4, np.nan], [1.5 * V, 0.0, 0.0], [2.5 * V, 0.0, 0.0]], np.float32)
    _, S, A = oracle_lib.sensor_update_trilinear(tmap, pts, identity_poses(1), 0.1, return_sums=True)
    m0 = 0.25 * Q + 0.75 * 1000
    np.testing.assert_allclose(S[0], m0 * m0 + 2.0 * Q * Q, rtol=1e-15)
    np.testing.assert_allclose(A[0], m0 + 2.0 * Q, rtol=1e-15)


def test_midpoint_is_the_mean_of_two_neighbours(oracle_lib):
    rng = np.random.default_rng(8)
    vals = rng.integers(-30000, 30000, (5, 5, 5)).astype(np.int16)
    tmap = make_map(vals, V)
    # g = (2, 1.5, 3.5): halfway between centres x = 1 and x = 2 at y = 1, z = 3
    pts = (np.array([[2.0], [1.5], [3.5]]) * V).astype(np.float32)
    _, S, _ = oracle_lib.sensor_update_trilinear(tmap, pts, identity_poses(1), 0.1, return_sums=True)
    m = 0.5 * (int(vals[3, 1, 1]) + int(vals[3, 1, 2]))
    assert S[0] == m * m


def test_log_weight_scale(oracle_lib):
    """l = -(s^2 / (2 sigma^2)) sum m^2, s = tau / Q, as for the nearest lookup."""
    vals = np.full((3, 3, 3), 500, np.int16)
    tmap = make_map(vals, V, tau=0.3)
    pts = (np.full((3, 10), 1.5) * V).astype(np.float32)
    lw, S, _ = oracle_lib.sensor_update_trilinear(tmap, pts, identity_poses(1), 0.2, return_sums=True)
    s = float(np.float32(0.3)) / 32767
    sg = float(np.float32(0.2))
    assert S[0] == 10 * 500.0 ** 2
    np.testing.assert_allclose(lw[0], -(s * s) / (2 * sg * sg) * S[0], rtol=1e-15)
