"""Pins for the oracle's sum reading of the sensor model (a particle's weight is
the sum of the points' Eq. 3 likelihoods, l_n = log sum_k exp(-c q_k^2)).

Each test checks the oracle against something it does not compute itself: a
closed form on lattice-aligned inputs (the voxels are known by construction,
the terms summed exactly with math.fsum), the single-point case where both
readings must agree, the all-outside closed form, and the bounds that relate
the two readings (Jensen's inequality: the log of a mean of exponentials is at
least the mean of the exponents, with equality when the terms are equal).
"""

import math

import numpy as np
import pytest

from tests.helpers import identity_poses, make_map, poses_from, random_rotations
from workloads.tsdf import f32


def score_const(tmap, sigma):
    s = 1.0 if tmap.dtype in ("f32", "f64") else float(tmap.tau) / tmap.Q
    return (s * s) / (2.0 * float(sigma) ** 2)


def _lattice_map(rng, dtype, nx=8, ny=6, nz=5, tau=0.3):
    if dtype in ("f32", "f64"):
        vals = rng.uniform(-tau, tau, size=(nz, ny, nx)).astype(np.float32 if dtype == "f32" else np.float64)
    else:
        lim = 127 if dtype == "i8" else 32767
        vals = rng.permutation(np.linspace(-lim, lim, nx * ny * nz).round()).reshape(nz, ny, nx)
        vals = vals.astype(np.int8 if dtype == "i8" else np.int16)
    return vals, make_map(vals, 0.125, tau=tau, dtype=dtype)


@pytest.mark.parametrize("dtype", ["i16", "i8", "f32", "f64"])
def test_sum_identity_pose_closed_form(oracle_lib, dtype):
    """Identity pose, dyadic voxel, points at voxel centres: each point's voxel is
    known, and l = log(sum_k exp(-c q_k^2)) with the terms added exactly."""
    rng = np.random.default_rng(31)
    vals, tmap = _lattice_map(rng, dtype)
    nz, ny, nx = vals.shape
    K = 301
    ii, jj, kk = rng.integers(0, nx, K), rng.integers(0, ny, K), rng.integers(0, nz, K)
    pts = ((np.stack([ii, jj, kk]).astype(np.float64) + 0.5) * tmap.voxel).astype(np.float32)
    sigma = f32(0.11)
    lw, S = oracle_lib.sensor_update_sum(tmap, pts, identity_poses(1), sigma, return_sum=True)
    c = score_const(tmap, sigma)
    q = vals[kk, jj, ii].astype(np.float64)
    expect = math.fsum(math.exp(-c * float(x) * float(x)) for x in q)
    assert abs(S[0] - expect) <= 1e-13 * expect
    assert abs(lw[0] - math.log(expect)) <= 1e-13


@pytest.mark.parametrize("dtype", ["i16", "i8", "f32"])
def test_single_point_scans_agree_with_the_product_reading(oracle_lib, dtype):
    """With one point the sum and the product of likelihoods are the same
    number: l_sum = log(exp(-c q^2)) = l_prod, for every particle and point."""
    rng = np.random.default_rng(32)
    vals, tmap = _lattice_map(rng, dtype)
    N = 9
    poses = poses_from(random_rotations(rng, N), rng.uniform(0.0, 0.9, (N, 3)))
    sigma = f32(0.13)
    for k in range(12):
        pt = rng.uniform(-0.4, 0.9, size=(3, 1)).astype(np.float32)
        ls = oracle_lib.sensor_update_sum(tmap, pt, poses, sigma)
        lp = oracle_lib.sensor_update(tmap, pt, poses, sigma)
        np.testing.assert_allclose(ls, lp, rtol=1e-14, atol=1e-15)


def test_sum_empty_scan_and_all_outside(oracle_lib):
    """No points: l = 0 (equal weights).  Every point outside the map reads +Q:
    l = log(K) - c Q^2."""
    rng = np.random.default_rng(33)
    vals = rng.integers(-32767, 32768, size=(4, 4, 4)).astype(np.int16)
    tmap = make_map(vals, 0.1, tau=0.3)
    sigma = f32(0.15)
    poses = poses_from(random_rotations(rng, 3), rng.uniform(0, 0.4, (3, 3)))
    assert np.all(oracle_lib.sensor_update_sum(tmap, np.zeros((3, 0), np.float32), poses, sigma) == 0.0)
    far = np.full((3, 50), 1e4, np.float32)
    lw = oracle_lib.sensor_update_sum(tmap, far, poses, sigma)
    c = score_const(tmap, sigma)
    np.testing.assert_allclose(lw, math.log(50) - c * 32767 ** 2, rtol=0, atol=1e-13)


def test_sum_reading_bounds(oracle_lib):
    """For random poses and scans: log K + l_prod / K <= l_sum <= log K (terms in
    (0, 1], mean of exponents below the log of the mean exponential), so a
    wrong sign, a wrong constant or a dropped term shows."""
    rng = np.random.default_rng(34)
    vals = rng.integers(-32767, 32768, size=(10, 12, 14)).astype(np.int16)
    tmap = make_map(vals, 0.1, tau=0.3)
    N, K = 29, 173
    poses = poses_from(random_rotations(rng, N), rng.uniform(0, 1.0, (N, 3)))
    pts = rng.uniform(-0.6, 0.6, size=(3, K)).astype(np.float32)
    sigma = f32(0.12)
    ls = oracle_lib.sensor_update_sum(tmap, pts, poses, sigma)
    lp = oracle_lib.sensor_update(tmap, pts, poses, sigma)
    assert np.all(ls <= math.log(K) + 1e-12)
    assert np.all(ls >= math.log(K) + lp / K - 1e-12)
    # strictly inside both bounds here (the points read different values)
    assert np.all(ls < math.log(K) - 1e-3) and np.all(ls > math.log(K) + lp / K + 1e-3)


def test_sum_particle_permutation_and_threads(oracle_lib):
    rng = np.random.default_rng(35)
    vals = rng.integers(-32767, 32768, size=(10, 12, 14)).astype(np.int16)
    tmap = make_map(vals, 0.1, tau=0.3)
    N = 37
    poses = poses_from(random_rotations(rng, N), rng.uniform(0, 1.0, (N, 3)))
    pts = rng.uniform(-0.6, 0.6, size=(3, 211)).astype(np.float32)
    lw = oracle_lib.sensor_update_sum(tmap, pts, poses, f32(0.15))
    perm = rng.permutation(N)
    lw_p = oracle_lib.sensor_update_sum(tmap, pts, np.ascontiguousarray(poses[:, perm]), f32(0.15))
    assert np.array_equal(lw_p, lw[perm])
    assert np.array_equal(oracle_lib.sensor_update_sum(tmap, pts, poses, f32(0.15), nthreads=5), lw)
