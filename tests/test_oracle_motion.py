"""Pins for the oracle's random numbers, motion update and uniform
initialisation (§III: particles start uniformly in free space; the motion model
moves every particle by the odometry with noise, §VI)."""

import math
import os

import numpy as np
import pytest
from scipy import stats

from tests.helpers import make_map, poses_from, random_rotations

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers(oracle_lib):
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        w = [int(x, 16) for x in r]
        out = oracle_lib.philox4x32(w[0:4], w[4:6])
        assert [int(x) for x in out] == w[6:10]


def rotation_log(R):
    """Rotation vector of a rotation matrix (angle below pi)."""
    c = max(-1.0, min(1.0, (np.trace(R) - 1.0) / 2.0))
    th = math.acos(c)
    v = np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    if th < 1e-12:
        return v / 2.0
    return v * th / (2.0 * math.sin(th))


def test_normals_are_standard_normal(oracle_lib):
    N = 100000
    P = poses_from(np.repeat(np.eye(3)[None], N, 0), np.zeros((N, 3)))
    _, nrm = oracle_lib.motion_update(P, np.r_[np.eye(3).ravel(), 0, 0, 0], 1.0, 1.0, seed=99, step=3,
                                      return_normals=True)
    x = nrm.ravel()
    assert abs(x.mean()) < 5 / math.sqrt(x.size)
    assert abs(x.var() - 1.0) < 5 * math.sqrt(2.0 / x.size)
    assert stats.kstest(x, "norm").pvalue > 1e-4
    c = np.corrcoef(nrm)
    assert np.all(np.abs(c - np.eye(6)) < 5 / math.sqrt(N))
    # another step gives other numbers
    _, nrm2 = oracle_lib.motion_update(P[:, :1000], np.r_[np.eye(3).ravel(), 0, 0, 0], 1.0, 1.0, seed=99, step=4,
                                       return_normals=True)
    assert not np.allclose(nrm2, nrm[:, :1000])


def test_noise_free_composition(oracle_lib):
    """sigma = 0: R' = R dR, t' = R dt + t exactly (float64 of the float32 inputs)."""
    rng = np.random.default_rng(1)
    N = 50
    P = poses_from(random_rotations(rng, N), rng.normal(0, 5, (N, 3)))
    dR = random_rotations(rng, 1)[0].astype(np.float32).astype(np.float64)
    dt = rng.normal(0, 1, 3).astype(np.float32).astype(np.float64)
    out = oracle_lib.motion_update(P, np.r_[dR.ravel(), dt], 0.0, 0.0, seed=1, step=0)
    for n in range(N):
        R = P[:9, n].astype(np.float64).reshape(3, 3)
        t = P[9:, n].astype(np.float64)
        np.testing.assert_allclose(out[:9, n].reshape(3, 3), R @ dR, atol=1e-15)
        np.testing.assert_allclose(out[9:, n], R @ dt + t, atol=1e-13)


def test_noise_enters_in_the_robot_frame(oracle_lib):
    """(R dR)^-1 R' = Exp(sigma_r n) and R^-1 (t' - t) - dt = sigma_t n for the normals drawn:
    the rotation noise multiplies the increment on the right and the translation
    noise is added to the increment before the pose rotates it."""
    rng = np.random.default_rng(2)
    N = 40
    P = poses_from(random_rotations(rng, N), rng.normal(0, 5, (N, 3)))
    dR = random_rotations(rng, 1)[0].astype(np.float32).astype(np.float64)
    dt = np.array([0.5, -0.25, 0.125])
    st, sr = 0.05, 0.03
    out, nrm = oracle_lib.motion_update(P, np.r_[dR.ravel(), dt], st, sr, seed=5, step=11, return_normals=True)
    for n in range(N):
        R = P[:9, n].astype(np.float64).reshape(3, 3)
        t = P[9:, n].astype(np.float64)
        Rn = out[:9, n].reshape(3, 3)
        # the float32 pose matrices are not exactly orthonormal: undo them exactly
        xi = rotation_log(np.linalg.solve(R @ dR, Rn))
        np.testing.assert_allclose(xi, np.float32(sr) * nrm[3:6, n], atol=1e-9)
        np.testing.assert_allclose(np.linalg.solve(R, out[9:, n] - t) - dt, np.float32(st) * nrm[0:3, n], atol=1e-9)


def test_translation_noise_statistics(oracle_lib):
    rng = np.random.default_rng(3)
    N = 20000
    R0 = random_rotations(rng, 1)[0]
    P = poses_from(np.repeat(R0[None], N, 0), np.zeros((N, 3)))
    out = oracle_lib.motion_update(P, np.r_[np.eye(3).ravel(), 0, 0, 0], 0.1, 0.0, seed=7, step=0)
    local = R0.T @ out[9:]           # back in the robot frame
    assert np.all(np.abs(local.mean(axis=1)) < 5 * 0.1 / math.sqrt(N))
    np.testing.assert_allclose(np.cov(local), 0.01 * np.eye(3), atol=5 * 0.01 * math.sqrt(2.0 / N))


def small_free_map(seed, dims=(7, 5, 4), frac=0.3, dtype="i16"):
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    free = rng.random((nz, ny, nx)) < frac
    if dtype == "f32":
        vals = np.where(free, 0.1, -0.1).astype(np.float32)
    else:
        vals = np.where(free, 100, -100).astype(np.int16 if dtype == "i16" else np.int8)
    return make_map(vals, 0.125, origin=(-0.5, 0.25, 1.0), dtype=dtype), free


@pytest.mark.parametrize("dtype", ["i16", "i8", "f32"])
def test_init_picks_the_rank_from_the_words(oracle_lib, dtype):
    """The chosen voxel is the free voxel of rank floor(U F / 2^64) in x-fastest
    order, U from the first two Philox words (brute force with Python integers);
    the position lies in that voxel."""
    tmap, free = small_free_map(4, dtype=dtype)
    flat = np.flatnonzero(free.ravel())
    F = flat.size
    N = 300
    seed = 0x1234_5678_9ABC
    poses, vox = oracle_lib.init_uniform(tmap, N, 0.1, seed)
    for n in range(N):
        w = oracle_lib.philox4x32([n, 0, 0, 2], [seed & 0xFFFFFFFF, seed >> 32])
        U = int(w[0]) | (int(w[1]) << 32)
        assert vox[n] == flat[(U * F) >> 64]
    nx, ny = tmap.nx, tmap.ny
    ijk = np.stack([vox % nx, (vox // nx) % ny, vox // (nx * ny)])
    lo = np.asarray(tmap.origin)[:, None] + ijk * tmap.voxel
    assert np.all(poses[9:] >= lo - 1e-6) and np.all(poses[9:] <= lo + tmap.voxel + 1e-6)


def test_init_is_uniform_over_free_voxels(oracle_lib):
    tmap, free = small_free_map(5, dims=(4, 3, 2), frac=0.5)
    F = int(free.sum())
    N = 60000
    _, vox = oracle_lib.init_uniform(tmap, N, 0.0, 77)
    counts = np.bincount(np.searchsorted(np.flatnonzero(free.ravel()), vox), minlength=F)
    assert counts.sum() == N
    assert stats.chisquare(counts).pvalue > 1e-4


def test_init_orientation(oracle_lib):
    tmap, _ = small_free_map(6)
    N = 20000
    a = 0.2
    poses, _ = oracle_lib.init_uniform(tmap, N, a, 9)
    R = poses[:9].T.reshape(N, 3, 3)
    np.testing.assert_allclose(np.einsum("nij,nkj->nik", R, R), np.repeat(np.eye(3)[None], N, 0), atol=1e-12)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-12)
    yaw = np.arctan2(R[:, 1, 0], R[:, 0, 0])
    pitch = -np.arcsin(np.clip(R[:, 2, 0], -1, 1))
    roll = np.arctan2(R[:, 2, 1], R[:, 2, 2])
    assert np.all(np.abs(pitch) <= a + 1e-12) and np.all(np.abs(roll) <= a + 1e-12)
    assert stats.kstest((yaw + math.pi) / (2 * math.pi), "uniform").pvalue > 1e-4
    assert stats.kstest((roll + a) / (2 * a), "uniform").pvalue > 1e-4


def test_init_without_free_space(oracle_lib):
    tmap = make_map(np.full((2, 2, 2), -5, np.int16), 0.1)
    with pytest.raises(ValueError):
        oracle_lib.init_uniform(tmap, 10, 0.0, 1)
