"""Pins of the pose-estimate oracle against closed forms and an independent
formulation (§III / §V pose estimate; the rotation reading is the weighted
chordal L2 mean)."""

import math

import numpy as np
import pytest

from oracle import estimate as E


def rodrigues(axis, ang):
    """Rotation about a unit axis by ang (Rodrigues' formula), float64."""
    u = np.asarray(axis, np.float64)
    u = u / np.linalg.norm(u)
    Kx = np.array([[0, -u[2], u[1]], [u[2], 0, -u[0]], [-u[1], u[0], 0]])
    return np.eye(3) + math.sin(ang) * Kx + (1 - math.cos(ang)) * (Kx @ Kx)


def poses_from(Rs, ts):
    P = np.zeros((12, len(Rs)), np.float32)
    for n, (R, t) in enumerate(zip(Rs, ts)):
        P[0:9, n] = np.asarray(R).reshape(9)
        P[9:12, n] = t
    return P


def quat_from_euler(roll, pitch, yaw):
    """(w, x, y, z) of Rz(yaw) Ry(pitch) Rx(roll), by half-angle products."""
    cr, sr = math.cos(roll / 2), math.sin(roll / 2)
    cp, sp = math.cos(pitch / 2), math.sin(pitch / 2)
    cy, sy = math.cos(yaw / 2), math.sin(yaw / 2)
    return np.array([cy * cp * cr + sy * sp * sr, cy * cp * sr - sy * sp * cr,
                     cy * sp * cr + sy * cp * sr, sy * cp * cr - cy * sp * sr])


def quat_matrix(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def test_position_is_weighted_average():
    # binary-exact inputs: the expected values are exact
    ts = [(1.0, 2.0, 3.0), (-4.0, 0.5, 8.0), (0.25, -2.0, -1.0)]
    P = poses_from([np.eye(3)] * 3, ts)
    for scale in (1.0, 3.0, 1e-3):
        w = np.array([0.5, 0.25, 0.25]) * scale
        mean, _, _ = E.pose_estimate(w, P)
        np.testing.assert_allclose(mean[9:12], [-0.4375, 0.625, 3.25], rtol=1e-15, atol=1e-15)


def test_zero_weights_read_as_equal():
    ts = [(1.0, 0.0, 0.0), (0.0, 2.0, 0.0), (0.0, 0.0, 4.0), (3.0, 2.0, 0.0)]
    P = poses_from([np.eye(3)] * 4, ts)
    mean, b, _ = E.pose_estimate(np.zeros(4), P)
    np.testing.assert_allclose(mean[9:12], [1.0, 1.0, 1.0], rtol=0, atol=0)
    assert b == 0


def test_single_particle_and_identical_rotations():
    R0 = rodrigues((0.3, -0.5, 0.8), 1.1)
    P = poses_from([R0] * 5, [(0.0, 0.0, 0.0)] * 5)
    mean, _, _ = E.pose_estimate(np.array([0.1, 0.3, 0.2, 0.15, 0.25]), P)
    np.testing.assert_allclose(mean[:9].reshape(3, 3), R0, atol=3e-7)


def test_rotations_about_one_axis_closed_form():
    # S = a R(alpha) + b R(beta) about a common axis u factors as
    # R(phi) ((a+b) u u^T + rho (I - u u^T)), phi = atan2(a sin alpha + b sin beta,
    # a cos alpha + b cos beta): the nearest rotation is R(phi).  The weights are
    # unequal, so a transposed result (R(-phi)) fails.
    u = (0.2, 0.9, -0.4)
    a, b, al, be = 0.7, 0.3, math.radians(10), math.radians(50)
    phi = math.atan2(a * math.sin(al) + b * math.sin(be), a * math.cos(al) + b * math.cos(be))
    P = poses_from([rodrigues(u, al), rodrigues(u, be)], [(0, 0, 0)] * 2)
    mean, _, _ = E.pose_estimate(np.array([a, b]), P)
    np.testing.assert_allclose(mean[:9].reshape(3, 3), rodrigues(u, phi), atol=5e-7)
    assert not np.allclose(mean[:9].reshape(3, 3), rodrigues(u, -phi), atol=1e-3)


def test_negative_determinant_needs_the_sign_correction():
    # S = 0.45 Rx(pi) + 0.3 Ry(pi) + 0.25 Rz(pi) = diag(-0.1, -0.4, -0.5), det < 0.
    # Over SO(3), trace(R^T S) is largest for R = diag(1, -1, -1) = Rx(pi); the
    # orthogonal polar factor without the correction would be -I (det -1).
    Rx, Ry, Rz = np.diag([1., -1, -1]), np.diag([-1., 1, -1]), np.diag([-1., -1, 1])
    P = poses_from([Rx, Ry, Rz], [(0, 0, 0)] * 3)
    mean, b, _ = E.pose_estimate(np.array([0.45, 0.3, 0.25]), P)
    np.testing.assert_allclose(mean[:9].reshape(3, 3), Rx, atol=1e-14)
    assert b == 0


def test_equals_quaternion_eigenvector_average():
    # Markley et al. 2007: for exact rotations, the chordal L2 mean is the
    # rotation of the top eigenvector of M = sum w q q^T.  The quaternions are
    # formed from the Euler angles directly, not from the matrices.
    rng = np.random.default_rng(7)
    n = 300
    e = np.array([0.2, -0.1, 2.5]) + rng.normal(0, math.radians(12), (n, 3))
    w = rng.exponential(1.0, n)
    qs = np.array([quat_from_euler(*row) for row in e])
    M = (qs.T * w) @ qs
    _, V = np.linalg.eigh(M)
    Rq = quat_matrix(V[:, -1])
    P = poses_from([quat_matrix(q) for q in qs], [(0, 0, 0)] * n)
    mean, _, _ = E.pose_estimate(w, P)
    np.testing.assert_allclose(mean[:9].reshape(3, 3), Rq, atol=1e-6)


def test_maximises_the_chordal_objective():
    rng = np.random.default_rng(3)
    n = 50
    Rs = [rodrigues(rng.normal(size=3), rng.uniform(0, math.pi)) for _ in range(n)]
    w = rng.uniform(0, 1, n)
    P = poses_from(Rs, [(0, 0, 0)] * n)
    mean, _, _ = E.pose_estimate(w, P)
    R = mean[:9].reshape(3, 3)
    np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-13)
    assert np.linalg.det(R) > 0
    S = (P[0:9].astype(np.float64) * w).sum(axis=1).reshape(3, 3)
    f = np.trace(R.T @ S)
    for _ in range(2000):
        Rp = rodrigues(rng.normal(size=3), rng.uniform(0, math.pi))
        assert np.trace(Rp.T @ S) <= f + 1e-12
    for eps in (1e-2, 1e-4):
        for _ in range(200):
            Rp = R @ rodrigues(rng.normal(size=3), eps)
            assert np.trace(Rp.T @ S) <= f + 1e-12


def test_best_particle_ties_and_nan():
    w = np.array([0.1, 0.4, 0.2, 0.4, np.nan, 0.3])
    assert E.best_particle(w) == 1
    assert E.best_particle(np.array([np.nan, 0.0, 0.0])) == 1
    assert E.best_particle(np.array([np.nan, -np.inf])) == -1
    assert E.best_particle(np.full(7, 0.25)) == 0
    P = poses_from([rodrigues((1, 0, 0), k) for k in range(6)], [(k, -k, 2 * k) for k in range(6)])
    _, b, bp = E.pose_estimate(np.nan_to_num(w), P)
    assert b == 1
    assert np.array_equal(bp, P[:, 1])


@pytest.mark.parametrize("n", [1, 2, 1000])
def test_brute_force_best(n):
    rng = np.random.default_rng(n)
    w = rng.integers(0, 5, n).astype(np.float64)
    best = max(range(n), key=lambda i: (w[i], -i))
    assert E.best_particle(w) == best
