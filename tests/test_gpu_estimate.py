"""Parity of the pose estimate (mcl_pose_estimate, through the C ABI) with the
CPU oracle.

Bars: best index and best pose bit-exact; the mean within a bound derived from
the float64 arithmetic.  Both sides add the same products in different orders:
the library's summation tree is at most 4 + 6 + 4 levels per block and 8 + 6 + 4
across blocks, numpy's pairwise sum at most 8 + log2(N / 8) levels, so each sum
differs by at most 64 u sum|terms| (u = 2^-53).  A perturbation dS of S moves
the nearest rotation by at most 2 |dS|_F / (s2 + s3') (s3' carrying the sign of
det S), and a backward-stable 4x4 eigensolver adds a few u |K| over the same
gap.  Where that bound is not small (S near a repeated case) the rotation is
not unique; there both sides must reach the same value of trace(R^T S).
"""

import math
import sys

import numpy as np
import pytest

from oracle import estimate as E
from tests import checks
from tests.helpers import poses_from, random_rotations
from workloads import configs

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "a GPU is required"
    return t


@pytest.fixture(scope="module")
def mcl():
    from paper_2310_04172_amd import mcl as m
    return m


def run_gpu(torch, mcl, w, P):
    wd = torch.from_numpy(np.ascontiguousarray(w, np.float64)).cuda()
    pd = torch.from_numpy(np.ascontiguousarray(P, np.float32)).cuda()
    mean, bi, bp = mcl.pose_estimate(wd, pd)
    torch.cuda.synchronize()
    return mean.cpu().numpy(), int(bi.cpu().numpy()[0]), bp.cpu().numpy()


def check(torch, mcl, w, P, what):
    say(f"estimate {what}: N={P.shape[1]}")
    g_mean, g_b, g_bp = run_gpu(torch, mcl, w, P)
    o_mean = checks.check_estimate(g_mean, g_b, g_bp, w, P, what)
    return g_mean, o_mean


def tracking_set(seed, n, spread_deg=5.0):
    rng = np.random.default_rng(seed)
    R0 = random_rotations(rng, 1)[0]
    ang = rng.normal(0, math.radians(spread_deg), (n, 3))
    th = np.linalg.norm(ang, axis=1)
    ax = ang / np.maximum(th, 1e-300)[:, None]
    Kx = np.zeros((n, 3, 3))
    Kx[:, 0, 1], Kx[:, 0, 2], Kx[:, 1, 2] = -ax[:, 2], ax[:, 1], -ax[:, 0]
    Kx = Kx - Kx.transpose(0, 2, 1)
    dR = np.eye(3) + np.sin(th)[:, None, None] * Kx + (1 - np.cos(th))[:, None, None] * (Kx @ Kx)
    t = np.array([20.0, 30.0, 1.5]) + rng.normal(0, 0.5, (n, 3))
    w = rng.exponential(1.0, n)
    return w / w.sum(), poses_from(R0 @ dR, t)


@pytest.mark.parametrize("n", [1, 2, 63, 1023, 1024, 1025, 4097, 100003])
def test_tracking_sets(torch, mcl, n):
    w, P = tracking_set(n, n)
    check(torch, mcl, w, P, f"tracking n={n}")


def test_global_set_max_size(torch, mcl):
    n = 1 << 21
    rng = np.random.default_rng(11)
    P = poses_from(random_rotations(rng, n), rng.uniform(0, 100, (n, 3)))
    w = rng.uniform(0, 1, n)
    check(torch, mcl, w / w.sum(), P, "global n=2^21")


def test_degenerate_symmetric_set(torch, mcl):
    # yaw evenly spaced over the full circle with equal weights: S = diag(0, 0, N)
    # up to rounding, every rotation about z attains the maximum
    n = 4096
    yaw = np.arange(n) * (2 * math.pi / n)
    R = np.zeros((n, 3, 3))
    R[:, 0, 0] = R[:, 1, 1] = np.cos(yaw)
    R[:, 0, 1], R[:, 1, 0] = -np.sin(yaw), np.sin(yaw)
    R[:, 2, 2] = 1
    P = poses_from(R, np.zeros((n, 3)))
    check(torch, mcl, np.full(n, 1.0 / n), P, "degenerate")


def test_ties_and_zero_weights(torch, mcl):
    rng = np.random.default_rng(5)
    n = 5000
    P = poses_from(random_rotations(rng, n), rng.normal(0, 3, (n, 3)))
    w = rng.integers(0, 4, n).astype(np.float64)          # many ties at the maximum
    g = check(torch, mcl, w, P, "integer weights with ties")
    check(torch, mcl, np.full(n, 0.25), P, "all equal")
    g_mean, o_mean = check(torch, mcl, np.zeros(n), P, "all zero")
    assert run_gpu(torch, mcl, np.zeros(n), P)[1] == 0
    w1 = np.zeros(n)
    w1[n - 1] = 2.0
    g_mean, _ = check(torch, mcl, w1, P, "one non-zero weight")
    # one particle carries all weight: its translation exactly, its rotation to float32 rounding
    assert np.array_equal(g_mean[9:12], P[9:12, n - 1].astype(np.float64))
    np.testing.assert_allclose(g_mean[:9], P[0:9, n - 1], atol=1e-6)


def test_pipeline_weights(torch, mcl, oracle_lib):
    """Weights as mcl_normalize produces them for a real scene, made by the oracle."""
    wl = configs.config1(n_particles=20000)
    lw = oracle_lib.sensor_update(wl.tmap, wl.points, wl.poses, wl.sigma, nthreads=8)
    w, _, _ = oracle_lib.normalize(lw)
    check(torch, mcl, w, wl.poses, "config1 weights")


def test_reproducible(torch, mcl):
    w, P = tracking_set(9, 300001)
    a = run_gpu(torch, mcl, w, P)
    b = run_gpu(torch, mcl, w, P)
    assert np.array_equal(a[0].view(np.uint64), b[0].view(np.uint64))
