"""Parity of the trilinear lookup (mcl_sensor_update_trilinear, through the C
ABI) with the CPU oracle.

Bar per particle, derived from the float32 arithmetic: the summation bound of
the nearest lookup (3e-6 relative) plus the interpolation error.  Each
interpolated value is within 10 eps M of the exact one (eps = 2^-24, M the
largest stored magnitude: three levels of lerps, each adding one rounding of
its fma and one of its difference), so
    |l_gpu - l| / |l| <= 3e-6 + 1e-6 + (20 eps M sum|m| + 100 K eps^2 M^2) / sum m^2
with sum|m| and sum m^2 from the oracle (the 1e-6 covers the float32 score
constant and product).
"""

import sys

import numpy as np
import pytest

from tests.helpers import identity_poses, make_map, poses_from, random_rotations
from workloads import configs
from workloads.tsdf import f32

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -24


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


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def big_m(tmap):
    return {"i16": 32767.0, "i8": 127.0}.get(tmap.dtype, float(tmap.tau))


def check(torch, mcl, oracle_lib, tmap, pts, poses, sigma, what, m=None):
    m = m or mcl.Map.from_tsdf(tmap)
    lw = mcl.sensor_update_trilinear(m, dev(torch, pts) if pts.shape[1] else None, dev(torch, poses), sigma)
    torch.cuda.synchronize()
    got = lw.cpu().numpy().astype(np.float64)
    ref, S, A = oracle_lib.sensor_update_trilinear(tmap, pts, poses, sigma, nthreads=8, return_sums=True)
    M = big_m(tmap)
    K = pts.shape[1]
    with np.errstate(divide="ignore", invalid="ignore"):
        bound = 4e-6 + (20 * EPS * M * A + 100 * K * (EPS * M) ** 2) / S
        rel = np.abs(got - ref) / np.abs(ref)
    zero = ref == 0
    assert np.all(got[zero] == 0), what
    bad = ~zero & (rel > bound)
    assert not bad.any(), f"{what}: {bad.sum()} particles off, worst rel {rel[~zero].max():.3g}"
    return got, ref


def random_case(seed, dims, N, K, dtype="i16", v=0.1):
    rng = np.random.default_rng(seed)
    nz, ny, nx = dims[2], dims[1], dims[0]
    if dtype == "f32":
        vals = rng.uniform(-0.3, 0.3, size=(nz, ny, nx)).astype(np.float32)
    else:
        lim = 32767 if dtype == "i16" else 127
        vals = rng.integers(-lim, lim + 1, size=(nz, ny, nx)).astype(np.int16 if dtype == "i16" else np.int8)
    tmap = make_map(vals, v, origin=(-0.2, 0.1, -0.05), tau=0.3, dtype=dtype)
    ext = np.array(dims) * v
    poses = poses_from(random_rotations(rng, N), rng.uniform(0, 1, (N, 3)) * ext)
    pts = rng.normal(0, 0.4 * ext.mean(), size=(3, K)).astype(np.float32)
    return tmap, pts, poses


@pytest.mark.parametrize("N,K", [(1, 1), (1, 63), (63, 1000), (65, 1025), (130, 4097), (7, 9000), (200, 64)])
@pytest.mark.parametrize("dtype", ["i16", "i8", "f32"])
def test_ragged_sizes(torch, mcl, oracle_lib, N, K, dtype):
    say(f"case: trilinear ragged N={N} K={K} dtype={dtype}")
    tmap, pts, poses = random_case(N * 71 + K, (21, 18, 13), N, K, dtype)
    check(torch, mcl, oracle_lib, tmap, pts, poses, f32(0.15), f"N={N} K={K} {dtype}")


def test_smooth_field_is_reproduced(torch, mcl, oracle_lib):
    """An affine field (integers) inside the map: every interpolation step of the
    GPU is exact up to the fma roundings, so the bound is met with room."""
    say("case: trilinear affine field")
    dims = (24, 20, 12)
    nx, ny, nz = dims
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    vals = (200 * i - 150 * j + 300 * k - 1000).astype(np.int16)
    tmap = make_map(vals, 0.125, tau=0.3)
    rng = np.random.default_rng(9)
    N, K = 64, 2048
    poses = poses_from(random_rotations(rng, N) * 0 + np.eye(3), rng.uniform(0.5, 0.8, (N, 3)))
    pts = rng.uniform(-0.4, 0.4, (3, K)).astype(np.float32)
    check(torch, mcl, oracle_lib, tmap, pts, poses, f32(0.2), "affine")


def test_outside_nan_and_empty(torch, mcl, oracle_lib):
    say("case: trilinear outside / NaN / K = 0")
    vals = np.full((4, 4, 4), 1000, np.int16)
    tmap = make_map(vals, 0.125)
    m = mcl.Map.from_tsdf(tmap)
    pts = np.array([[1e4, np.nan, -1e4, 0.25 * 0.125, 0.5 * 0.125, 4.0 * 0.125],
                    [0.0, 0.0, 0.0, 1.5 * 0.125, 1.5 * 0.125, 1.5 * 0.125],
                    [0.0, 0.0, 0.0, 2.5 * 0.125, 2.5 * 0.125, 2.5 * 0.125]], np.float32)
    check(torch, mcl, oracle_lib, tmap, pts, identity_poses(3), f32(0.1), "outside", m)
    lw = mcl.sensor_update_trilinear(m, None, dev(torch, identity_poses(5)), f32(0.1))
    assert np.all(lw.cpu().numpy() == 0.0)


def test_independent_of_batch(torch, mcl):
    """A particle's log-weight has the same bits alone, in a batch, and permuted."""
    say("case: trilinear batch independence")
    tmap, pts, poses = random_case(3, (30, 25, 12), 300, 5000)
    m = mcl.Map.from_tsdf(tmap)
    X, P = dev(torch, pts), dev(torch, poses)
    a = mcl.sensor_update_trilinear(m, X, P, f32(0.2)).cpu().numpy()
    perm = np.random.default_rng(0).permutation(300)
    b = mcl.sensor_update_trilinear(m, X, dev(torch, poses[:, perm]), f32(0.2)).cpu().numpy()
    assert np.array_equal(a[perm], b)
    c = mcl.sensor_update_trilinear(m, X, dev(torch, poses[:, 17:18]), f32(0.2)).cpu().numpy()
    assert c[0] == a[17]


def test_global_workload_sampled(torch, mcl, oracle_lib):
    """The global-localisation workload at full size (N = 10^6): a seeded
    1,024-particle subset against the oracle."""
    w = configs.config2()
    say(f"case: trilinear global full size N={w.N} K={w.K}")
    m = mcl.Map.from_tsdf(w.tmap)
    lw = mcl.sensor_update_trilinear(m, dev(torch, w.points), dev(torch, w.poses), w.sigma)
    torch.cuda.synchronize()
    got = lw.cpu().numpy().astype(np.float64)
    sub = configs.subset_indices(2, w.N, 1024)
    ps = np.ascontiguousarray(w.poses[:, sub])
    ref, S, A = oracle_lib.sensor_update_trilinear(w.tmap, w.points, ps, w.sigma, nthreads=16, return_sums=True)
    bound = 4e-6 + (20 * EPS * 32767.0 * A + 100 * w.K * (EPS * 32767.0) ** 2) / S
    rel = np.abs(got[sub] - ref) / np.abs(ref)
    assert np.all(rel <= bound), f"worst rel {rel.max():.3g}"
    # nearest and trilinear differ, but not wildly, on a real map
    near = mcl.sensor_update(m, dev(torch, w.points), dev(torch, w.poses), w.sigma).cpu().numpy()
    assert np.median(np.abs(near[sub] - got[sub]) / np.abs(near[sub])) < 0.2
