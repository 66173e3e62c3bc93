"""Parity of the sparse coarse/fine map (mcl_map_upload_bricks + mcl_sensor_update,
through the C ABI) with the CPU oracle, and bit-identity with the dense layout
holding the same values (same index recipe, values and summation order)."""

import sys

import numpy as np
import pytest

from tests.helpers import make_map, poses_from, random_rotations
from workloads import configs
from workloads.tsdf import f32, to_bricks

pytestmark = pytest.mark.gpu
RTOL = 1e-5


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


def sparse_of(mcl, tmap, coords, values):
    return mcl.Map.from_bricks(tmap.dims, tmap.voxel, tmap.origin, tmap.tau, tmap.dtype, coords, values)


def assert_bits(got, ref, what):
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), what


def case(seed, dims, dtype, N, K):
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    Q = {"i16": 32767, "i8": 127, "f32": np.float32(0.3)}[dtype]
    if dtype == "f32":
        vals = rng.uniform(-0.3, 0.3, (nz, ny, nx)).astype(np.float32)
    else:
        vals = rng.integers(-Q, Q + 1, (nz, ny, nx)).astype(np.int16 if dtype == "i16" else np.int8)
    m = rng.random(((nz + 3) // 4, (ny + 3) // 4, (nx + 3) // 4)) < 0.6
    sgn = np.where(rng.random(m.shape) < 0.5, Q, -Q)
    for bz, by, bx in zip(*np.nonzero(m)):
        vals[4 * bz:4 * bz + 4, 4 * by:4 * by + 4, 4 * bx:4 * bx + 4] = sgn[bz, by, bx]
    tmap = make_map(vals, 0.1, origin=(-0.3, 0.2, -0.1), tau=0.3, dtype=dtype)
    ext = np.array(dims) * 0.1
    poses = poses_from(random_rotations(rng, N), rng.uniform(0, 1, (N, 3)) * ext)
    pts = rng.normal(0, 0.4 * ext.mean(), (3, K)).astype(np.float32)
    return tmap, pts, poses


@pytest.mark.parametrize("N,K", [(1, 1), (63, 1000), (65, 4097), (7, 9000)])
@pytest.mark.parametrize("dtype", ["i16", "i8", "f32"])
def test_sparse_matches_oracle_and_dense(torch, mcl, oracle_lib, N, K, dtype):
    say(f"case: sparse N={N} K={K} {dtype}")
    tmap, pts, poses = case(N + K, (23, 18, 13), dtype, N, K)
    co, va = to_bricks(tmap)
    sm = sparse_of(mcl, tmap, co, va)
    dm = mcl.Map.from_tsdf(tmap)
    X, P = dev(torch, pts), dev(torch, poses)
    ld = mcl.sensor_update(dm, X, P, f32(0.15)).cpu().numpy()
    ls = mcl.sensor_update(sm, X, P, f32(0.15)).cpu().numpy()
    assert_bits(ls, ld, "sparse vs dense")
    ref = oracle_lib.sensor_update_bricks(tmap.dims, tmap.voxel, tmap.origin, tmap.tau, dtype, co, va, pts, poses,
                                          f32(0.15))
    assert np.all(np.abs(ls - ref) <= RTOL * np.abs(ref))


def banded_case(seed, dims, dtype, N, K, clustered):
    """Values inside the band only in thin z slabs and one x half, +-Q
    elsewhere: many blocks are not stored, so the offset table mixes stored
    and unstored entries along every axis."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    Q = {"i16": 32767, "i8": 127, "f32": np.float32(0.3)}[dtype]
    np_t = {"i16": np.int16, "i8": np.int8, "f32": np.float32}[dtype]
    vals = np.where(rng.random((nz, ny, nx)) < 0.5, Q, -Q).astype(np_t)
    for z0 in range(2, nz, 11):
        band = vals[z0:z0 + 2, :, : nx // 2]
        if dtype == "f32":
            band[...] = rng.uniform(-0.3, 0.3, band.shape)
        else:
            band[...] = rng.integers(-Q, Q + 1, band.shape)
    tmap = make_map(vals, 0.1, origin=(-0.3, 0.2, -0.1), tau=0.3, dtype=dtype)
    ext = np.array(dims) * 0.1
    if clustered:
        c = rng.uniform(0.3, 0.7, 3) * ext
        t = c + rng.normal(0, 0.05, (N, 3))
        rot = random_rotations(rng, 1)
        poses = poses_from(np.repeat(rot, N, axis=0), t)
    else:
        poses = poses_from(random_rotations(rng, N), rng.uniform(0, 1, (N, 3)) * ext)
    pts = rng.normal(0, 0.3 * ext.mean(), (3, K)).astype(np.float32)
    return tmap, pts, poses


@pytest.mark.parametrize("N,K", [(65, 4097), (200, 9000)])
@pytest.mark.parametrize("dtype", ["i16", "i8", "f32"])
@pytest.mark.parametrize("clustered", [False, True])
def test_stored_blocks_with_gaps(torch, mcl, oracle_lib, N, K, dtype, clustered):
    say(f"case: sparse banded N={N} K={K} {dtype} clustered={clustered}")
    tmap, pts, poses = banded_case(7 * N + K, (203, 150, 45), dtype, N, K, clustered)
    co, va = to_bricks(tmap)
    sm = sparse_of(mcl, tmap, co, va)
    dm = mcl.Map.from_tsdf(tmap)
    X, P = dev(torch, pts), dev(torch, poses)
    ld = mcl.sensor_update(dm, X, P, f32(0.15)).cpu().numpy()
    assert_bits(mcl.sensor_update(sm, X, P, f32(0.15)).cpu().numpy(), ld, "banded sparse vs dense")
    ref = oracle_lib.sensor_update_bricks(tmap.dims, tmap.voxel, tmap.origin, tmap.tau, dtype, co, va, pts, poses,
                                          f32(0.15))
    assert np.all(np.abs(ld - ref) <= RTOL * np.abs(ref))


def test_empty_listing_reads_q(torch, mcl, oracle_lib):
    say("case: sparse map without bricks")
    tmap, pts, poses = case(5, (12, 12, 12), "i16", 40, 2000)
    sm = sparse_of(mcl, tmap, np.zeros((0, 3), np.int32), np.zeros((0, 64), np.int16))
    ls = mcl.sensor_update(sm, dev(torch, pts), dev(torch, poses), f32(0.2)).cpu().numpy()
    ref = oracle_lib.sensor_update_bricks(tmap.dims, tmap.voxel, tmap.origin, tmap.tau, "i16",
                                          np.zeros((0, 3), np.int32), np.zeros((0, 64), np.int16), pts, poses, f32(0.2))
    assert np.all(np.abs(ls - ref) <= RTOL * np.abs(ref))


def test_map_beyond_the_dense_limit(torch, mcl, oracle_lib):
    """A 4096 x 4096 x 192 int16 grid (6.4 GB dense, past the 4 GiB dense layout
    limit) with band bricks only in a region: parity on particles around it."""
    say("case: sparse map beyond 4 GiB dense")
    rng = np.random.default_rng(9)
    dims = (4096, 4096, 192)
    bx, by, bz = np.meshgrid(np.arange(600, 640), np.arange(900, 930), np.arange(8, 20), indexing="ij")
    co = np.stack([bx.ravel(), by.ravel(), bz.ravel()], 1).astype(np.int32)
    va = rng.integers(-32767, 32768, (co.shape[0], 64)).astype(np.int16)
    v = 0.05
    lo = np.array([600 * 4, 900 * 4, 8 * 4]) * v
    hi = np.array([640 * 4, 930 * 4, 20 * 4]) * v
    N, K = 200, 6000
    poses = poses_from(random_rotations(rng, N), rng.uniform(lo, hi, (N, 3)))
    pts = rng.normal(0, 1.5, (3, K)).astype(np.float32)
    sm = mcl.Map.from_bricks(dims, f32(v), (0.0, 0.0, 0.0), f32(0.15), "i16", co, va)
    ls = mcl.sensor_update(sm, dev(torch, pts), dev(torch, poses), f32(0.075)).cpu().numpy()
    ref = oracle_lib.sensor_update_bricks(dims, f32(v), (0.0, 0.0, 0.0), f32(0.15), "i16", co, va, pts, poses,
                                          f32(0.075), nthreads=8)
    assert np.all(np.abs(ls - ref) <= RTOL * np.abs(ref))
    assert np.unique(np.round(ref, 3)).size > N // 2     # the region is actually read


def test_pool_past_4gib(torch, mcl, oracle_lib):
    """float32 blocks of 8 x 32 x 4 voxels take 4 KiB each, so 1.2 M stored
    blocks make a pool past 4 GiB: the table then holds slot numbers and the
    lookup forms 64-bit addresses.  One brick listed per block for y < 120 m,
    every brick of a region round the particles; parity with the oracle."""
    say("case: sparse pool past 4 GiB (float32, 1.2 M stored blocks)")
    rng = np.random.default_rng(31)
    dims = (4096, 4096, 128)
    nbx, nby, nbz = 1024, 1024, 32
    listed = np.zeros((nbz, nby, nbx), bool)
    listed[:, 0:600:8, 0::2] = True           # the first brick of every block with block y < 75
    listed[4:20, 400:440, 800:840] = True     # all bricks of the region
    bz, by, bx = np.nonzero(listed)
    co = np.stack([bx, by, bz], 1).astype(np.int32)
    del listed
    tau = f32(0.15)
    va = rng.uniform(-0.15, 0.15, (co.shape[0], 64)).astype(np.float32)
    v = f32(0.05)
    sm = mcl.Map.from_bricks(dims, v, (0.0, 0.0, 0.0), tau, "f32", co, va)
    say(f"stored bricks {co.shape[0]}, device bytes {sm.device_bytes}")
    assert sm.device_bytes > 2 ** 32
    lo = np.array([800 * 4, 400 * 4, 4 * 4]) * v
    hi = np.array([840 * 4, 440 * 4, 20 * 4]) * v
    N, K = 130, 3000
    poses = poses_from(random_rotations(rng, N), rng.uniform(lo, hi, (N, 3)))
    pts = rng.normal(0, 1.5, (3, K)).astype(np.float32)
    ls = mcl.sensor_update(sm, dev(torch, pts), dev(torch, poses), f32(0.075)).cpu().numpy()
    with pytest.raises(mcl.MclError):   # a batched tick takes sparse maps below 4 GiB only
        mcl.tick([mcl.Filter(sm, dev(torch, pts), dev(torch, poses), f32(0.075), 1)])
    del sm
    ref = oracle_lib.sensor_update_bricks(dims, v, (0.0, 0.0, 0.0), tau, "f32", co, va, pts, poses, f32(0.075),
                                          nthreads=8)
    assert np.all(np.abs(ls - ref) <= RTOL * np.abs(ref))
    assert np.unique(np.round(ref, 3)).size > N // 2


def test_global_workload_sparse_equals_dense(torch, mcl):
    w = configs.config2()
    say("case: sparse warehouse map, N = 10^6")
    co, va = to_bricks(w.tmap)
    sm = sparse_of(mcl, w.tmap, co, va)
    dm = mcl.Map.from_tsdf(w.tmap)
    X, P = dev(torch, w.points), dev(torch, w.poses)
    ld = mcl.sensor_update(dm, X, P, w.sigma).cpu().numpy()
    assert_bits(mcl.sensor_update(sm, X, P, w.sigma).cpu().numpy(), ld, "global workload")
    # particles converged round the true pose (most points in the band)
    xyz, rpy = configs.gaussian_particles(np.random.default_rng(4), *w.gt, w.N, s_xyz=0.05, s_rpy_deg=1.0)
    Pc = dev(torch, configs.poses_soa(xyz, rpy))
    ldc = mcl.sensor_update(dm, X, Pc, w.sigma).cpu().numpy()
    assert_bits(mcl.sensor_update(sm, X, Pc, w.sigma).cpu().numpy(), ldc, "global workload, converged")
    nb = ((w.tmap.nx + 3) // 4) * ((w.tmap.ny + 3) // 4) * ((w.tmap.nz + 3) // 4)
    say(f"stored bricks {co.shape[0]} of {nb} ({co.shape[0] / nb:.1%}); device bytes sparse {sm.device_bytes}, "
        f"dense {dm.device_bytes}")
    # listed values (2 B each) <= sparse footprint < dense footprint
    assert co.shape[0] * 64 * 2 <= sm.device_bytes < dm.device_bytes // 2


def test_sparse_guards(torch, mcl):
    tmap, pts, poses = case(6, (8, 8, 8), "i16", 4, 10)
    co, va = to_bricks(tmap)
    sm = sparse_of(mcl, tmap, co, va)
    P = dev(torch, poses)
    with pytest.raises(mcl.MclError):
        mcl.sensor_update_trilinear(sm, dev(torch, pts), P, f32(0.1))
    with pytest.raises(mcl.MclError):
        mcl.init_uniform(sm, 10, 0.0, 1)
    with pytest.raises(mcl.MclError):   # a brick listed twice
        sparse_of(mcl, tmap, np.r_[co[:1], co[:1]], np.r_[va[:1], va[:1]])
    with pytest.raises(mcl.MclError):   # outside the brick grid
        sparse_of(mcl, tmap, np.array([[2, 0, 0]], np.int32), va[:1])
