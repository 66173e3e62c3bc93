"""Where the nearest lookup reads the map's coarse level (launch config field
`coarse`, through the C ABI): chosen per wave (0), global mask bytes (1) or
bits in LDS (2).  The three must give the same bits (same values, same
summation order), and those bits must meet the float32 bar against the CPU
oracle.  Cases: one and several chunks and pieces, ragged tails, groups
shorter than a wave, all storage types, particles spread over the map and
clustered round one pose (the two regimes the per-wave choice separates), the
full global-localisation workload in both regimes, a map whose bit table is
too large for LDS (every mode falls back to the global bytes), and one whose
table fits LDS only with more waves per workgroup."""

import sys

import numpy as np
import pytest

from tests.helpers import make_map, poses_from, random_rotations
from workloads import configs
from workloads.tsdf import f32

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


def all_modes(mcl, m, X, P, sigma, dtype):
    K, N = X.shape[1], P.shape[1]
    out = []
    try:
        for mode in (0, 1, 2):
            mcl.set_launch_config(dtype, K, N, (4, 0, mode))
            out.append(mcl.sensor_update(m, X, P, sigma).cpu().numpy())
    finally:
        mcl.set_launch_config(dtype, K, N, None)
    return out


def assert_same(outs, what):
    for i, o in enumerate(outs[1:], 1):
        assert np.array_equal(o.view(np.uint32), outs[0].view(np.uint32)), (what, i)


def banded_map(rng, dims, dtype):
    """Random values in a band of slabs, +-Q elsewhere, so that both mixed and
    uniform bricks occur."""
    nx, ny, nz = dims
    Q = {"i16": 32767, "i8": 127, "f32": np.float32(0.3)}[dtype]
    np_t = {"i16": np.int16, "i8": np.int8, "f32": np.float32}[dtype]
    vals = np.where(rng.random((nz, ny, nx)) < 0.5, Q, -Q).astype(np_t)
    for z0 in range(1, nz, 7):
        band = vals[z0:z0 + 2]
        if dtype == "f32":
            band[...] = rng.uniform(-0.3, 0.3, band.shape)
        else:
            band[...] = rng.integers(-Q, Q + 1, band.shape)
    return make_map(vals, 0.1, origin=(-0.3, 0.2, -0.1), tau=0.3, dtype=dtype)


@pytest.mark.parametrize("N,K", [(1, 1), (63, 1000), (65, 4097), (129, 9000)])
@pytest.mark.parametrize("dtype", ["i16", "i8", "f32"])
@pytest.mark.parametrize("clustered", [False, True])
def test_modes_agree(torch, mcl, oracle_lib, N, K, dtype, clustered):
    say(f"case: coarse modes N={N} K={K} {dtype} clustered={clustered}")
    rng = np.random.default_rng(N * 3 + K + clustered)
    dims = (40, 70, 30)
    tmap = banded_map(rng, dims, dtype)
    ext = np.array(dims) * 0.1
    t = ext * 0.5 + rng.normal(0, 0.05, (N, 3)) if clustered else rng.uniform(0, 1, (N, 3)) * ext
    poses = poses_from(random_rotations(rng, N), t)
    pts = rng.normal(0, 0.3 * ext.mean(), (3, K)).astype(np.float32)
    m = mcl.Map.from_tsdf(tmap)
    outs = all_modes(mcl, m, dev(torch, pts), dev(torch, poses), f32(0.15), dtype)
    assert_same(outs, f"N={N} K={K} {dtype}")
    ref = oracle_lib.sensor_update(tmap, pts, poses, f32(0.15))
    assert np.all(np.abs(outs[0] - ref) <= RTOL * np.abs(ref))


@pytest.mark.parametrize("spread", ["global", "tracking"])
def test_modes_agree_global_workload(torch, mcl, spread):
    w = configs.config2()
    say(f"case: coarse modes, warehouse N = 10^6 ({spread})")
    P = w.poses
    if spread == "tracking":
        xyz, rpy = configs.gaussian_particles(np.random.default_rng(11), *w.gt, w.N, s_xyz=0.05, s_rpy_deg=1.0)
        P = configs.poses_soa(xyz, rpy)
    m = mcl.Map.from_tsdf(w.tmap)
    outs = all_modes(mcl, m, dev(torch, w.points), dev(torch, P), w.sigma, "i16")
    assert_same(outs, spread)


def test_bit_table_too_large_for_lds(torch, mcl, oracle_lib):
    """1024 x 2048 x 256 int8 voxels = 524,288 bricks: the bit table (64 KiB +
    4 bytes) exceeds the LDS budget, so every mode reads the global bytes."""
    say("case: coarse modes, map beyond the LDS bit-table budget")
    rng = np.random.default_rng(21)
    dims = (1024, 2048, 256)
    vals = np.full(dims[::-1], 127, np.int8)
    vals[100:140, 900:1000, 400:520] = rng.integers(-127, 128, (40, 100, 120)).astype(np.int8)
    tmap = make_map(vals, 0.05, dtype="i8", tau=0.15)
    N, K = 70, 3000
    lo = np.array([400, 900, 100]) * 0.05
    hi = np.array([520, 1000, 140]) * 0.05
    poses = poses_from(random_rotations(rng, N), rng.uniform(lo, hi, (N, 3)))
    pts = rng.normal(0, 1.0, (3, K)).astype(np.float32)
    m = mcl.Map.from_tsdf(tmap)
    outs = all_modes(mcl, m, dev(torch, pts), dev(torch, poses), f32(0.075), "i8")
    assert_same(outs, "large map")
    ref = oracle_lib.sensor_update(tmap, pts, poses, f32(0.075))
    assert np.all(np.abs(outs[0] - ref) <= RTOL * np.abs(ref))
    assert np.unique(np.round(ref, 3)).size > N // 2


@pytest.mark.parametrize("wpb", [2, 4, 8])
def test_large_bit_table_in_lds(torch, mcl, oracle_lib, wpb):
    """1024 x 2048 x 128 int8 voxels = 262,144 bricks: a 32 KiB bit table, which
    fits LDS but at 2 or 4 waves per workgroup would leave too few waves per
    compute unit, so the launch raises its waves per workgroup.  Every shape
    and mode gives the same bits, within the bar of the oracle."""
    say(f"case: coarse modes, 32 KiB bit table, {wpb} waves per workgroup")
    rng = np.random.default_rng(23)
    dims = (1024, 2048, 128)
    vals = np.full(dims[::-1], 127, np.int8)
    vals[40:80, 900:1000, 400:520] = rng.integers(-127, 128, (40, 100, 120)).astype(np.int8)
    tmap = make_map(vals, 0.05, dtype="i8", tau=0.15)
    N, K = 130, 5000
    lo = np.array([400, 900, 40]) * 0.05
    hi = np.array([520, 1000, 80]) * 0.05
    poses = poses_from(random_rotations(rng, N), rng.uniform(lo, hi, (N, 3)))
    pts = rng.normal(0, 1.0, (3, K)).astype(np.float32)
    m = mcl.Map.from_tsdf(tmap)
    X, P = dev(torch, pts), dev(torch, poses)
    outs = []
    try:
        for mode in (0, 1, 2):
            mcl.set_launch_config("i8", K, N, (wpb, 0, mode))
            outs.append(mcl.sensor_update(m, X, P, f32(0.075)).cpu().numpy())
    finally:
        mcl.set_launch_config("i8", K, N, None)
    assert_same(outs, f"32 KiB table, {wpb} waves")
    ref = oracle_lib.sensor_update(tmap, pts, poses, f32(0.075))
    assert np.all(np.abs(outs[0] - ref) <= RTOL * np.abs(ref))
    assert np.unique(np.round(ref, 3)).size > N // 2


def test_tick_on_one_map_modes_agree(torch, mcl):
    """A batched tick whose filters share one map holds that map's read bits in
    LDS; clustered and spread filters, every coarse mode, and the single-filter
    calls give the same bits."""
    say("case: coarse modes in a batched tick on one map")
    rng = np.random.default_rng(5)
    dims = (40, 70, 30)
    tmap = banded_map(rng, dims, "i16")
    m = mcl.Map.from_tsdf(tmap)
    ext = np.array(dims) * 0.1
    filters = []
    for i, (N, K) in enumerate([(3000, 5000), (700, 1500), (64, 9000), (5, 4096)]):
        t = ext * 0.5 + rng.normal(0, 0.05, (N, 3)) if i % 2 else rng.uniform(0, 1, (N, 3)) * ext
        poses = poses_from(random_rotations(rng, N), t)
        pts = rng.normal(0, 0.3 * ext.mean(), (3, K)).astype(np.float32)
        filters.append(mcl.Filter(m, dev(torch, pts), dev(torch, poses), f32(0.15), int(rng.integers(0, 2 ** 63))))
    singles = [mcl.sensor_update(m, f.points, f.poses, f.sigma).cpu().numpy() for f in filters]
    try:
        for mode in (0, 1, 2):
            mcl.set_launch_config("i16", 5000, 3000, (4, 0, mode))
            mcl.tick(filters)
            torch.cuda.synchronize()
            for i, f in enumerate(filters):
                got = f.logw.cpu().numpy()
                assert np.array_equal(got.view(np.uint32), singles[i].view(np.uint32)), (mode, i)
    finally:
        mcl.set_launch_config("i16", 5000, 3000, None)


def test_tick_graph_replay_follows_the_map(torch, mcl):
    """A graph captured for a tick on map A replays for the same sizes on map B
    (same dimensions, other values): the LDS read bits must be B's.  Every
    replay is checked against the single-filter calls, with eager work between
    the replays."""
    say("case: tick graph replay across maps of one size")
    rng = np.random.default_rng(9)
    dims = (40, 70, 30)
    maps = []
    for k in range(2):
        tmap = banded_map(rng, dims, "i16")
        if k == 1:  # flip which slabs hold band values
            tmap.values[...] = np.roll(tmap.values, 3, axis=0)
        maps.append(mcl.Map.from_tsdf(tmap))
    ext = np.array(dims) * 0.1
    s = torch.cuda.Stream()
    for rep, mi in enumerate((0, 1, 0, 1)):
        filters = []
        for i, (N, K) in enumerate([(2000, 3000), (300, 5000)]):
            t = ext * 0.5 + rng.normal(0, 0.05, (N, 3)) if i else rng.uniform(0, 1, (N, 3)) * ext
            poses = poses_from(random_rotations(rng, N), t)
            pts = rng.normal(0, 0.3 * ext.mean(), (3, K)).astype(np.float32)
            filters.append(mcl.Filter(maps[mi], dev(torch, pts), dev(torch, poses), f32(0.15),
                                      int(rng.integers(0, 2 ** 63))))
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            mcl.tick(filters, graph=True, stream=s)
        s.synchronize()
        got = [f.logw.cpu().numpy() for f in filters]
        _ = torch.ones(1 << 20, device="cuda").sum().item()
        for i, f in enumerate(filters):
            ref = mcl.sensor_update(f.map, f.points, f.poses, f.sigma).cpu().numpy()
            assert np.array_equal(got[i].view(np.uint32), ref.view(np.uint32)), (rep, i)
