"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars: voxel indices and resampled indices bit-exact; log-weights within 1e-5
relative of the float64 / exact-integer oracle; normalised weights within a few
ulps of the oracle run on the GPU's own log-weights.
"""

import math
import sys

import numpy as np
import pytest

from tests import checks
from tests.helpers import identity_poses, make_map, poses_from, random_rotations, score_const, seed_for_draw
from workloads import configs
from workloads.tsdf import f32

pytestmark = pytest.mark.gpu

RTOL_LOGW = checks.RTOL_LOGW


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


def gpu_logw(torch, mcl, tmap, pts, poses, sigma):
    m = mcl.Map.from_tsdf(tmap)
    lw = mcl.sensor_update(m, dev(torch, pts), dev(torch, poses), sigma)
    torch.cuda.synchronize()
    return lw.cpu().numpy()


assert_logw_close = checks.assert_logw_close


# ------------------------------------------------------------- sensor update
def test_identity_pose_bit_exact(torch, mcl, oracle_lib):
    """Small |q| keeps every float32 partial sum exact: the GPU must reproduce
    -(S * c) bit for bit."""
    say("case: identity pose closed form")
    rng = np.random.default_rng(5)
    nx, ny, nz, v = 12, 10, 9, 0.125
    vals = rng.integers(-64, 65, size=(nz, ny, nx)).astype(np.int16)
    tmap = make_map(vals, v, tau=0.3)
    K = 3000
    ii, jj, kk = rng.integers(0, nx, K), rng.integers(0, ny, K), rng.integers(0, nz, K)
    pts = ((np.stack([ii, jj, kk]).astype(np.float64) + 0.5) * v).astype(np.float32)
    sigma = f32(0.1)
    lw = gpu_logw(torch, mcl, tmap, pts, identity_poses(3), sigma)
    S = sum(int(q) ** 2 for q in vals[kk, jj, ii])
    assert S < 2 ** 24
    c = np.float32(score_const(tmap.dtype, tmap.tau, sigma))
    expect = -(np.float32(S) * c)
    assert np.all(lw == expect)


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
    say(f"case: ragged N={N} K={K} dtype={dtype}")
    tmap, pts, poses = random_case(N * 131 + K, (21, 18, 13), N, K, dtype)
    lw = gpu_logw(torch, mcl, tmap, pts, poses, f32(0.15))
    ref = oracle_lib.sensor_update(tmap, pts, poses, f32(0.15))
    assert_logw_close(lw, ref, f"N={N} K={K} {dtype}")


@pytest.mark.parametrize("block", [(8, 32, 4), (8, 8, 2), (4, 4, 4)])
@pytest.mark.parametrize("dtype", ["i16", "i8", "f32"])
def test_truncated_bricks(torch, mcl, oracle_lib, dtype, block):
    """Maps whose blocks (x, y, z extents; 8 x 32 x 4 is the library's brick) are
    wholly +-Q (mixed signs too), partly Q, or cut by the map edge (dims not
    multiples of the block): the coarse class test must never change a result."""
    say(f"case: truncated bricks {dtype} block={block}")
    rng = np.random.default_rng(17)
    dims = (23, 45, 14)
    tmap, pts, poses = random_case(5, dims, 150, 5000, dtype)
    Q = {"i16": 32767, "i8": 127, "f32": np.float32(0.3)}[dtype]
    vals = tmap.values
    nz, ny, nx = vals.shape
    sx, sy, sz = block
    for bz in range(0, nz, sz):
        for by in range(0, ny, sy):
            for bx in range(0, nx, sx):
                r = rng.random()
                blk = vals[bz:bz + sz, by:by + sy, bx:bx + sx]
                if r < 0.3:
                    blk[...] = Q
                elif r < 0.45:
                    blk[...] = -Q
                elif r < 0.6:
                    blk[...] = np.where(rng.random(blk.shape) < 0.5, Q, -Q)
                elif r < 0.7:
                    blk[...] = Q
                    blk.flat[rng.integers(0, blk.size)] = Q - (1 if dtype != "f32" else np.float32(1e-3))
    lw = gpu_logw(torch, mcl, tmap, pts, poses, f32(0.15))
    ref = oracle_lib.sensor_update(tmap, pts, poses, f32(0.15))
    assert_logw_close(lw, ref, f"truncated bricks {dtype} {block}")


def test_empty_scan(torch, mcl):
    say("case: K=0")
    tmap, pts, poses = random_case(1, (8, 8, 8), 100, 5)
    m = mcl.Map.from_tsdf(tmap)
    lw = mcl.sensor_update(m, None, dev(torch, poses), f32(0.1))
    assert np.all(lw.cpu().numpy() == 0.0)


def test_voxel_indices_bit_exact_random(torch, mcl, oracle_lib):
    say("case: debug indices random")
    tmap, pts, poses = random_case(77, (37, 29, 11), 150, 2000)
    # exact face and special values too
    extra = np.array([[0.0, -0.0, np.nan, np.inf, -np.inf, 1e30, 3.7e-3],
                      [0.0, 0.0, 0.0, 0.0, 0.0, 0.0, -2.5e-2],
                      [0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0]], np.float32)
    pts = np.ascontiguousarray(np.hstack([pts, extra]))
    m = mcl.Map.from_tsdf(tmap)
    got = mcl.debug_voxel_indices(m, dev(torch, pts), dev(torch, poses)).cpu().numpy()
    ref = oracle_lib.voxel_indices(tmap, pts, poses)
    assert np.array_equal(got, ref)
    assert 0.05 < np.mean(ref >= 0) < 0.95


def test_negative_zero_coordinates(torch, mcl, oracle_lib):
    """A pose translation of -0.0 at a zero origin with points of -0.0 selects
    voxel 0, as +0.0 does; a negative coordinate that underflows to -0.0 in the
    fused recipe is outside, its positive mirror inside."""
    say("case: -0.0 coordinates")
    tmap = make_map(np.arange(4 * 4 * 4, dtype=np.int16).reshape(4, 4, 4) * 100, 0.125)
    poses = identity_poses(2)
    poses[9:, 0] = -0.0
    pts = np.array([[-0.0, 0.0, -0.0, 0.0625], [-0.0, 0.0, 0.0, -0.0], [-0.0, -0.0, 0.0, -0.0]], np.float32)
    m = mcl.Map.from_tsdf(tmap)
    got = mcl.debug_voxel_indices(m, dev(torch, pts), dev(torch, poses)).cpu().numpy()
    ref = oracle_lib.voxel_indices(tmap, pts, poses)
    assert np.array_equal(got, ref) and np.all(ref == 0)
    lw = mcl.sensor_update(m, dev(torch, pts), dev(torch, poses), f32(0.1)).cpu().numpy()
    assert np.all(lw == 0.0)
    poses = identity_poses(2)
    poses[2, 0], poses[2, 1] = np.float32(-1e-30), np.float32(1e-30)
    pts = np.array([[0.0], [0.0], [1e-30]], np.float32)
    got = mcl.debug_voxel_indices(m, dev(torch, pts), dev(torch, poses)).cpu().numpy()
    ref = oracle_lib.voxel_indices(tmap, pts, poses)
    assert np.array_equal(got, ref) and ref[0, 0] == -1 and ref[1, 0] == 0


def test_permutation_and_determinism(torch, mcl):
    """Bit-identical results for the same particle whatever its slot, N, run or
    stream (the sums have a fixed order and no atomics)."""
    say("case: determinism")
    tmap, pts, poses = random_case(9, (40, 40, 20), 300, 9000)
    m = mcl.Map.from_tsdf(tmap)
    P = dev(torch, poses)
    X = dev(torch, pts)
    a = mcl.sensor_update(m, X, P, f32(0.2)).cpu().numpy()
    b = mcl.sensor_update(m, X, P, f32(0.2)).cpu().numpy()
    assert np.array_equal(a, b)
    perm = np.random.default_rng(0).permutation(300)
    c = mcl.sensor_update(m, X, dev(torch, poses[:, perm]), f32(0.2)).cpu().numpy()
    assert np.array_equal(c, a[perm])
    d = mcl.sensor_update(m, X, dev(torch, poses[:, 17:18]), f32(0.2)).cpu().numpy()
    assert d[0] == a[17]
    # ten more runs, alternating the default stream and a side stream, and the
    # whole chain (normalise, resample): the same bits every time
    side = torch.cuda.Stream()
    w0, wq0, lz0 = mcl.normalize(dev(torch, a))
    idx0, _ = mcl.resample(wq0, 5, 3, P)
    ref = [x.cpu().numpy() for x in (w0, wq0, lz0, idx0)]
    for r in range(10):
        s = side if r % 2 else torch.cuda.current_stream()
        with torch.cuda.stream(s):
            lw = mcl.sensor_update(m, X, P, f32(0.2), stream=s)
            w, wq, lz = mcl.normalize(lw, stream=s)
            idx, _ = mcl.resample(wq, 5, 3, P, stream=s)
        s.synchronize()
        assert np.array_equal(lw.cpu().numpy().view(np.uint32), a.view(np.uint32)), r
        for x, y in zip((w, wq, lz, idx), ref):
            assert np.array_equal(x.cpu().numpy().view(np.uint8), y.view(np.uint8)), r


# --------------------------------------------------------- workload configs
@pytest.fixture(scope="module")
def cfg1():
    return configs.config1()


def test_config1_full(torch, mcl, oracle_lib, cfg1):
    w = cfg1
    say(f"case: plain-small all particles N={w.N} K={w.K}")
    lw = gpu_logw(torch, mcl, w.tmap, w.points, w.poses, w.sigma)
    ref = oracle_lib.sensor_update(w.tmap, w.points, w.poses, w.sigma)
    assert_logw_close(lw, ref, "config1")
    m = mcl.Map.from_tsdf(w.tmap)
    got = mcl.debug_voxel_indices(m, dev(torch, w.points), dev(torch, w.poses)).cpu().numpy()
    assert np.array_equal(got, oracle_lib.voxel_indices(w.tmap, w.points, w.poses))


def full_chain(torch, mcl, w):
    m = mcl.Map.from_tsdf(w.tmap)
    P = dev(torch, w.poses)
    lw = mcl.sensor_update(m, dev(torch, w.points), P, w.sigma)
    wt, wq, lz = mcl.normalize(lw)
    idx, pout = mcl.resample(wq, w.seed, 0, P)
    torch.cuda.synchronize()
    return (lw.cpu().numpy(), wt.cpu().numpy(), wq.cpu().numpy(), float(lz.cpu().numpy()[0]),
            idx.cpu().numpy(), pout.cpu().numpy())


def check_chain_properties(lw, wq, idx, pout, poses):
    """Properties of the GPU chain's own outputs that hold at any size (no oracle):
    systematic resampling copies particle i floor or ceil of N W_i / T times, in
    non-decreasing order, and the gathered poses are those of the indices."""
    N = lw.shape[0]
    assert np.all(np.diff(idx) >= 0) and idx[0] >= 0 and idx[-1] < N
    cnt = np.bincount(idx, minlength=N)
    W = wq.astype(object)
    T = int(sum(W))
    exp_lo = np.array([(N * int(x)) // T for x in W]) if T else np.ones(N, np.int64)
    assert np.all(cnt >= exp_lo) and np.all(cnt <= exp_lo + 1)
    assert np.array_equal(pout, poses[:, idx])


def check_weight_stages(torch, mcl, oracle_lib, lw32, poses, seed, tick=0):
    """Normalisation and resampling, each fed the same oracle-made input as the
    oracle: log-sum-exp and weights within the bound of
    checks.normalize_bounds, fixed-point weights within one unit plus that
    bound, resampled indices and gathered poses bit-exact."""
    lw32 = np.ascontiguousarray(lw32, np.float32)
    wt, wq, lz = mcl.normalize(dev(torch, lw32))
    wq_ref = checks.check_normalize(oracle_lib, lw32, wq.cpu().numpy(), float(lz.cpu().numpy()[0]),
                                    wt.cpu().numpy(), "normalise")
    idx, pout = mcl.resample(dev(torch, wq_ref), seed, tick, dev(torch, poses))
    checks.check_resample(oracle_lib, wq_ref, seed, tick, idx.cpu().numpy(), poses, pout.cpu().numpy(), "resample")


def test_config1_chain(torch, mcl, oracle_lib, cfg1):
    w = cfg1
    say("case: plain-small chain")
    lw, wt, wq, lz, idx, pout = full_chain(torch, mcl, w)
    ref = oracle_lib.sensor_update(w.tmap, w.points, w.poses, w.sigma)
    assert_logw_close(lw, ref, "config1 chain")
    check_chain_properties(lw, wq, idx, pout, w.poses)
    check_weight_stages(torch, mcl, oracle_lib, ref.astype(np.float32), w.poses, w.seed)


@pytest.fixture(scope="module")
def cfg2():
    return configs.config2()


def test_config2_full_size_sampled(torch, mcl, oracle_lib, cfg2):
    """The global-localisation workload at full size (N = 10^6, the benchmark's
    launch): a seeded 4,096-particle subset of the log-weights against the oracle,
    and the whole normalise + resample chain."""
    w = cfg2
    say(f"case: plain-global full size N={w.N} K={w.K}")
    lw, wt, wq, lz, idx, pout = full_chain(torch, mcl, w)
    sub = configs.subset_indices(2, w.N)
    ref = oracle_lib.sensor_update(w.tmap, w.points, np.ascontiguousarray(w.poses[:, sub]), w.sigma, nthreads=8)
    assert_logw_close(lw[sub], ref, "config2 subset")
    check_chain_properties(lw, wq, idx, pout, w.poses)
    # full-size normalise + resample on oracle-made log-weights: the subset's
    # oracle values drawn with replacement (seeded) to all N particles
    boot = ref[np.random.default_rng(22).integers(0, ref.shape[0], w.N)].astype(np.float32)
    check_weight_stages(torch, mcl, oracle_lib, boot, w.poses, w.seed)
    # voxel indices of 32 sampled particles, bit for bit
    m = mcl.Map.from_tsdf(w.tmap)
    ps = np.ascontiguousarray(w.poses[:, sub[:32]])
    got = mcl.debug_voxel_indices(m, dev(torch, w.points), dev(torch, ps)).cpu().numpy()
    assert np.array_equal(got, oracle_lib.voxel_indices(w.tmap, w.points, ps))


# ------------------------------------------------------------ maximum sizes
def test_max_points(torch, mcl, oracle_lib):
    """K = MCL_MAX_POINTS: 256 pieces of 4096 points per particle, whose partial
    sums the combine kernel adds in its deepest tree; 70 particles (one full
    and one ragged group)."""
    K, N = mcl.MAX_POINTS, 70
    say(f"case: sensor update at K = {K}, N = {N}")
    tmap, pts, poses = random_case(77, (40, 36, 20), N, K, "i16")
    lw = gpu_logw(torch, mcl, tmap, pts, poses, f32(0.15))
    ref = oracle_lib.sensor_update(tmap, pts, poses, f32(0.15), nthreads=8)
    assert_logw_close(lw, ref, "K = MCL_MAX_POINTS")


def test_max_particles(torch, mcl, oracle_lib):
    """N = MCL_MAX_PARTICLES: first with K = 1 against the oracle everywhere,
    then normalisation and resampling of the result; then with K =
    MCL_MAX_POINTS as well (2.2e12 evaluations, 8.4 M work items, a 2 GiB
    partials workspace) against the oracle on sampled particles."""
    N = mcl.MAX_PARTICLES
    say(f"case: sensor update at N = {N}, K = 1")
    tmap, pts1, poses = random_case(78, (40, 36, 20), N, 1, "i16")
    m = mcl.Map.from_tsdf(tmap)
    P = dev(torch, poses)
    lw = mcl.sensor_update(m, dev(torch, pts1), P, f32(0.15)).cpu().numpy()
    ref = oracle_lib.sensor_update(tmap, pts1, poses, f32(0.15), nthreads=8)
    assert_logw_close(lw, ref, "N = MCL_MAX_PARTICLES, K = 1")
    check_weight_stages(torch, mcl, oracle_lib, ref.astype(np.float32), poses, 0x0123456789ABCDEF)
    K = mcl.MAX_POINTS
    say(f"case: sensor update at N = {N}, K = {K}")
    rng = np.random.default_rng(79)
    ext = np.array(tmap.dims) * tmap.voxel
    pts = rng.normal(0, 0.4 * ext.mean(), size=(3, K)).astype(np.float32)
    lw = mcl.sensor_update(m, dev(torch, pts), P, f32(0.15)).cpu().numpy()
    sub = np.r_[0, 1, 63, 64, N // 2, N - 65, N - 64, N - 1, rng.integers(0, N, 16)]
    ref = oracle_lib.sensor_update(tmap, pts, np.ascontiguousarray(poses[:, sub]), f32(0.15), nthreads=8)
    assert_logw_close(lw[sub], ref, "N = MCL_MAX_PARTICLES, K = MCL_MAX_POINTS (sampled)")


def test_dense_map_near_4gib(torch, mcl, oracle_lib):
    """int16 2048 x 2048 x 496 voxels: 4.16 GB of bricks, 97 % of the dense
    layout's 32-bit offset range, so the address sums wrap modulo 2^32 on the
    way to offsets near 2^32.  Values inside the band in the two far corners,
    particles in both (offsets near 0 and near 2^32); parity with the oracle."""
    say("case: dense int16 map of 4.16 GB")
    rng = np.random.default_rng(41)
    nx, ny, nz = 2048, 2048, 496
    vals = np.full((nz, ny, nx), 32767, np.int16)
    vals[-40:, -256:, -256:] = rng.integers(-32767, 32768, (40, 256, 256)).astype(np.int16)
    vals[:40, :256, :256] = rng.integers(-32767, 32768, (40, 256, 256)).astype(np.int16)
    v = 0.05
    tmap = make_map(vals, v, origin=(0.0, 0.0, 0.0), tau=0.15, dtype="i16")
    m = mcl.Map.from_tsdf(tmap)
    assert 4.1e9 < m.device_bytes < 2 ** 32
    N, K = 128, 4096
    lo = np.array([128, 128, 20]) * v
    hi = np.array([nx - 128, ny - 128, nz - 20]) * v
    t = np.where(np.arange(N)[:, None] % 2 == 0, lo, hi) + rng.uniform(-3, 3, (N, 3)) * np.array([1, 1, 0.2])
    poses = poses_from(random_rotations(rng, N), t)
    pts = rng.normal(0, 2.0, (3, K)).astype(np.float32)
    lw = mcl.sensor_update(m, dev(torch, pts), dev(torch, poses), f32(0.075)).cpu().numpy()
    del m
    ref = oracle_lib.sensor_update(tmap, pts, poses, f32(0.075), nthreads=8)
    assert_logw_close(lw, ref, "4.16 GB map")
    assert np.unique(np.round(ref[0::2], 3)).size > N // 4 and np.unique(np.round(ref[1::2], 3)).size > N // 4


# ------------------------------------------------------------ weights edges
def test_normalize_resample_edges(torch, mcl, oracle_lib):
    say("case: weight edge cases")
    rng = np.random.default_rng(3)
    for N in (1, 2, 4095, 4096, 4097, 70001):
        lw = (-np.abs(rng.normal(0, 300, N)) - 1e4).astype(np.float32)
        poses = rng.normal(size=(12, N)).astype(np.float32)
        check_weight_stages(torch, mcl, oracle_lib, lw, poses, 0xDEADBEEF12345678, N)
    # all-zero fixed-point weights: equal weights, identity
    N = 5000
    idx, _ = mcl.resample(dev(torch, np.zeros(N, np.uint64)), 12345, 0)
    assert np.array_equal(idx.cpu().numpy(), np.arange(N))
    # one dominating particle
    lw = np.full(N, -1e5, np.float32)
    lw[4321] = -10.0
    wt, wq, lz = mcl.normalize(dev(torch, lw))
    assert wq.cpu().numpy()[4321] == 2 ** 42 and int(wq.cpu().numpy().sum()) == 2 ** 42
    top = seed_for_draw(oracle_lib, 2 ** 64 - 1, 3)   # the largest offset r = T - 1
    idx, _ = mcl.resample(wq, top, 3)
    assert np.all(idx.cpu().numpy() == 4321)
    # largest N
    N = mcl.MAX_PARTICLES
    wq = dev(torch, np.full(N, 2 ** 21, np.uint64))
    idx, _ = mcl.resample(wq, top, 3)
    assert np.array_equal(idx.cpu().numpy(), np.arange(N))
