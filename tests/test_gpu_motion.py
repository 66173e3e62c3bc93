"""Parity of the motion update, the uniform initialisation and the random
numbers (through the C ABI) with the CPU oracle.

Bars: Philox words bit-exact (known answers and random counters); the initial
positions bit-exact (their float32 steps are fixed; they also fix the chosen
voxel); rotations and moved poses within bounds derived from float32
arithmetic against the float64 oracle fed the same random words:
  * a normal from Box-Muller in float32 is within 2e-6 (1 + r) of the exact one
    (logf, sqrtf, sincosf within a few ulps; the angle 2 pi u carries one
    rounding of pi and one of the product), r <= sqrt(2 ln 2^24) < 5.8;
  * a noise vector sigma n is then within sigma * 1.4e-5;
  * float32 products of 3x3 matrices with entries <= 1 add a few 1e-7;
so rotation entries agree within 2e-6 + 3e-5 sigma_r, and translations within
2e-6 (1 + |t| + |dt|) + 3e-5 sigma_t.
"""

import math
import sys

import numpy as np
import pytest

from tests.helpers import make_map, poses_from, random_rotations
from workloads import configs

pytestmark = pytest.mark.gpu


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


def test_philox_matches(torch, mcl, oracle_lib):
    say("case: philox")
    rng = np.random.default_rng(1)
    cases = [([0, 0, 0, 0], [0, 0]), ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2),
             ([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344], [0xa4093822, 0x299f31d0])]
    cases += [(list(rng.integers(0, 2 ** 32, 4)), list(rng.integers(0, 2 ** 32, 2))) for _ in range(50)]
    for c, k in cases:
        assert np.array_equal(mcl.debug_philox(c, k), oracle_lib.philox4x32(c, k)), (c, k)


def motion_case(seed, N):
    rng = np.random.default_rng(seed)
    P = poses_from(random_rotations(rng, N), rng.normal(0, 20, (N, 3)))
    dR = random_rotations(rng, 1)[0] if seed % 2 else np.eye(3)
    dt = rng.normal(0, 0.5, 3)
    delta = np.r_[dR.ravel(), dt].astype(np.float32)
    return P, delta


def check_motion(got, ref, P, delta, st, sr, what):
    tol_r = 2e-6 + 3e-5 * sr
    err_r = np.abs(got[:9] - ref[:9]).max()
    assert err_r <= tol_r, (what, err_r, tol_r)
    tol_t = 2e-6 * (1 + np.abs(P[9:]).max(axis=0) + np.abs(delta[9:]).max()) + 3e-5 * st
    err_t = np.abs(got[9:] - ref[9:]).max(axis=0)
    assert np.all(err_t <= tol_t), (what, err_t.max())


@pytest.mark.parametrize("N", [1, 255, 1000, 65537])
@pytest.mark.parametrize("st,sr", [(0.0, 0.0), (0.1, 0.1), (0.02, 0.5)])
def test_motion_update(torch, mcl, oracle_lib, N, st, sr):
    say(f"case: motion N={N} sigma=({st}, {sr})")
    P, delta = motion_case(N + int(st * 100), N)
    seed, step = 0xABCDEF0123, 17
    got = mcl.motion_update(dev(torch, P), delta, st, sr, seed, step).cpu().numpy()
    ref = oracle_lib.motion_update(P, delta, st, sr, seed, step)
    check_motion(got, ref, P, delta, st, sr, f"N={N}")


@pytest.mark.parametrize("N", [1, 1000, 65537])
@pytest.mark.parametrize("st,sr", [(0.0, 0.0), (0.5, 0.087)])
def test_init_gaussian(torch, mcl, oracle_lib, N, st, sr):
    """Initialisation round a pose estimate: bit for bit the motion update of N
    copies of the estimate by the identity increment, and within the motion
    bounds of the oracle's motion update of those copies."""
    say(f"case: init round a pose N={N} sigma=({st}, {sr})")
    rng = np.random.default_rng(N)
    mean = poses_from(random_rotations(rng, 1), rng.normal(0, 20, (1, 3)))[:, 0]
    seed, step = 0x5EED, 1
    got = mcl.init_gaussian(mean, N, st, sr, seed, step).cpu().numpy()
    copies = np.ascontiguousarray(np.repeat(mean[:, None], N, axis=1))
    ident = np.r_[np.eye(3).ravel(), 0.0, 0.0, 0.0].astype(np.float32)
    moved = mcl.motion_update(dev(torch, copies), ident, st, sr, seed, step).cpu().numpy()
    assert np.array_equal(got.view(np.uint32), moved.view(np.uint32))
    ref = oracle_lib.motion_update(copies, ident, st, sr, seed, step)
    check_motion(got, ref, copies, ident, st, sr, f"init N={N}")
    if st > 0 and N > 1000:
        # the spread is the requested one (0.5 m per axis, in the estimate's frame)
        d = (mean[:9].reshape(3, 3).astype(np.float64).T @ (got[9:] - mean[9:, None]).astype(np.float64))
        assert np.all(np.abs(d.std(axis=1) / st - 1.0) < 0.02), d.std(axis=1)


def test_motion_in_place_and_determinism(torch, mcl):
    say("case: motion in place")
    P, delta = motion_case(3, 5000)
    a = mcl.motion_update(dev(torch, P), delta, 0.1, 0.1, 5, 9).cpu().numpy()
    X = dev(torch, P)
    mcl.motion_update(X, delta, 0.1, 0.1, 5, 9, poses_out=X)
    assert np.array_equal(X.cpu().numpy(), a)
    b = mcl.motion_update(dev(torch, P), delta, 0.1, 0.1, 5, 10).cpu().numpy()
    assert not np.array_equal(a, b)
    # a particle's draw does not depend on N
    c = mcl.motion_update(dev(torch, P[:, :100]), delta, 0.1, 0.1, 5, 9).cpu().numpy()
    assert np.array_equal(c, a[:, :100])


def free_map(seed, dims, frac, dtype):
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    free = rng.random((nz, ny, nx)) < frac
    if dtype == "f32":
        vals = np.where(free, 0.2, -0.1).astype(np.float32)
    else:
        vals = np.where(free, 100, -100).astype(np.int16 if dtype == "i16" else np.int8)
    return make_map(vals, 0.125, origin=(-0.5, 0.25, 1.0), dtype=dtype)


def check_init(got, ref, what):
    assert np.array_equal(got[9:].view(np.uint32), ref[9:].astype(np.float32).view(np.uint32)), what
    err = np.abs(got[:9] - ref[:9]).max()
    assert err <= 2e-6, (what, err)


@pytest.mark.parametrize("dtype", ["i16", "i8", "f32"])
@pytest.mark.parametrize("dims,frac", [((7, 5, 4), 0.3), ((130, 70, 9), 0.6), ((64, 64, 64), 0.001)])
def test_init_uniform(torch, mcl, oracle_lib, dtype, dims, frac):
    say(f"case: init {dtype} dims={dims} frac={frac}")
    tmap = free_map(sum(dims), dims, frac, dtype)
    m = mcl.Map.from_tsdf(tmap)
    N = 4097
    seed = 0x5EED_0000_1111
    got = mcl.init_uniform(m, N, 0.3, seed).cpu().numpy()
    ref, _ = oracle_lib.init_uniform(tmap, N, 0.3, seed)
    check_init(got, ref, f"{dtype} {dims}")


def test_init_edge_maps(torch, mcl, oracle_lib):
    say("case: init edge maps")
    one = np.full((3, 4, 5), -7, np.int16)
    one[2, 3, 4] = 1                         # the last voxel is the only free one
    tmap = make_map(one, 0.2, origin=(1.0, 2.0, 3.0))
    m = mcl.Map.from_tsdf(tmap)
    got = mcl.init_uniform(m, 1000, 0.0, 3).cpu().numpy()
    ref, vox = oracle_lib.init_uniform(tmap, 1000, 0.0, 3)
    assert np.all(vox == one.size - 1)
    check_init(got, ref, "one free voxel")
    none = make_map(np.full((3, 3, 3), -1, np.int16), 0.1)
    mn = mcl.Map.from_tsdf(none)
    with pytest.raises(mcl.MclError):
        mcl.init_uniform(mn, 10, 0.0, 1)


def test_init_global_workload_map(torch, mcl, oracle_lib):
    """The warehouse map of the global-localisation workload, N = 10^6."""
    w = configs.config2()
    say("case: init on the warehouse map, N = 10^6")
    m = mcl.Map.from_tsdf(w.tmap)
    N = 1_000_000
    got = mcl.init_uniform(m, N, 0.05, 2024).cpu().numpy()
    ref, _ = oracle_lib.init_uniform(w.tmap, N, 0.05, 2024)
    check_init(got, ref, "warehouse")


def test_full_loop_runs(torch, mcl):
    """init -> sensor -> normalise -> estimate -> resample -> motion, twice, all on
    the device: shapes and finiteness (the parts are checked one by one above)."""
    w = configs.config1()
    m = mcl.Map.from_tsdf(w.tmap)
    P = mcl.init_uniform(m, 20000, 0.05, 1)
    X = dev(torch, w.points)
    for step in range(2):
        lw = mcl.sensor_update(m, X, P, w.sigma)
        wt, wq, _ = mcl.normalize(lw)
        mean, bi, _ = mcl.pose_estimate(wt, P)
        _, P2 = mcl.resample(wq, 12345, step, P)
        P = mcl.motion_update(P2, np.r_[np.eye(3).ravel(), 0.1, 0, 0], 0.02, 0.01, 7, step)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(P.cpu().numpy())) and np.all(np.isfinite(mean.cpu().numpy()))
