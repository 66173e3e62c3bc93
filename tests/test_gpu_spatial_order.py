"""The spatial order of the sensor update (mcl_set_spatial_order_min), through the C ABI.

A dense-map filter large enough is counting-sorted by the x-y cell of its
particles before the lookups, and each particle's result is written back to its
own index.  The contract: every output is bit-identical with and without the
order (single calls, both readings, one and several pieces, the batched tick
eagerly and from a graph), and the ordered results follow the oracle.  Cases
cover one crowded cell (every particle in it), particles outside the map and
NaN positions, ragged counting blocks, and the global-localisation workload at
full size with the default threshold.
"""

import sys

import numpy as np
import pytest

from tests import checks
from tests.helpers import make_map, poses_from, random_rotations
from workloads import configs
from workloads.tsdf import f32

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


@pytest.fixture
def order_min(mcl):
    """Sets the threshold for one test and restores it afterwards."""
    prev = mcl.get_spatial_order_min()
    yield mcl.set_spatial_order_min
    mcl.set_spatial_order_min(prev)


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def case(seed, dims, N, K, dtype, layout, v=0.1, tau=0.3):
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    if dtype == "f32":
        vals = rng.uniform(-tau, tau, size=(nz, ny, nx)).astype(np.float32)
        vals[:, :, : nx // 3] = np.float32(tau)
    else:
        lim = 32767 if dtype == "i16" else 127
        vals = rng.integers(-lim, lim + 1, size=(nz, ny, nx)).astype(np.int16 if dtype == "i16" else np.int8)
        vals[:, :, : nx // 3] = lim
    tmap = make_map(vals, v, origin=(-0.2, 0.1, -0.05), tau=tau, dtype=dtype)
    ext = np.array(dims) * v
    origin = np.array(tmap.origin, np.float64)
    if layout == "cluster":      # every particle in one cell of the order
        t = origin + ext * 0.5 + rng.uniform(-0.2, 0.2, (N, 3)) * v
    else:
        t = origin + rng.uniform(0, 1, (N, 3)) * ext
    if layout == "edges":        # outside the map on either side, and NaN positions
        t[0::7, 0] = origin[0] - 3.0 * ext[0]
        t[1::7, 1] = origin[1] + 5.0 * ext[1]
        t[2::11, :2] = np.nan
    poses = poses_from(random_rotations(rng, N), t)
    pts = rng.normal(0, 0.4 * ext.mean(), size=(3, K)).astype(np.float32)
    return tmap, pts, poses


def bits(x):
    return np.ascontiguousarray(x).view(np.uint32)


CASES = [
    (5000, 9000, "i16", "uniform"),   # two counting blocks (one ragged), three pieces: the combine writes back
    (3000, 3000, "i8", "cluster"),    # one cell holds all, one piece: the sensor kernel writes back
    (4096, 4097, "f32", "uniform"),   # exactly one counting block, a ragged second piece
    (777, 1025, "i16", "edges"),      # particles outside the map and at NaN positions
    (1, 5000, "i16", "uniform"),      # one particle: one counting block of one, a 63-lane empty group
    (65, 300, "i8", "edges"),         # a full and a one-particle group, one short piece
]


@pytest.mark.parametrize("N,K,dtype,layout", CASES)
def test_single_calls_ordered_equal_unordered(torch, mcl, oracle_lib, order_min, N, K, dtype, layout):
    say(f"case: spatial order, single calls, N={N} K={K} {dtype} {layout}")
    tmap, pts, poses = case(N + K, (48, 40, 16), N, K, dtype, layout)
    m = mcl.Map.from_tsdf(tmap)
    X, P = dev(torch, pts), dev(torch, poses)
    sigma = f32(0.15)
    out = {}
    for name, thr in (("ordered", 0), ("unordered", -1)):
        order_min(thr)
        lw = mcl.sensor_update(m, X, P, sigma).cpu().numpy()
        ls = mcl.sensor_update_sum(m, X, P, sigma).cpu().numpy()
        out[name] = (lw, ls)
    for a, b, what in zip(out["ordered"], out["unordered"], ("product", "sum")):
        assert np.array_equal(bits(a), bits(b)), f"{what} reading: ordered and unordered results differ"
    fin = np.flatnonzero(np.isfinite(poses).all(axis=0))
    sub = fin if fin.size <= 600 else np.sort(np.random.default_rng(N).choice(fin, 600, replace=False))
    ps = np.ascontiguousarray(poses[:, sub])
    ref = oracle_lib.sensor_update(tmap, pts, ps, sigma, nthreads=8)
    checks.assert_logw_close(out["ordered"][0][sub], ref, f"ordered product reading N={N} K={K}")
    ref_s = oracle_lib.sensor_update_sum(tmap, pts, ps, sigma, nthreads=8)
    err = np.abs(out["ordered"][1][sub].astype(np.float64) - ref_s)
    assert np.all(err <= checks.sum_logw_tol(tmap.tau, sigma, ref_s)), "ordered sum reading off the oracle"


def test_no_alloc_call_equals_ordered(torch, mcl, order_min):
    """The no-allocation call never orders; the ordered call gives its bits."""
    say("case: spatial order vs the no-allocation call")
    tmap, pts, poses = case(31, (48, 40, 16), 2000, 5000, "i16", "uniform")
    m = mcl.Map.from_tsdf(tmap)
    X, P = dev(torch, pts), dev(torch, poses)
    order_min(0)
    a = mcl.sensor_update(m, X, P, f32(0.15)).cpu().numpy()
    lw = torch.empty(2000, dtype=torch.float32, device="cuda")
    mcl.sensor_update_noalloc(m, X, P, f32(0.15), lw)
    assert np.array_equal(bits(a), bits(lw.cpu().numpy()))


def tick_outputs(torch, mcl, maps, specs, seed, graph, stream):
    rng = np.random.default_rng(seed)
    filters = []
    for mi, N, K, layout in specs:
        tmap, m = maps[mi]
        _, pts, poses = case(int(rng.integers(0, 1 << 30)), tmap.dims, N, K, tmap.dtype, layout)
        filters.append(mcl.Filter(m, dev(torch, pts), dev(torch, poses), f32(0.12), int(rng.integers(0, 2 ** 63)),
                                  want_estimate=len(filters) % 2 == 0))
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        mcl.tick(filters, graph=graph, stream=stream)
    stream.synchronize()
    res = []
    for f in filters:
        est = (f.est_mean, f.est_idx, f.est_pose) if f.est_mean is not None else ()
        res.append([x.cpu().numpy() for x in (f.logw, f.w, f.wq, f.log_z, f.idx, f.poses_out, *est)])
    return res


def test_tick_ordered_equal_unordered(torch, mcl, order_min):
    """A tick whose filters are partly ordered (threshold between their sizes),
    all ordered, and none: the same bits for every output of every filter,
    eagerly and replayed from graphs (two replays per setting, with new job
    contents of the same shape)."""
    say("case: spatial order in the batched tick")
    rng = np.random.default_rng(4)
    maps = []
    for dtype in ("i16", "i8"):
        t, _, _ = case(int(rng.integers(0, 1000)), (48, 40, 16), 1, 1, dtype, "uniform")
        maps.append((t, mcl.Map.from_tsdf(t)))
    specs = [(0, 5000, 9000, "uniform"), (1, 300, 700, "cluster"), (0, 4097, 4096, "edges"),
             (1, 64, 5000, "uniform"), (0, 2000, 12000, "cluster")]
    s = torch.cuda.Stream()
    ref = {}                            # job contents (seed) -> outputs of the first run
    for thr in (-1, 10 ** 7, 0):       # none; the three largest filters; all
        order_min(thr)
        for graph in (False, True):
            for rep in range(2 if graph else 1):
                got = tick_outputs(torch, mcl, maps, specs, 50 + rep, graph, s)
                if rep not in ref:
                    ref[rep] = got
                    continue
                for i, (a, b) in enumerate(zip(got, ref[rep])):
                    for x, y in zip(a, b):
                        assert np.array_equal(x.view(np.uint8), y.view(np.uint8)), \
                            f"threshold {thr} graph={graph} replay {rep} job {i}"


def test_global_workload_full_size(torch, mcl, order_min):
    """The global-localisation workload (10^6 particles x 28,660 points) takes
    the order at the default threshold; every log-weight equals the unordered
    launch's, bit for bit."""
    w = configs.config2()
    assert mcl.get_spatial_order_min() == 1 << 30 and (1 << 30) <= w.N * w.K
    say(f"case: spatial order, global workload N={w.N} K={w.K}")
    m = mcl.Map.from_tsdf(w.tmap)
    X, P = dev(torch, w.points), dev(torch, w.poses)
    order_min(1 << 30)
    a = mcl.sensor_update(m, X, P, w.sigma).cpu().numpy()
    order_min(-1)
    b = mcl.sensor_update(m, X, P, w.sigma).cpu().numpy()
    assert np.array_equal(bits(a), bits(b))
