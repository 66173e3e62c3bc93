"""Batched tick (mcl_tick), graph replay and launch-shape tuning, through the C ABI.

The contract: every filter in a tick gets bit for bit the results of the
single-filter calls (sensor update, normalisation, pose estimate for the
filters that ask for one, resampling), eagerly or replayed from a captured
graph, and no launch shape changes any result.  The batched workload itself
(64 filters on the warehouse map) is checked against the CPU oracle directly.
"""

import sys

import numpy as np
import pytest

from tests import checks
from tests.helpers import make_map, poses_from, random_rotations
from workloads import configs
from workloads.tsdf import f32, to_bricks

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


def small_map(rng, dtype, dims=(40, 36, 20), v=0.1):
    nx, ny, nz = dims
    if dtype == "f32":
        vals = rng.uniform(-0.3, 0.3, size=(nz, ny, nx)).astype(np.float32)
        vals[:, :, : nx // 2] = 0.3
    else:
        lim = 32767 if dtype == "i16" else 127
        vals = rng.integers(-lim, lim + 1, size=(nz, ny, nx)).astype(np.int16 if dtype == "i16" else np.int8)
        vals[:, :, : nx // 2] = lim
    return make_map(vals, v, origin=(-0.5, 0.25, -0.1), tau=0.3, dtype=dtype)


def job_set(torch, mcl, seed, maps, specs):
    rng = np.random.default_rng(seed)
    filters = []
    for (mi, N, K) in specs:
        tmap, m = maps[mi]
        ext = np.array(tmap.dims) * tmap.voxel
        poses = poses_from(random_rotations(rng, N), rng.uniform(0, 1, (N, 3)) * ext)
        pts = rng.normal(0, 0.3 * ext.mean(), size=(3, K)).astype(np.float32) if K else None
        f = mcl.Filter(m, dev(torch, pts) if K else None, dev(torch, poses), f32(0.1 + 0.05 * mi),
                       int(rng.integers(0, 2 ** 63)), want_estimate=len(filters) % 2 == 0)
        filters.append(f)
    return filters


def single(torch, mcl, f):
    lw = (mcl.sensor_update_trilinear if f.trilinear else mcl.sensor_update)(f.map, f.points, f.poses, f.sigma)
    w, wq, lz = mcl.normalize(lw)
    idx, pout = mcl.resample(wq, f.seed, f.tick, f.poses)
    est = mcl.pose_estimate(w, f.poses) if f.est_mean is not None else ()
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (lw, w, wq, lz, idx, pout, *est)]


def outputs(torch, f):
    torch.cuda.synchronize()
    est = (f.est_mean, f.est_idx, f.est_pose) if f.est_mean is not None else ()
    return [x.cpu().numpy() for x in (f.logw, f.w, f.wq, f.log_z, f.idx, f.poses_out, *est)]


def assert_same(a, b, what):
    assert len(a) == len(b), what
    names = ("logw", "w", "wq", "log_z", "idx", "poses_out", "est_mean", "est_idx", "est_pose")
    for n, x, y in zip(names, a, b):
        assert x.dtype == y.dtype and np.array_equal(x.view(np.uint8), y.view(np.uint8)), f"{what}: {n} differs"


@pytest.fixture(scope="module")
def maps(torch, mcl):
    rng = np.random.default_rng(1)
    out = []
    for dtype in ("i16", "i8", "f32", "i16"):
        t = small_map(rng, dtype)
        out.append((t, mcl.Map.from_tsdf(t)))
    return out


SPECS = [(0, 1, 1), (1, 63, 1025), (2, 65, 9000), (0, 1000, 5000), (3, 130, 0), (1, 5000, 4096),
         (2, 7, 4097), (0, 4097, 300), (3, 2000, 12000)]


def test_tick_matches_single_calls(torch, mcl, maps):
    say("case: tick eager vs single calls, mixed storage types")
    filters = job_set(torch, mcl, 3, maps, SPECS)
    mcl.tick(filters)
    got = [outputs(torch, f) for f in filters]
    for i, f in enumerate(filters):
        assert_same(got[i], single(torch, mcl, f), f"job {i} (N={f.N}, K={f.K})")


def test_tick_graph_replay(torch, mcl, maps):
    """A captured chain replays correctly for new job contents and a different
    job count, with eager work and synchronisation between replays."""
    say("case: tick graph replay")
    s = torch.cuda.Stream()
    for rep, (seed, specs) in enumerate([(10, SPECS), (11, SPECS[::-1]), (12, SPECS[2:7]), (13, SPECS)]):
        filters = job_set(torch, mcl, seed, maps, specs)
        if rep == 2:  # a tick without any pose estimate between ticks with them
            for f in filters:
                f.est_mean = f.est_idx = f.est_pose = None
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            mcl.tick(filters, graph=True, stream=s)
        s.synchronize()
        got = [outputs(torch, f) for f in filters]
        # eager work on the default stream between replays
        _ = torch.ones(1 << 20, device="cuda").sum().item()
        for i, f in enumerate(filters):
            assert_same(got[i], single(torch, mcl, f), f"replay {rep} job {i}")


def test_tick_max_jobs(torch, mcl, maps):
    """MCL_MAX_JOBS filters in one tick (every storage type, N from 1 to 40, K
    from 0 to 300, every second filter with a pose estimate), eager and
    replayed from a graph: the job searches over 4,096 entries and the prefix
    offsets hold, and a seeded sample of filters (with the first and the last)
    gets its single calls' results bit for bit."""
    n = mcl.MAX_JOBS
    say(f"case: tick with {n} filters")
    rng = np.random.default_rng(77)
    specs = [(int(rng.integers(0, 4)), int(rng.integers(1, 41)), int(rng.integers(0, 301))) for _ in range(n)]
    filters = job_set(torch, mcl, 78, maps, specs)
    sample = sorted({0, n - 1, *rng.choice(n, size=126, replace=False).tolist()})
    s = torch.cuda.Stream()
    for graph in (False, True):
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            mcl.tick(filters, graph=graph, stream=s)
        s.synchronize()
        for i in sample:
            f = filters[i]
            assert_same(outputs(torch, f), single(torch, mcl, f), f"graph={graph} job {i} (N={f.N}, K={f.K})")


def test_tick_one_launch_weights_equal_chains(torch, mcl, maps):
    """The tick's weights stage with one workgroup per filter (all filters at
    most the limit: one launch, or two around the pose estimates) and as the
    launch chains (limit 0, or one filter above it): the same bits, eagerly and
    replayed from graphs."""
    say("case: tick weights stage, one launch vs chains")
    prev = mcl.get_weights_fused_max()
    specs = [(0, 1, 1), (1, 63, 1025), (2, 65, 9000), (0, 1000, 5000), (3, 130, 0), (1, 4096, 4096),
             (2, 7, 4097), (0, 4095, 300), (3, 2000, 12000)]
    s = torch.cuda.Stream()
    try:
        for est in (True, False):
            results = []
            for limit in (4096, 0, 1000):       # 1000: the larger filters take the chains
                mcl.set_weights_fused_max(limit)
                for graph in (False, True):
                    filters = job_set(torch, mcl, 21, maps, specs)
                    if not est:
                        for f in filters:
                            f.est_mean = f.est_idx = f.est_pose = None
                    torch.cuda.synchronize()
                    with torch.cuda.stream(s):
                        mcl.tick(filters, graph=graph, stream=s)
                    s.synchronize()
                    results.append((limit, graph, [outputs(torch, f) for f in filters]))
            for limit, graph, got in results[1:]:
                for i in range(len(specs)):
                    assert_same(got[i], results[0][2][i], f"est={est} limit={limit} graph={graph} job {i}")
    finally:
        mcl.set_weights_fused_max(prev)


def test_launch_shapes_are_bit_identical(torch, mcl, tmp_path, monkeypatch):
    say("case: launch shapes")
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("MCL_TUNE_CACHE", str(cache))   # the tuner appends its result here
    w = configs.config1()
    m = mcl.Map.from_tsdf(w.tmap)
    P, X = dev(torch, w.poses), dev(torch, w.points)
    ref = mcl.sensor_update(m, X, P, w.sigma).cpu().numpy()
    try:
        for wpb in (2, 4, 8):
            for bpc in (0, 1, 2, 8, 32):
                mcl.set_launch_config("i16", w.K, w.N, (wpb, bpc))
                got = mcl.sensor_update(m, X, P, w.sigma).cpu().numpy()
                assert np.array_equal(got, ref), (wpb, bpc)
        for runs in (1, 2, 8, 64):
            for coarse, l8 in ((0, 1), (0, 8), (1, 0), (2, 0)):
                mcl.set_launch_config("i16", w.K, w.N, (4, 0, coarse, runs, l8))
                got = mcl.sensor_update(m, X, P, w.sigma).cpu().numpy()
                assert np.array_equal(got, ref), (runs, coarse, l8)
        best = mcl.autotune(m, X, P, w.sigma)
        assert best[0] in (2, 4, 8) and best[1] in (0, 2, 4, 8, 16) and best[2] in (0, 1, 2)
        assert best[3] in (0, 1, 2, 4, 8, 16, 64) and 0 <= best[4] <= 8
        assert mcl.get_launch_config("i16", w.K, w.N) == best
        last = cache.read_text().strip().splitlines()[-1].split()
        kc, nc = int(np.ceil(np.log2(w.K))), int(np.ceil(np.log2(w.N)))
        assert [int(x) for x in last[1:]] == [0, kc, nc, *best], last
        assert np.array_equal(mcl.sensor_update(m, X, P, w.sigma).cpu().numpy(), ref)
    finally:
        mcl.set_launch_config("i16", w.K, w.N, None)


@pytest.fixture(scope="module")
def mixed_maps(torch, mcl, maps):
    """The same small maps, the first three also held as sparse brick pools
    (every sensor group of a tick: dense and sparse, each storage type)."""
    out = list(maps)
    for t, _ in maps[:3]:
        co, va = to_bricks(t)
        out.append((t, mcl.Map.from_bricks(t.dims, t.voxel, t.origin, t.tau, t.dtype, co, va)))
    return out


MIXED = [(4, 1, 1), (5, 63, 1025), (6, 65, 9000), (0, 1000, 5000), (4, 130, 0), (5, 5000, 4096),
         (6, 7, 4097), (1, 4097, 300), (4, 2000, 12000), (2, 300, 2000), (3, 90, 700)]


def test_tick_with_sparse_maps(torch, mcl, mixed_maps):
    """Dense and sparse maps of every storage type in one tick, eager and from
    captured graphs with new contents and another job count: every filter
    gets the single-filter calls' bits (a sparse map gives the dense map's)."""
    say("case: tick with dense and sparse maps")
    filters = job_set(torch, mcl, 31, mixed_maps, MIXED)
    mcl.tick(filters)
    got = [outputs(torch, f) for f in filters]
    for i, f in enumerate(filters):
        assert_same(got[i], single(torch, mcl, f), f"eager job {i} (N={f.N}, K={f.K})")
    s = torch.cuda.Stream()
    for rep, (seed, specs) in enumerate([(32, MIXED), (33, MIXED[::-1][:7]), (34, MIXED)]):
        filters = job_set(torch, mcl, seed, mixed_maps, specs)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            mcl.tick(filters, graph=True, stream=s)
        s.synchronize()
        got = [outputs(torch, f) for f in filters]
        _ = torch.ones(1 << 20, device="cuda").sum().item()
        for i, f in enumerate(filters):
            assert_same(got[i], single(torch, mcl, f), f"replay {rep} job {i}")
    # a filter on a sparse map gives every bit it gives on the dense map with the same values
    t0, dm = mixed_maps[0]
    sm = mixed_maps[4][1]
    rng = np.random.default_rng(35)
    ext = np.array(t0.dims) * t0.voxel
    P = dev(torch, poses_from(random_rotations(rng, 300), rng.uniform(0, 1, (300, 3)) * ext))
    X = dev(torch, rng.normal(0, 0.3 * ext.mean(), size=(3, 3000)).astype(np.float32))
    a = mcl.Filter(sm, X, P, f32(0.2), 7, want_estimate=True)
    b = mcl.Filter(dm, X, P, f32(0.2), 7, want_estimate=True)
    mcl.tick([a])
    mcl.tick([b])
    assert_same(outputs(torch, a), outputs(torch, b), "sparse vs dense map")


def test_tick_with_trilinear_lookups(torch, mcl, mixed_maps):
    """Trilinear filters (dense maps) beside nearest ones on dense and sparse
    maps in one tick, eager and replayed: every filter gets the bits of its
    single-filter calls; a sparse map with the trilinear lookup is refused."""
    say("case: tick with trilinear, nearest and sparse jobs")
    s = torch.cuda.Stream()
    sparse = {id(m) for _, m in mixed_maps[4:]}
    for rep, (seed, specs) in enumerate([(41, MIXED), (42, MIXED[::-1]), (43, MIXED[:6])]):
        filters = job_set(torch, mcl, seed, mixed_maps, specs)
        for i, f in enumerate(filters):
            f.trilinear = i % 3 != 2 and id(f.map) not in sparse   # two of three dense-map filters
        torch.cuda.synchronize()
        if rep == 0:
            mcl.tick(filters)
        else:
            with torch.cuda.stream(s):
                mcl.tick(filters, graph=True, stream=s)
            s.synchronize()
        got = [outputs(torch, f) for f in filters]
        _ = torch.ones(1 << 20, device="cuda").sum().item()
        assert any(f.trilinear for f in filters)
        for i, f in enumerate(filters):
            assert_same(got[i], single(torch, mcl, f), f"rep {rep} job {i} (trilinear {f.trilinear})")
    bad = job_set(torch, mcl, 44, mixed_maps, [(4, 10, 100)])[0]
    bad.trilinear = True
    with pytest.raises(mcl.MclError):
        mcl.tick([bad])


def test_tick_alone_equals_in_mix(torch, mcl, maps):
    """A filter gives the same bits alone and inside a larger batch."""
    say("case: alone vs mix")
    filters = job_set(torch, mcl, 21, maps, SPECS)
    mcl.tick(filters)
    mixed = [outputs(torch, f) for f in filters]
    for i in (0, 3, 8):
        mcl.tick([filters[i]])
        assert_same(outputs(torch, filters[i]), mixed[i], f"job {i} alone")


def test_runs_do_not_change_bits(torch, mcl, maps):
    """A small filter alone has few (group, piece) pairs, so its groups are
    split into 64 runs; beside a large filter (over 16,384 pairs) a tick uses
    one run per group.  Both must give the same bits."""
    say("case: run split alone vs one run in a large tick")
    small, big = job_set(torch, mcl, 51, maps, [(0, 100, 1000), (1, 300000, 60000)])
    mcl.tick([small])
    alone = outputs(torch, small)
    mcl.tick([small, big])
    assert_same(outputs(torch, small), alone, "small filter in a large tick")
    assert_same(outputs(torch, big), single(torch, mcl, big), "large filter")


@pytest.fixture(scope="module")
def cfg4():
    return configs.config4()


def test_config4_tick_matches_oracle(torch, mcl, oracle_lib, cfg4):
    """The batched workload (64 filters on the 1024x1024x128 warehouse map,
    N log-uniform in [2048, 524288], VLP-16 16x1800 and OS0-64 64x1024 scans) as
    one graph-replayed tick, then the same graph replayed on the resampled sets
    (tick 1).  Every filter against the oracle: 64 seeded particles'
    log-weights within 1e-5, the whole normalisation within its float64 bound
    and the whole resampling bit for bit (on the GPU's own weights), the pose
    estimate of every eighth filter within its bound."""
    tmap, specs = cfg4
    say(f"case: config-4 tick vs oracle, {len(specs)} filters, sum N {sum(f.N for f in specs)}")
    m = mcl.Map.from_tsdf(tmap)
    filters = [mcl.Filter(m, dev(torch, sp.points), dev(torch, sp.poses), sp.sigma, sp.seed, want_w=True,
                          want_estimate=i % 8 == 0) for i, sp in enumerate(specs)]
    rng = np.random.default_rng(404)
    s = torch.cuda.Stream()
    Ns = [sp.N for sp in specs]
    assert min(Ns) < 4096 and max(Ns) > 300000
    for tick in (0, 1):
        inputs = [f.poses.cpu().numpy() for f in filters]
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            mcl.tick(filters, graph=True, stream=s)
        s.synchronize()
        for i, (f, sp, P) in enumerate(zip(filters, specs, inputs)):
            what = f"tick {tick} filter {i} (N={f.N}, K={f.K})"
            sub = np.sort(rng.choice(f.N, size=min(64, f.N), replace=False))
            checks.check_update(oracle_lib, tmap, sp.points, P, sp.sigma, f.logw.cpu().numpy(),
                                f.wq.cpu().numpy(), f.log_z.cpu().numpy()[0], f.idx.cpu().numpy(), f.seed,
                                f.tick, sub, poses_out=f.poses_out.cpu().numpy(), w=f.w.cpu().numpy(), what=what)
            if f.est_mean is not None:
                checks.check_estimate(f.est_mean.cpu().numpy(), f.est_idx.cpu().numpy()[0],
                                      f.est_pose.cpu().numpy(), f.w.cpu().numpy(), P, what)
        say(f"tick {tick}: every filter matches the oracle")
        for f in filters:    # the resampled set is the next tick's input
            f.poses, f.poses_out = f.poses_out, f.poses
            f.tick += 1


def test_tick_nowait_and_deferred_map_free(torch, mcl, maps):
    """A tick with MCL_TICK_NOWAIT returns MCL_EBUSY (enqueuing nothing) while
    the stream's previous tick still holds the table staging buffer, and runs
    once it is free; mcl_map_free waits for the work enqueued on the map, so a
    map freed right after its update leaves the results intact."""
    say("case: tick nowait (EBUSY) and deferred map free")
    w = configs.config2(n_particles=262144)
    m = mcl.Map.from_tsdf(w.tmap)
    P, X = dev(torch, w.poses), dev(torch, w.points)
    s = torch.cuda.Stream()
    a, b = job_set(torch, mcl, 61, maps, [(0, 3000, 5000), (1, 2000, 4000)])
    with torch.cuda.stream(s):
        mcl.tick([a, b], stream=s)      # the stream's tick workspace, grown once (growth synchronises)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        lw = mcl.sensor_update(m, X, P, w.sigma, stream=s)     # ~5 ms of work ahead of the ticks
        assert mcl.tick([a], stream=s, nowait=True)            # staging buffer free: enqueued
        busy = not mcl.tick([b], stream=s, nowait=True)        # the first tick's table copy has not run yet
        assert mcl.tick([b], stream=s)                         # waits for the buffer, then runs
    assert busy, "expected MCL_EBUSY while the previous tick's table copy waits behind the sensor update"
    ref = mcl.sensor_update(m, X, P, w.sigma, stream=s)
    s.synchronize()
    for f in (a, b):
        assert_same(outputs(torch, f), single(torch, mcl, f), "tick after EBUSY")
    # deferred free: update on the side stream, free at once, then reuse memory
    with torch.cuda.stream(s):
        out = mcl.sensor_update(m, X, P, w.sigma, stream=s)
    m.close()
    junk = torch.full((64 << 20,), -7, dtype=torch.int16, device="cuda")   # may take the freed memory
    s.synchronize()
    torch.cuda.synchronize()
    assert torch.equal(out, ref) and torch.equal(lw, ref)
    del junk
