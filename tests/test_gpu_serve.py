"""The serving engine: every robot's result is the same served in the mix as
replayed alone with the single-filter calls (bit for bit), under a memory
budget small enough to make robots wait for admission."""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("n_streams,depth,order", [(2, 1, "fifo"), (1, 2, "fifo"), (2, 1, "stale")])
def test_served_equals_alone(n_streams, depth, order):
    import torch
    from paper_2310_04172_amd import mcl
    from paper_2310_04172_amd.serve import Engine, Robot, update_draw
    from workloads import served

    say(f"case: served engine, small trace, {n_streams} streams x {depth} ticks, order {order}")
    sw = served.build(n_robots=12, trace_s=2.0, rate_hz=10.0, scans_per_map=2, map_subset=[0, 3])
    for sp in sw.robots:          # keep the test small: scale particle counts down
        sp.n_global = 1 + sp.n_global // 64
        sp.n_track = 1 + sp.n_track // 16
    dev = torch.device("cuda:0")
    maps = [mcl.Map.from_tsdf(t) for t in sw.tmaps]
    vals = [torch.from_numpy(t.values).to(dev) for t in sw.tmaps]
    scans = [[torch.from_numpy(p).to(dev) for p in lst] for lst in sw.scans]

    def robots():
        return [Robot(sp.rid, maps[sp.map_idx], scans[sp.map_idx][sp.scan_idx], served.sigma_for(sw.tmaps[sp.map_idx]),
                      [(3, "global"), (None, "track")]) for sp in sw.robots]

    def init(r, phase, probe=False):
        sp = sw.robots[r.rid]
        n = sp.n_global if phase == "global" else sp.n_track
        if probe:
            return n
        return served.device_particles(torch, sw.tmaps[sp.map_idx], vals[sp.map_idx], n, phase, sp.gt,
                                       seed=(r.rid << 1) | (phase == "track"), device=dev)

    big = max(mcl.job_bytes(sp.n_global, scans[sp.map_idx][sp.scan_idx].shape[1]) for sp in sw.robots)
    eng = Engine(robots(), init, budget_bytes=3 * big, max_evals_per_tick=2e9, seed=9, n_streams=n_streams,
                 depth=depth, order=order)
    st = eng.run(sw.trace)
    summ = st.summary()
    say(f"served: {summ}")
    assert st.completed > 0 and st.completed + st.dropped <= st.arrived
    assert st.max_resident_bytes <= 3 * big
    # replay each robot alone, update by update, with the single-filter calls
    for r in eng.robots:
        if r.poses is None:
            continue
        alone = Robot(r.rid, r.map, r.points, r.sigma, [(3, "global"), (None, "track")])
        poses = None
        for n in range(r.completed):
            if poses is None:
                poses = init(alone, alone.phase)
            lw = mcl.sensor_update(alone.map, alone.points, poses, alone.sigma)
            _, wq, _ = mcl.normalize(lw, want_w=False)
            _, poses = mcl.resample(wq, update_draw(9, r.rid, n), poses)
            if n + 1 == 3:
                alone.phase_i = 1
                poses = None
        if poses is None:
            poses = init(alone, alone.phase)
        torch.cuda.synchronize()
        assert torch.equal(poses, r.poses), f"robot {r.rid} after {r.completed} updates"
