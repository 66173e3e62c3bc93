"""The measurement calls of the gather roofline, through the C ABI: the replay
issues the sensor kernel's own gathers, so the values it adds up are the ones
the sensor update squares; each call runs and writes its sink."""

import sys

import numpy as np
import pytest

from tests.helpers import make_map, poses_from, random_rotations, score_const
from workloads.tsdf import f32

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_replay_reads_the_sensor_updates_values():
    """Sum over the replayed gathers of q^2 (one pass) equals the sum over the
    particles of the sensor update's sum of squares -logw / c, within float32
    rounding of two summation orders; r passes give r times that; the masked
    single-gather replay gives the same total."""
    import torch
    from paper_2310_04172_amd import mcl

    say("case: gather replay against the sensor update")
    rng = np.random.default_rng(12)
    nx, ny, nz = 40, 70, 24
    vals = rng.integers(-32767, 32768, size=(nz, ny, nx)).astype(np.int16)
    vals[:, :, : nx // 2] = 32767          # bricks wholly at +Q: read the sentinel
    tm = make_map(vals, 0.1, origin=(-0.3, 0.2, -0.1), tau=0.3)
    m = mcl.Map.from_tsdf(tm)
    ext = np.array(tm.dims) * tm.voxel
    N, K = 128, 9001
    P = torch.from_numpy(poses_from(random_rotations(rng, N), rng.uniform(0, 1, (N, 3)) * ext)).cuda()
    X = torch.from_numpy(rng.normal(0, 0.3 * ext.mean(), size=(3, K)).astype(np.float32)).cuda()
    sigma = f32(0.15)
    lw = mcl.sensor_update(m, X, P, sigma).cpu().numpy().astype(np.float64)
    want = float(np.sum(-lw / score_const("i16", tm.tau, sigma)))
    npiece = -(-K // 4096)
    blocks = (N // 64 * npiece + 3) // 4
    sink = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    for masked, two in ((False, True), (True, False)):
        offs = mcl.bench_gather_offsets(m, X, P, masked=masked)
        assert offs.shape == (N, K)
        for reps in (1, 3):
            mcl.bench_gather_replay(m, offs, reps, two, blocks, sink)
            got = float(sink.double().sum().cpu())
            assert abs(got - reps * want) <= 1e-5 * reps * want, (masked, reps, got, reps * want)
    # the ceiling kernels run and fill their sinks
    region = torch.ones(1 << 24, dtype=torch.uint8, device="cuda")
    gsink = torch.zeros(64 * 256, dtype=torch.float32, device="cuda")
    mcl.bench_line_gather(region, 10, 16, 2, 3, 64, gsink, bytes_per_lane=2)
    mcl.bench_l1_gather(region, 4, 2, 2, 64, gsink)
    mcl.bench_stream_read(region, 64, gsink)
    torch.cuda.synchronize()
    assert torch.isfinite(gsink).all()
