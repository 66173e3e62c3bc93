"""The no-allocation sensor update (mcl_sensor_update_noalloc), through the C
ABI: bit for bit the results of mcl_sensor_update, on two calls in a row (the
second smaller, so it reads a scratch array that still holds the first call's
partials), plus one without partials; sizes beyond the fixed array are refused
before anything runs.  On the global workload mcl_sensor_update reads the
particles' pose constants from its table and the no-allocation call passes them
between lanes, so the first case also checks that the two paths agree bit for
bit."""

import ctypes as C
import sys

import numpy as np
import pytest

from tests.helpers import make_map, poses_from, random_rotations
from workloads import configs
from workloads.tsdf import f32

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def noalloc(torch, mcl, m, pts, poses, sigma):
    lib = mcl.lib()
    N, K = poses.shape[1], pts.shape[1]
    out = torch.empty(N, dtype=torch.float32, device=poses.device)
    st = lib.mcl_sensor_update_noalloc(m.handle, C.c_void_p(pts.data_ptr()), K, C.c_void_p(poses.data_ptr()), N,
                                       float(sigma), C.c_void_p(out.data_ptr()),
                                       C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == mcl.MCL_OK, lib.mcl_last_error()
    return out


def test_noalloc_matches_sensor_update():
    import torch
    from paper_2310_04172_amd import mcl

    dev = torch.device("cuda:0")
    w = configs.config2(n_particles=300000)
    say(f"case: no-allocation sensor update, global workload N={w.N} K={w.K}")
    m = mcl.Map.from_tsdf(w.tmap)
    P, X = torch.from_numpy(w.poses).to(dev), torch.from_numpy(w.points).to(dev)
    a = noalloc(torch, mcl, m, X, P, w.sigma)
    ref_a = mcl.sensor_update(m, X, P, w.sigma)
    torch.cuda.synchronize()
    assert torch.equal(a.view(torch.int32), ref_a.view(torch.int32))

    rng = np.random.default_rng(8)
    vals = rng.integers(-32767, 32768, size=(20, 36, 40)).astype(np.int16)
    tm = make_map(vals, 0.1, origin=(-0.5, 0.25, -0.1), tau=0.3)
    m2 = mcl.Map.from_tsdf(tm)
    ext = np.array(tm.dims) * tm.voxel
    for N, K in ((4097, 9001), (130, 4000)):   # smaller partials, then none
        say(f"case: no-allocation sensor update, small map N={N} K={K}")
        Pb = torch.from_numpy(poses_from(random_rotations(rng, N), rng.uniform(0, 1, (N, 3)) * ext)).to(dev)
        Xb = torch.from_numpy(rng.normal(0, 0.3 * ext.mean(), size=(3, K)).astype(np.float32)).to(dev)
        b = noalloc(torch, mcl, m2, Xb, Pb, f32(0.15))
        ref_b = mcl.sensor_update(m2, Xb, Pb, f32(0.15))
        torch.cuda.synchronize()
        assert torch.equal(b.view(torch.int32), ref_b.view(torch.int32)), (N, K)

    # beyond the fixed array: refused on the host, nothing enqueued
    lib = mcl.lib()
    fake = C.c_void_p(0x1000)
    N, K = mcl.MAX_PARTICLES, 40000          # 10 pieces x 2^21 floats = 80 MiB
    st = lib.mcl_sensor_update_noalloc(m.handle, fake, K, C.c_void_p(0x100000000), N, 0.1,
                                       C.c_void_p(0x800000000), None)
    assert st == mcl.MCL_ERANGE and b"scratch array" in lib.mcl_last_error()
