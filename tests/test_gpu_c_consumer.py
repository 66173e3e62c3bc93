"""The C ABI from a plain C program, with no Python or torch in its path.

tests/c/mcl_consumer.c includes only include/mcl.h and the HIP runtime's C
API; it is built here with gcc, linked to the library and run on the GPU.  It
updates one filter through the single-filter calls, then that filter and a
second one (1.5 sigma, the next update) as one graph-captured tick, replayed
after its outputs were partly cleared, with the map freed while the replay may
still run, and checks that a NULL map is refused.  Its outputs are compared
here with the oracle: log-weights within 1e-5, the normalisation within its
float64 bound, the resampling bit for bit, and the tick's copy of the first
filter bit-identical to the single calls.  N = 3,000 takes the one-launch
weights shape, N = 5,000 the launch chains; K = 5,000 spans two scan pieces.
"""

import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

from tests import checks
from tests.helpers import make_map, poses_from, random_rotations
from workloads.tsdf import f32

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2310_04172_amd")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def build(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    exe = str(tmp_path / "mcl_consumer")
    subprocess.run([gcc, "-std=c11", "-Wall", "-D__HIP_PLATFORM_AMD__", f"-I{rocm}/include",
                    f"-I{os.path.join(ROOT, 'include')}", os.path.join(ROOT, "tests", "c", "mcl_consumer.c"),
                    "-o", exe, f"-L{rocm}/lib", "-lamdhip64", f"-L{PKG}", "-lmcl", f"-Wl,-rpath,{rocm}/lib",
                    f"-Wl,-rpath,{PKG}"], check=True)
    return exe


def load(d, s, N):
    def f(name, dt, n):
        a = np.fromfile(os.path.join(d, f"{s}_{name}.bin"), dtype=dt)
        assert a.size == n, (s, name, a.size)
        return a
    return {"logw": f("logw", np.float32, N), "w": f("w", np.float64, N), "wq": f("wq", np.uint64, N),
            "lz": f("lz", np.float64, 1), "idx": f("idx", np.int32, N),
            "pout": f("pout", np.float32, 12 * N).reshape(12, N)}


def check_set(oracle, out, tmap, pts, poses, sigma, seed, tick, what):
    ref = oracle.sensor_update(tmap, pts, poses, sigma)
    checks.assert_logw_close(out["logw"], ref, f"{what} log-weights")
    checks.check_normalize(oracle, out["logw"], out["wq"], float(out["lz"][0]), out["w"], what)
    checks.check_resample(oracle, out["wq"], seed, tick, out["idx"], poses, out["pout"], what)


@pytest.mark.parametrize("N", [3000, 5000])
def test_c_program_against_the_oracle(oracle_lib, tmp_path, N):
    exe = build(tmp_path)
    rng = np.random.default_rng(600 + N)
    nx, ny, nz, voxel, tau = 40, 36, 20, 0.1, 0.3
    origin = (-0.5, 0.25, -0.1)
    vals = rng.integers(-32767, 32768, size=(nz, ny, nx)).astype(np.int16)
    vals[:, :, : nx // 2] = 32767
    tmap = make_map(vals, voxel, origin=origin, tau=tau)
    K = 5000
    ext = np.array([nx, ny, nz]) * voxel
    poses = poses_from(random_rotations(rng, N), rng.uniform(0, 1, (N, 3)) * ext + np.array(origin))
    pts = rng.normal(0, 0.3 * ext.mean(), size=(3, K)).astype(np.float32)
    sigma = f32(0.15)
    seed = int(rng.integers(0, 2 ** 63))
    vals.tofile(tmp_path / "map.bin")
    np.ascontiguousarray(pts).tofile(tmp_path / "points.bin")
    np.ascontiguousarray(poses).tofile(tmp_path / "poses.bin")
    fmt = lambda x: "%.9g" % float(np.float32(x))
    args = [exe, str(tmp_path), str(nx), str(ny), str(nz), fmt(voxel), *[fmt(o) for o in origin], fmt(tau),
            str(K), str(N), fmt(sigma), str(seed)]
    say(f"case: C consumer N={N} K={K}")
    r = subprocess.run(args, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.returncode, r.stdout, r.stderr)
    one, t0, t1 = (load(tmp_path, s, N) for s in ("single", "tick0", "tick1"))
    check_set(oracle_lib, one, tmap, pts, poses, sigma, seed, 0, f"C single N={N}")
    for k in one:
        assert np.array_equal(one[k].view(np.uint8), t0[k].view(np.uint8)), f"tick copy differs in {k}"
    sigma1 = np.float32(1.5) * np.float32(sigma)
    check_set(oracle_lib, t1, tmap, pts, poses, sigma1, seed + 1, 1, f"C tick second filter N={N}")
