"""The C-ABI library: it loads, exports every symbol the header declares, and
rejects bad arguments on the host before touching the device (no GPU needed)."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcl.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mcl_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def mcl():
    from paper_2310_04172_amd import mcl as m
    return m


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("mcl_map_upload", "mcl_map_free", "mcl_sensor_update", "mcl_normalize", "mcl_resample",
              "mcl_debug_voxel_indices", "mcl_last_error", "mcl_tick", "mcl_job_bytes", "mcl_autotune",
              "mcl_set_launch_config", "mcl_pose_estimate", "mcl_sensor_update_trilinear", "mcl_motion_update",
              "mcl_init_uniform", "mcl_map_upload_bricks", "mcl_map_bytes", "mcl_sensor_update_sum"):
        assert f in names


def test_library_exports_every_declared_symbol(mcl):
    lib = mcl.lib()
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_argument_errors_are_reported_on_the_host(mcl):
    lib = mcl.lib()
    P = C.c_void_p
    fake = P(0x1000)
    # NULL map / pointers, bad sizes, bad sigma: rejected before any device work
    assert lib.mcl_sensor_update(None, fake, 10, fake, 10, 0.1, P(0x2000), None) == mcl.MCL_EINVAL
    assert b"NULL map" in lib.mcl_last_error()
    assert lib.mcl_sensor_update_trilinear(None, fake, 10, fake, 10, 0.1, P(0x2000), None) == mcl.MCL_EINVAL
    assert lib.mcl_sensor_update_trilinear(fake, fake, 10, fake, 10, float("nan"), P(0x2000), None) == mcl.MCL_EINVAL
    assert lib.mcl_sensor_update_sum(None, fake, 10, fake, 10, 0.1, P(0x2000), None) == mcl.MCL_EINVAL
    assert lib.mcl_sensor_update_sum(fake, fake, 10, fake, 10, -0.1, P(0x2000), None) == mcl.MCL_EINVAL
    assert lib.mcl_normalize(None, 10, None, fake, None, None) == mcl.MCL_EINVAL
    assert lib.mcl_normalize(fake, 0, None, P(0x9000), None, None) == mcl.MCL_EINVAL
    assert lib.mcl_normalize(fake, mcl.MAX_PARTICLES + 1, None, P(0x90000000), None, None) == mcl.MCL_ERANGE
    assert lib.mcl_resample(fake, 10, 0, 0, P(0x9000), fake, None, None) == mcl.MCL_EINVAL
    assert lib.mcl_resample(fake, 0, 0, 0, P(0x9000), None, None, None) == mcl.MCL_EINVAL
    assert lib.mcl_map_free(None) == mcl.MCL_EINVAL
    assert lib.mcl_pose_estimate(None, fake, 10, P(0x9000), None, None, None) == mcl.MCL_EINVAL
    assert lib.mcl_pose_estimate(fake, fake, 0, P(0x90000), None, None, None) == mcl.MCL_EINVAL
    assert lib.mcl_pose_estimate(fake, fake, mcl.MAX_PARTICLES + 1, P(0x9000000000), None, None,
                                 None) == mcl.MCL_ERANGE
    assert lib.mcl_pose_estimate(P(0x10000), P(0x20000), 100, P(0x10008), None, None, None) == mcl.MCL_EINVAL
    assert lib.mcl_pose_estimate(P(0x10000), P(0x20000), 100, P(0x90000), P(0x90010), None,
                                 None) == mcl.MCL_EINVAL
    d12 = (C.c_float * 12)(*([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0]))
    assert lib.mcl_motion_update(None, fake, 10, d12, 0.1, 0.1, 1, 1, None) == mcl.MCL_EINVAL
    assert lib.mcl_motion_update(fake, fake, 0, d12, 0.1, 0.1, 1, 1, None) == mcl.MCL_EINVAL
    assert lib.mcl_motion_update(fake, fake, 10, d12, -0.1, 0.1, 1, 1, None) == mcl.MCL_EINVAL
    assert lib.mcl_motion_update(P(0x10000), P(0x10004), 10, d12, 0.1, 0.1, 1, 1, None) == mcl.MCL_EINVAL
    bad = (C.c_float * 12)(*([float("nan")] + [0.0] * 11))
    assert lib.mcl_motion_update(fake, fake, 10, bad, 0.1, 0.1, 1, 1, None) == mcl.MCL_EINVAL
    assert lib.mcl_init_uniform(None, fake, 10, 0.1, 1, None) == mcl.MCL_EINVAL
    assert lib.mcl_init_uniform(fake, fake, 10, -1.0, 1, None) == mcl.MCL_EINVAL
    assert lib.mcl_init_uniform(fake, fake, mcl.MAX_PARTICLES + 1, 0.1, 1, None) == mcl.MCL_ERANGE
    # sparse maps: bricks outside the grid or listed twice, before any allocation
    d = mcl.MapDesc(8, 8, 8, 0.1, (C.c_float * 3)(0, 0, 0), 0.3, 0)
    h = P()
    vals = (C.c_int16 * 128)()
    assert lib.mcl_map_upload_bricks(C.byref(d), 1, (C.c_int32 * 3)(2, 0, 0), vals, None, C.byref(h)) == mcl.MCL_EINVAL
    assert b"outside the grid" in lib.mcl_last_error()
    assert lib.mcl_map_upload_bricks(C.byref(d), 2, (C.c_int32 * 6)(1, 1, 1, 1, 1, 1), vals, None,
                                     C.byref(h)) == mcl.MCL_EINVAL
    assert b"listed twice" in lib.mcl_last_error()
    assert lib.mcl_map_upload_bricks(C.byref(d), -1, None, None, None, C.byref(h)) == mcl.MCL_EINVAL
    # overlapping output and input
    assert lib.mcl_normalize(P(0x10000), 100, None, P(0x10010), None, None) == mcl.MCL_EINVAL
    d = mcl.MapDesc(0, 4, 4, 0.1, (C.c_float * 3)(0, 0, 0), 0.3, 0)
    h = P()
    assert lib.mcl_map_upload(C.byref(d), fake, None, C.byref(h)) == mcl.MCL_EINVAL
    d = mcl.MapDesc(4, 4, 4, -0.1, (C.c_float * 3)(0, 0, 0), 0.3, 0)
    assert lib.mcl_map_upload(C.byref(d), fake, None, C.byref(h)) == mcl.MCL_EINVAL
    d = mcl.MapDesc(4, 4, 4, 0.1, (C.c_float * 3)(0, 0, 0), 0.3, 7)
    assert lib.mcl_map_upload(C.byref(d), fake, None, C.byref(h)) == mcl.MCL_EINVAL
    d = mcl.MapDesc(65536, 65536, 4096, 0.1, (C.c_float * 3)(0, 0, 0), 0.3, 0)
    assert lib.mcl_map_upload(C.byref(d), fake, None, C.byref(h)) == mcl.MCL_ERANGE


def test_tick_and_tuning_argument_errors(mcl):
    lib = mcl.lib()
    P = C.c_void_p
    assert lib.mcl_tick(None, 1, 0, None) == mcl.MCL_EINVAL
    jobs = (mcl.FilterJob * 2)()
    jobs[0] = mcl.FilterJob(P(0x1000), P(0x2000), 10, P(0x3000), 10, 0.1, P(0x4000), None, P(0x5000), None, 7, 0,
                            P(0x6000), None)
    jobs[1] = mcl.FilterJob(P(0x1000), P(0x2000), 10, P(0x3000), 10, -1.0, P(0x4000), None, P(0x5000), None, 7, 0,
                            P(0x6000), None)
    assert lib.mcl_tick(jobs, 2, 0, None) == mcl.MCL_EINVAL
    assert b"job 1" in lib.mcl_last_error()
    assert lib.mcl_tick(jobs, mcl.MAX_JOBS + 1, 0, None) == mcl.MCL_ERANGE
    # a pose estimate needs the weights; its optional outputs need est_mean
    jobs[1].sigma = 0.1
    jobs[1].est_mean = P(0x7000)
    assert lib.mcl_tick(jobs, 2, 0, None) == mcl.MCL_EINVAL and b"needs the weights" in lib.mcl_last_error()
    jobs[1].est_mean = None
    jobs[1].est_idx = P(0x7100)
    assert lib.mcl_tick(jobs, 2, 0, None) == mcl.MCL_EINVAL and b"without est_mean" in lib.mcl_last_error()
    jobs[1].est_idx = None
    jobs[1].score = 7
    assert lib.mcl_tick(jobs, 2, 0, None) == mcl.MCL_EINVAL and b"score must be" in lib.mcl_last_error()
    jobs[1].score = mcl.SCORE_PRODUCT
    jobs[1].lookup = 5   # neither nearest nor trilinear
    assert lib.mcl_tick(jobs, 2, 0, None) == mcl.MCL_EINVAL and b"lookup must be" in lib.mcl_last_error()
    assert lib.mcl_job_bytes(0, 5) == 0
    assert lib.mcl_map_bytes(None) == 0
    assert lib.mcl_job_bytes(1000, 28800) > 1000 * 120
    bad = mcl.LaunchConfig(3, 0)
    assert lib.mcl_set_launch_config(0, 1000, 1000, C.byref(bad)) == mcl.MCL_EINVAL
    assert lib.mcl_set_launch_config(5, 1000, 1000, None) == mcl.MCL_EINVAL
    assert lib.mcl_autotune(None, None, 0, None, 0, 0.1, None, None, None) == mcl.MCL_EINVAL
    # the one-launch weights limit: [0, 4096], host state only
    prev = mcl.get_weights_fused_max()
    assert prev == 4096
    assert lib.mcl_set_weights_fused_max(-1) == mcl.MCL_ERANGE
    assert lib.mcl_set_weights_fused_max(4097) == mcl.MCL_ERANGE
    assert mcl.get_weights_fused_max() == prev
    assert mcl.set_weights_fused_max(1000) == prev and mcl.get_weights_fused_max() == 1000
    assert mcl.set_weights_fused_max(prev) == 1000
    # the spatial order's threshold: any value, negative turns it off; host state only
    prev = mcl.get_spatial_order_min()
    assert prev == 1 << 30
    assert lib.mcl_set_spatial_order_min(-1) == mcl.MCL_OK and mcl.get_spatial_order_min() == -1
    assert mcl.set_spatial_order_min(0) == -1 and mcl.get_spatial_order_min() == 0
    assert mcl.set_spatial_order_min(prev) == 0 and mcl.get_spatial_order_min() == prev
    # measurement calls: NULL arguments, sizes, sinks shorter than the grid
    assert lib.mcl_bench_gather_offsets(None, P(0x1000), 10, P(0x2000), 10, 0, P(0x3000), None) == mcl.MCL_EINVAL
    assert lib.mcl_bench_gather_replay(P(0x1000), P(0x2000), 100, 10, 1, 1, 1, P(0x3000), 256, None) == mcl.MCL_EINVAL
    assert lib.mcl_bench_line_gather(P(0x1000), 1 << 20, 14, 64, 4, 1, 1, 8, P(0x2000), 8 * 256, None) == mcl.MCL_EINVAL
    assert b"exceed the region" in lib.mcl_last_error()
    assert lib.mcl_bench_line_gather(P(0x1000), 1 << 30, 14, 3, 4, 1, 1, 8, P(0x2000), 8 * 256, None) == mcl.MCL_EINVAL
    assert lib.mcl_bench_l1_gather(P(0x1000), 4096, 4, 2, 1, 8, P(0x2000), 8 * 256, None) == mcl.MCL_EINVAL
    assert lib.mcl_bench_l1_gather(P(0x1000), 8192, 4, 2, 1, 8, P(0x2000), 100, None) == mcl.MCL_EINVAL
    assert lib.mcl_bench_stream_read(P(0x1000), 17, 8, P(0x2000), 8 * 256, None) == mcl.MCL_EINVAL


def test_binding_constants_match_the_header(mcl):
    """Status codes, flags and limits the binding uses are the header's."""
    text = open(HEADER).read()
    want = {"MCL_OK": mcl.MCL_OK, "MCL_EINVAL": mcl.MCL_EINVAL, "MCL_ENOMEM": mcl.MCL_ENOMEM,
            "MCL_EDEVICE": mcl.MCL_EDEVICE, "MCL_ERANGE": mcl.MCL_ERANGE, "MCL_EBUSY": mcl.MCL_EBUSY,
            "MCL_TICK_GRAPH": mcl.TICK_GRAPH, "MCL_TICK_NOWAIT": mcl.TICK_NOWAIT, "MCL_MAX_JOBS": mcl.MAX_JOBS,
            "MCL_LOOKUP_NEAREST": mcl.LOOKUP_NEAREST, "MCL_LOOKUP_TRILINEAR": mcl.LOOKUP_TRILINEAR,
            "MCL_SCORE_PRODUCT": mcl.SCORE_PRODUCT, "MCL_SCORE_SUM": mcl.SCORE_SUM,
            "MCL_WQ_SHIFT": mcl.WQ_SHIFT}
    for name, val in want.items():
        m = re.search(r"#define\s+" + name + r"\s+\(?(-?\d+)\)?", text)
        assert m and int(m.group(1)) == val, name
    for name, val in (("MCL_MAX_PARTICLES", mcl.MAX_PARTICLES), ("MCL_MAX_POINTS", mcl.MAX_POINTS)):
        m = re.search(r"#define\s+" + name + r"\s+\(1 << (\d+)\)", text)
        assert m and 1 << int(m.group(1)) == val, name


def test_binding_structs_match_the_header(mcl, tmp_path):
    """The ctypes mirrors of the header's structs have its sizes and field
    offsets (a C program built from the header with gcc prints them)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = {"mcl_map_desc": mcl.MapDesc, "mcl_filter_job": mcl.FilterJob, "mcl_launch_config": mcl.LaunchConfig}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "mcl.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'    printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_tune_cache_is_read_back(tmp_path):
    """Launch settings persisted by the tuner (MCL_TUNE_CACHE) are read back by a
    new process on the same kind of GPU and ignored for another; later lines
    win.  Run in a child process (the cache is read at the first lookup); with
    no GPU the library tags the device "unknown"."""
    import subprocess
    import sys
    cache = tmp_path / "tune.txt"
    cache.write_text("unknown 0 15 20 2 8 1 4 5\n"        # int16, K class 2^15, N class 2^20
                     "gfx000/1 0 15 20 8 16 2 64 3\n"     # another GPU: ignored
                     "unknown 1 10 10 8 0 0 2 0\n"
                     "unknown 1 10 10 2 4 0 1 7\n")       # later line wins
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2310_04172_amd import mcl\n"
            "print(mcl.get_launch_config('i16', 28660, 1000000))\n"
            "print(mcl.get_launch_config('i8', 1000, 600))\n"
            "print(mcl.get_launch_config('f32', 1000, 600))\n") % ROOT
    env = dict(os.environ, MCL_TUNE_CACHE=str(cache), HIP_VISIBLE_DEVICES="")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, check=True).stdout
    lines = out.strip().splitlines()
    assert lines == ["(2, 8, 1, 4, 5)", "(2, 4, 0, 1, 7)", "(4, 0, 0, 0, 0)"], out


def test_c_consumer_builds(tmp_path):
    """The plain-C consumer (tests/c/mcl_consumer.c: mcl.h and the HIP runtime's
    C API only) compiles as C11 without warnings and links to the library; the
    GPU test runs it."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    if gcc is None or not os.path.exists(os.path.join(rocm, "include", "hip", "hip_runtime_api.h")):
        pytest.skip("gcc or the HIP headers not available")
    pkg = os.path.join(ROOT, "paper_2310_04172_amd")
    r = subprocess.run([gcc, "-std=c11", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
                        f"-I{rocm}/include", f"-I{os.path.join(ROOT, 'include')}",
                        os.path.join(ROOT, "tests", "c", "mcl_consumer.c"), "-o", str(tmp_path / "mcl_consumer"),
                        f"-L{rocm}/lib", "-lamdhip64", f"-L{pkg}", "-lmcl"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
