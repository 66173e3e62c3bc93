"""The seeded input generator: determinism, exact ray casts, voxelisation, quantisation."""

import numpy as np

from workloads import configs
from workloads.scene import Scene, box_sdf, euler_zyx_to_matrix
from workloads.tsdf import build_map, f32, quantise, voxelise


def _small_scene():
    return configs.office_scene(configs.rng(99, 0), extent=(3.2, 3.2), floor_z=0.4, n_boxes=5,
                                side=(0.3, 1.0))


def test_config1_is_deterministic():
    a, b = configs.config1(64), configs.config1(64)
    assert np.array_equal(a.points, b.points) and np.array_equal(a.poses, b.poses)
    assert np.array_equal(a.tmap.values, b.tmap.values) and a.seed == b.seed
    assert a.points.dtype == np.float32 and a.poses.shape == (12, 64)
    assert 1000 < a.K < 16 * 360


def test_raycast_hits_lie_on_surfaces():
    sc = _small_scene()
    sc.cylinders = np.array([[2.2, 2.3, 0.25, 0.4, 3.0]])
    origin = np.array([1.6, 1.5, 1.2])
    assert sc.sdf(origin[None])[0] > 0
    dirs = configs.beam_dirs(16, 360, -30, 30)
    t = sc.raycast(origin, dirs)
    hit = np.isfinite(t)
    assert hit.mean() > 0.3
    x = origin + t[hit, None] * dirs[hit]
    assert np.max(np.abs(sc.sdf(x))) < 1e-9
    # nothing is hit before the reported distance: the SDF stays positive along the ray
    for frac in (0.25, 0.5, 0.9, 0.99):
        xm = origin + frac * t[hit, None] * dirs[hit]
        assert np.all(sc.sdf(xm) > 0)


def test_box_sdf_is_distance_outside():
    b = np.array([0.0, 0.0, 0.0, 1.0, 2.0, 0.5])
    rng = np.random.default_rng(0)
    p = rng.uniform(-1, 3, size=(500, 3))
    nearest = np.clip(p, b[:3], b[3:])
    outside = np.any((p < b[:3]) | (p > b[3:]), axis=1)
    d = box_sdf(p, b)
    np.testing.assert_allclose(d[outside], np.linalg.norm(p - nearest, axis=1)[outside], rtol=1e-12)
    assert np.all(d[~outside] <= 0)


def test_voxelise_matches_direct_evaluation_and_quantisation():
    sc = _small_scene()
    dims, v, tau = (32, 32, 20), f32(0.1), f32(0.3)
    d, _ = voxelise(sc, dims, v, (0, 0, 0), tau, "f64")
    c = (np.stack(np.meshgrid(*[np.arange(n) for n in dims], indexing="ij"), -1) + 0.5) * v
    direct = np.clip(sc.sdf(c.reshape(-1, 3)), -tau, tau).reshape(dims).transpose(2, 1, 0)
    np.testing.assert_allclose(d, direct, rtol=0, atol=1e-15)
    for dtype, Q in (("i16", 32767), ("i8", 127)):
        q = quantise(d, tau, dtype)
        assert np.max(np.abs(q.astype(np.float64) * tau / Q - d)) <= tau / Q / 2 * (1 + 1e-12)
        m = build_map(sc, dims, v, (0, 0, 0), tau, dtype)
        assert np.array_equal(m.values, q)


def test_euler_is_a_rotation():
    rng = np.random.default_rng(1)
    R = euler_zyx_to_matrix(*rng.uniform(-3, 3, size=(3, 50)))
    np.testing.assert_allclose(R @ R.transpose(0, 2, 1), np.broadcast_to(np.eye(3), R.shape), atol=1e-14)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, rtol=1e-14)
    # yaw only: rotation about z
    Rz = euler_zyx_to_matrix(0.0, 0.0, np.pi / 2)
    np.testing.assert_allclose(Rz @ np.array([1.0, 0, 0]), [0, 1, 0], atol=1e-15)


def test_free_voxel_particles_are_free():
    w = configs.config1(16)
    xyz, rpy = configs.free_voxel_particles(configs.rng(7, 3), w.tmap, 2000)
    ijk = np.floor((xyz - np.asarray(w.tmap.origin)) / w.tmap.voxel).astype(int)
    assert np.all(w.tmap.values[ijk[:, 2], ijk[:, 1], ijk[:, 0]] > 0)
    assert np.all(np.abs(rpy[:, :2]) <= 5 * np.pi / 180) and np.all(np.abs(rpy[:, 2]) <= np.pi)
