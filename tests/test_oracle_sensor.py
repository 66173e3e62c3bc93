"""Pins for the oracle's sensor update (transform, voxel lookup, Eq. 3 score).

Each test checks the oracle against something it does not compute itself:
exact rational geometry, closed forms on lattice-aligned inputs, exact
symmetries of the voxel grid, and the analytic signed distance of the scene the
map was voxelised from (with a rigorous Lipschitz error bound).
"""

import math
from fractions import Fraction
from fractions import Fraction as F

import numpy as np
import pytest

from tests.helpers import identity_poses, make_map, poses_from, random_rotations
from workloads.scene import Scene
from workloads.tsdf import build_map, f32

SQ3_2 = math.sqrt(3.0) / 2.0


def score_const(tmap, sigma):
    s = 1.0 if tmap.dtype in ("f32", "f64") else float(tmap.tau) / tmap.Q
    return (s * s) / (2.0 * float(sigma) ** 2)


# ----------------------------------------------------------------- geometry
def test_voxel_index_matches_exact_geometry(oracle_lib):
    """Away from cell faces, the float32 recipe must select the voxel that exactly
    contains R p + t: pins rotation layout (row-major R, not R^T), translation,
    origin, voxel size, bounds and the x-fastest linear index."""
    rng = np.random.default_rng(11)
    dims = (16, 12, 10)
    tmap = make_map(np.zeros(dims[::-1], np.int16), 0.1, origin=(-0.35, 0.2, -0.15))
    n_pose, K = 6, 300
    R = random_rotations(rng, n_pose)
    t = rng.uniform([-0.3, 0.2, -0.15], [1.2, 1.3, 0.8], size=(n_pose, 3))
    poses = poses_from(R, t)
    pts = rng.uniform(-1.0, 1.0, size=(3, K)).astype(np.float32)
    lin = oracle_lib.voxel_indices(tmap, pts, poses)
    v = F(float(tmap.voxel))
    o = [F(float(x)) for x in tmap.origin]
    checked = inside_count = 0
    for n in range(n_pose):
        Rn = [[F(float(poses[3 * j + a, n])) for a in range(3)] for j in range(3)]
        tn = [F(float(poses[9 + j, n])) for j in range(3)]
        for k in range(K):
            p = [F(float(pts[a, k])) for a in range(3)]
            g = [(sum(Rn[j][a] * p[a] for a in range(3)) + tn[j] - o[j]) / v for j in range(3)]
            if any(abs(gj - round(gj)) < F(1, 1000) for gj in g):
                continue
            fl = [math.floor(gj) for gj in g]
            inside = all(0 <= fl[j] < dims[j] for j in range(3))
            expect = fl[0] + dims[0] * (fl[1] + dims[1] * fl[2]) if inside else -1
            assert lin[n, k] == expect, (n, k, g)
            checked += 1
            inside_count += inside
    assert checked > 0.95 * n_pose * K
    assert 0.2 * checked < inside_count < 0.9 * checked


def test_cell_faces_are_half_open(oracle_lib):
    """A point exactly on a face belongs to the upper cell; the far face is outside;
    a point of -0.0 under the identity pose is in voxel 0; NaN is outside."""
    nx, ny, nz = 4, 3, 2
    v = 0.125
    tmap = make_map(np.zeros((nz, ny, nx), np.int16), v)
    pts = np.array([[0.0, v, 3 * v, 4 * v, -0.0, np.nan, 0.5 * v],
                    [0.0, 0.0, 2 * v, 0.0, 0.0, 0.0, 3 * v],
                    [0.0, v, v, 0.0, 0.0, 0.0, 0.0]], np.float32)
    lin = oracle_lib.voxel_indices(tmap, pts, identity_poses(1))[0]
    assert list(lin) == [0, 1 + nx * (0 + ny * 1), 3 + nx * (2 + ny * 1), -1, 0, -1, -1]


def test_negative_zero_grid_coordinate_is_inside(oracle_lib):
    """Translation -0.0 at a zero origin and a point of -0.0 select voxel 0, as
    +0.0 does (the recipe maps an offset of -0.0 to +0.0)."""
    tmap = make_map(np.zeros((2, 2, 2), np.int16), 0.125)
    poses = identity_poses(1)
    poses[9:, 0] = -0.0
    pts = np.array([[-0.0], [-0.0], [-0.0]], np.float32)
    assert oracle_lib.voxel_indices(tmap, pts, poses)[0, 0] == 0


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("dtype", ["i16", "i8", "f32", "f64"])
def test_identity_pose_exact_score(oracle_lib, dtype):
    """Identity pose, dyadic voxel, points at voxel centres: indices are known
    integers and the score is the closed form -c * sum q^2 (exact integer sum)."""
    rng = np.random.default_rng(5)
    nx, ny, nz = 8, 6, 5
    v, tau, sigma = 0.125, 0.3, f32(0.11)
    if dtype in ("f32", "f64"):
        vals = rng.uniform(-tau, tau, size=(nz, ny, nx)).astype(np.float32 if dtype == "f32" else np.float64)
    else:
        lim = 127 if dtype == "i8" else 32767
        vals = rng.permutation(np.linspace(-lim, lim, nx * ny * nz).round()).reshape(nz, ny, nx)
        vals = vals.astype(np.int8 if dtype == "i8" else np.int16)
    tmap = make_map(vals, v, tau=tau, dtype=dtype)
    K = 257
    ii, jj, kk = rng.integers(0, nx, K), rng.integers(0, ny, K), rng.integers(0, nz, K)
    pts = ((np.stack([ii, jj, kk]).astype(np.float64) + 0.5) * v).astype(np.float32)
    lw, S = oracle_lib.sensor_update(tmap, pts, identity_poses(1), sigma, return_sum=True)
    q = vals[kk, jj, ii].astype(np.float64)
    if dtype in ("f32", "f64"):
        expect = math.fsum(float(x) * float(x) for x in q)
        assert abs(S[0] - expect) <= 1e-14 * expect
    else:
        expect = sum(int(x) * int(x) for x in q)
        assert S[0] == expect
    c = score_const(tmap, sigma)
    assert lw[0] == pytest.approx(-expect * c, rel=1e-15)
    # single-point scans: each l is exactly -c q^2 of its own voxel
    for k in range(0, K, 37):
        l1, s1 = oracle_lib.sensor_update(tmap, pts[:, k:k + 1], identity_poses(1), sigma, return_sum=True)
        assert s1[0] == float(q[k]) ** 2


def test_empty_scan_and_all_outside(oracle_lib):
    rng = np.random.default_rng(2)
    vals = rng.integers(-32767, 32768, size=(4, 4, 4)).astype(np.int16)
    tmap = make_map(vals, 0.1, tau=0.3)
    sigma = f32(0.15)
    poses = poses_from(random_rotations(rng, 3), rng.uniform(0, 0.4, (3, 3)))
    lw = oracle_lib.sensor_update(tmap, np.zeros((3, 0), np.float32), poses, sigma)
    assert np.all(lw == 0.0)
    far = np.full((3, 50), 1e4, np.float32)
    lw, S = oracle_lib.sensor_update(tmap, far, poses, sigma, return_sum=True)
    assert np.all(S == 50 * 32767 ** 2)
    np.testing.assert_allclose(lw, -50 * 32767 ** 2 * score_const(tmap, sigma), rtol=1e-15)


def test_particle_permutation_and_threads(oracle_lib):
    """Particles are independent: permuting them permutes l bit for bit, and the
    multi-threaded split gives the single-threaded result."""
    rng = np.random.default_rng(8)
    vals = rng.integers(-32767, 32768, size=(10, 12, 14)).astype(np.int16)
    tmap = make_map(vals, 0.1, tau=0.3)
    N = 37
    poses = poses_from(random_rotations(rng, N), rng.uniform(0, 1.0, (N, 3)))
    pts = rng.uniform(-0.6, 0.6, size=(3, 211)).astype(np.float32)
    lw = oracle_lib.sensor_update(tmap, pts, poses, f32(0.15))
    perm = rng.permutation(N)
    lw_p = oracle_lib.sensor_update(tmap, pts, np.ascontiguousarray(poses[:, perm]), f32(0.15))
    assert np.array_equal(lw_p, lw[perm])
    lw_t = oracle_lib.sensor_update(tmap, pts, poses, f32(0.15), nthreads=5)
    assert np.array_equal(lw_t, lw)


# ------------------------------------------------------------ exact symmetry
def _signed_perm(rng):
    P = np.zeros((3, 3))
    P[np.arange(3), rng.permutation(3)] = rng.choice([-1.0, 1.0], size=3)
    return P


def _move_map(vals, origin, v, P, d):
    """Map B with B(P x + d) = A(x) for a signed axis permutation P and a shift d
    that is a whole number of voxels; exact integer bookkeeping in half-voxels."""
    nz, ny, nx = vals.shape
    n = np.array([nx, ny, nz])
    o = np.asarray(origin) / v
    corners = np.stack([P @ o + d / v, P @ (o + n) + d / v])
    o_b = corners.min(axis=0)
    n_b = np.abs(P) @ n
    ib = np.stack(np.meshgrid(*[np.arange(int(m)) for m in n_b], indexing="ij"), -1).reshape(-1, 3)
    xb2 = 2 * (o_b + ib) + 1                      # centres of B, in half voxels
    xa2 = (P.T @ (xb2 - 2 * d / v).T).T           # back to A's frame
    ia = ((xa2 - 2 * o - 1) / 2).round().astype(int)
    out = np.empty((int(n_b[2]), int(n_b[1]), int(n_b[0])), vals.dtype)
    out[ib[:, 2], ib[:, 1], ib[:, 0]] = vals[ia[:, 2], ia[:, 1], ia[:, 0]]
    return out, tuple(o_b * v)


def test_rigid_motion_invariance_exact(oracle_lib):
    """Grid symmetries (signed axis permutations, whole-voxel shifts) applied to both
    the map and the particle poses leave every sum of squares exactly unchanged.
    All float32 operations are exact on these lattice inputs, so this pins the
    transform, the index and the bounds handling bit for bit."""
    rng = np.random.default_rng(21)
    v, tau = 0.25, 0.75
    vals = rng.integers(-32767, 32768, size=(7, 9, 11)).astype(np.int16)
    origin = (-1.0, 0.5, -0.75)
    tA = make_map(vals, v, origin=origin, tau=tau)
    N, K = 24, 180
    Rs = np.stack([_signed_perm(rng) for _ in range(N)])
    ts = v * rng.integers(-2, 8, size=(N, 3)).astype(np.float64)
    poses = poses_from(Rs, ts)
    frac = rng.choice([0.25, 0.5, 0.75], size=(3, K))
    pts = (v * (rng.integers(-6, 6, size=(3, K)) + frac)).astype(np.float32)
    lA, SA = oracle_lib.sensor_update(tA, pts, poses, f32(0.3), return_sum=True)
    for trial in range(4):
        P = _signed_perm(rng)
        d = v * rng.integers(-5, 6, size=3).astype(np.float64)
        vb, ob = _move_map(vals, origin, v, P, d)
        tB = make_map(vb, v, origin=ob, tau=tau)
        RB = np.einsum("ij,njk->nik", P, Rs)
        tBt = ts @ P.T + d
        lB, SB = oracle_lib.sensor_update(tB, pts, poses_from(RB, tBt), f32(0.3), return_sum=True)
        assert np.array_equal(SA, SB), trial
    # the test is not vacuous: some points land inside, some outside
    lin = oracle_lib.voxel_indices(tA, pts, poses)
    assert 0.1 < np.mean(lin >= 0) < 0.9


# ------------------------------------------------------- analytic scene bound
def _sphere_scene(centres, radii):
    return Scene(spheres=np.column_stack([centres, radii]))


def _analytic_logw(scene, tau, pts, poses, c_metric):
    """l from the exact SDF at the exact transformed point (float64), clamped."""
    out = np.empty(poses.shape[1])
    bound = np.empty(poses.shape[1])
    P = pts.astype(np.float64)
    dan = []
    for n in range(poses.shape[1]):
        R = poses[:9, n].astype(np.float64).reshape(3, 3)
        t = poses[9:, n].astype(np.float64)
        x = (R @ P).T + t
        d = np.clip(scene.sdf(x), -tau, tau)
        out[n] = -c_metric * np.sum(d * d)
        dan.append(d)
    return out, dan


def _lipschitz_bound(dan, delta, c_metric):
    # |d_vox - d_an| <= delta per point, so |d_vox^2 - d_an^2| <= delta (2|d_an| + delta)
    return np.array([c_metric * np.sum(delta * (2 * np.abs(d) + delta)) for d in dan])


def test_analytic_scene_bound_and_rigid_motion(oracle_lib):
    """Voxelised l stays within a rigorous bound of the analytic l (the SDF is
    1-Lipschitz: |d_vox - d| <= v sqrt(3)/2 + s/2), and moving map and poses by
    the same arbitrary rigid motion keeps both within that bound.  Points sit on
    the spheres' surfaces (and a few off them), so the bound is tight: a wrong
    transform shifts l by far more than the bound (checked too)."""
    rng = np.random.default_rng(3)
    v, tau = 0.05, 0.2
    dims = (48, 48, 40)
    ext = np.array(dims) * v
    centre = ext / 2
    cA = centre + rng.uniform(-0.35, 0.35, size=(4, 3))
    rad = rng.uniform(0.15, 0.3, size=4)
    sA = _sphere_scene(cA, rad)
    mA = build_map(sA, dims, v, (0, 0, 0), tau, "i16")
    sigma = f32(tau / 2)
    s = float(mA.tau) / 32767
    c_metric = 1.0 / (2.0 * float(sigma) ** 2)
    delta = float(mA.voxel) * (SQ3_2 + 1e-3) + s / 2
    # world points on the surfaces, plus 20 % jittered off them
    K = 400
    which = rng.integers(0, 4, K)
    dirs = rng.normal(size=(K, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    xw = cA[which] + rad[which, None] * dirs
    xw[: K // 5] += rng.normal(0, 0.05, size=(K // 5, 3))
    # a particle at a random pose near the centre; scan points in its sensor frame
    N = 6
    Rs = random_rotations(rng, N)
    ts = centre + rng.uniform(-0.2, 0.2, size=(N, 3))
    poses = poses_from(Rs, ts)
    R0 = poses[:9, 0].astype(np.float64).reshape(3, 3)
    t0 = poses[9:, 0].astype(np.float64)
    pts = ((xw - t0) @ R0).T.astype(np.float32)        # R0^T (x - t0)
    lA = oracle_lib.sensor_update(mA, pts, poses, sigma)
    anA, danA = _analytic_logw(sA, float(mA.tau), pts, poses, c_metric)
    bA = _lipschitz_bound(danA, delta, c_metric)
    assert np.all(np.abs(lA - anA) <= bA)
    # discriminating: the true pose (particle 0) scores best on both sides, and a transposed rotation (a plausible layout mistake) breaks the bound
    assert np.argmax(anA) == 0 and np.argmax(lA) == 0
    posesT = poses.copy()
    posesT[:9] = poses[:9].reshape(3, 3, N).transpose(1, 0, 2).reshape(9, N)
    lT = oracle_lib.sensor_update(mA, pts, posesT, sigma)
    assert abs(lT[0] - anA[0]) > bA[0]

    # arbitrary rigid motion of world (scene) and poses together
    Rm = random_rotations(rng, 1)[0]
    dm = rng.uniform(-0.1, 0.1, size=3)
    move = lambda x: (x - centre) @ Rm.T + centre + dm
    sB = _sphere_scene(move(cA), rad)
    mB = build_map(sB, dims, v, (0, 0, 0), tau, "i16")
    RB = np.einsum("ij,njk->nik", Rm, poses[:9].T.reshape(N, 3, 3).astype(np.float64))
    tB = move(poses[9:].T.astype(np.float64))
    posesB = poses_from(RB, tB)
    lB = oracle_lib.sensor_update(mB, pts, posesB, sigma)
    anB, danB = _analytic_logw(sB, float(mB.tau), pts, posesB, c_metric)
    bB = _lipschitz_bound(danB, delta, c_metric)
    # posesB are rounded to float32, so the analytic values move by rounding only
    np.testing.assert_allclose(anB, anA, rtol=1e-3, atol=1e-2 * c_metric * delta ** 2 * K)
    assert np.all(np.abs(lB - anB) <= bB)
    assert np.all(np.abs(lB - lA) <= bA + bB + np.abs(anB - anA))


# ------------------------------------------------- the index recipe, exactly
def _round_f32(x: Fraction, neg_zero: bool = False) -> float:
    """Nearest float32 to an exact rational (ties to even), as a Python float;
    a zero result takes the sign of x (or neg_zero for an exact zero)."""
    if x == 0:
        return -0.0 if neg_zero else 0.0
    s = -1 if x < 0 else 1
    a = abs(x)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    e = max(e, -126)
    ulp = Fraction(2) ** (e - 23)
    q = round(a / ulp)                       # Fraction.__round__: half to even
    if q == 0:
        return -0.0 if s < 0 else 0.0
    r = float(q * ulp)
    if r >= 2.0 ** 128 - 2.0 ** 103:         # beyond the largest float32 after rounding
        r = math.inf
    return s * r


def _fma32(a, b, c) -> float:
    a, b, c = float(a), float(b), float(c)
    exact = Fraction(a) * Fraction(b) + Fraction(c)
    both_neg_zero = (exact == 0 and math.copysign(1, a) * math.copysign(1, b) < 0 and math.copysign(1, c) < 0)
    return _round_f32(exact, neg_zero=both_neg_zero)


def _index_exact(tmap, pose, p):
    inv_v = np.float32(1.0 / float(tmap.voxel))
    dims = (tmap.nx, tmap.ny, tmap.nz)
    ijk = []
    for j in range(3):
        a = [np.float32(np.float32(pose[3 * j + k]) * inv_v) for k in range(3)]
        b = np.float32(np.float32(np.float32(pose[9 + j]) - np.float32(tmap.origin[j])) * inv_v) + np.float32(0.0)
        g = _fma32(a[0], p[0], b)
        g = _fma32(a[1], p[1], g)
        g = _fma32(a[2], p[2], g)
        if math.copysign(1.0, g) < 0 or not (g < dims[j]):
            return -1
        ijk.append(int(g))
    return ijk[0] + tmap.nx * (ijk[1] + tmap.ny * ijk[2])


def test_index_recipe_against_exact_rational_fma(oracle_lib):
    """Every fused multiply-add of the recipe redone in exact rational arithmetic
    with one rounding to float32: indices bit for bit, on random rotations and on
    points placed on and next to cell faces (where one rounding more or less, or
    another operation order, changes the voxel)."""
    rng = np.random.default_rng(17)
    nx, ny, nz = 9, 7, 5
    v = 0.1
    tmap = make_map(np.zeros((nz, ny, nx), np.int16), v, origin=(-0.35, 0.2, -0.15))
    R = random_rotations(rng, 6)
    t = rng.uniform(-0.1, 0.1, (6, 3))
    poses = poses_from(R, t)
    # points whose world image lands exactly on faces for the first pose
    face = []
    for _ in range(200):
        ijk = rng.integers(0, [nx + 1, ny + 1, nz + 1])
        xw = np.asarray(tmap.origin) + ijk * float(np.float32(v))
        face.append(R[0].T @ (xw - t[0]))
    pts = np.concatenate([np.array(face).T, rng.uniform(-0.6, 0.6, (3, 200))], axis=1).astype(np.float32)
    # nudge a third of the points by one ulp
    pts[:, ::3] = np.nextafter(pts[:, ::3], np.float32(np.inf))
    lin = oracle_lib.voxel_indices(tmap, pts, poses)
    for n in range(poses.shape[1]):
        for k in range(pts.shape[1]):
            assert lin[n, k] == _index_exact(tmap, poses[:, n], pts[:, k]), (n, k)


def test_negative_zero_from_underflow_is_outside(oracle_lib):
    """A negative exact coordinate too small for float32 rounds to -0.0 in the
    fused recipe; it lies below 0 and reads outside.  The same magnitude with a
    positive sign rounds to +0.0 and is inside."""
    tmap = make_map(np.zeros((2, 2, 2), np.int16), 0.125)
    poses = identity_poses(2)
    poses[2, 0] = np.float32(-1e-30)       # r02: a tiny coupling of z into x,
    poses[2, 1] = np.float32(1e-30)        # negative, then positive
    pts = np.array([[0.0], [0.0], [1e-30]], np.float32)
    lin = oracle_lib.voxel_indices(tmap, pts, poses)
    assert lin[0, 0] == -1 and lin[1, 0] == 0
    assert _index_exact(tmap, poses[:, 0], pts[:, 0]) == -1
    assert _index_exact(tmap, poses[:, 1], pts[:, 0]) == 0
