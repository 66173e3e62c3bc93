"""Comparisons of the HIP path's outputs with the CPU oracle, shared by the GPU
tests (no method arithmetic here: every expected value comes from `oracle`).

Bars:
 * log-weights within 1e-5 relative of the oracle (float32 sums of squares
   along a fixed tree; the derivation is in the sensor kernel's header); for
   the sum reading, within the absolute bound of sum_logw_tol;
 * normalisation, fed the same float32 log-weights on both sides: log Z and the
   weights within the float64 bound below, the fixed-point weights within one
   unit plus that bound;
 * resampling, fed the same fixed-point weights: ancestor indices and gathered
   poses bit for bit.
"""

from __future__ import annotations

import math

import numpy as np

RTOL_LOGW = 1e-5
U64 = 2.0 ** -53     # unit roundoff of float64


def assert_logw_close(gpu, ref, what=""):
    ref = np.asarray(ref, np.float64)
    err = np.abs(np.asarray(gpu).astype(np.float64) - ref)
    bad = err > RTOL_LOGW * np.abs(ref)
    assert not bad.any(), f"{what}: {bad.sum()} particles off, worst rel {np.max(err / np.maximum(np.abs(ref), 1e-300))}"


def sum_logw_tol(tau, sigma, ref):
    """Absolute bound on the sum reading's float32 log-weights, per particle.

    Each likelihood 2^(k2 q^2): q^2 and k2 q^2 round once each and k2 once from
    float64, so the exponent is off by at most 3 u |k2 q^2| (u = 2^-24), i.e. the
    term by 3 u c q^2 <= 3 u tau^2 / (2 sigma^2) relative; the exponential adds 2
    ulps.  The positive terms are summed along the product reading's tree: 15
    roundings in a lane, 6 in the butterfly, 3 over a piece's chunks, at most 8
    over the pieces: 32 u relative on S.  log S then carries S's relative error
    as an absolute one, plus 2 ulps of log and 1 of the float32 result.  Total:
    36 u + 3 u tau^2 / (2 sigma^2) + 3 u |l|."""
    u = 2.0 ** -24
    r = float(tau) ** 2 / (2.0 * float(sigma) ** 2)
    return 36 * u + 3 * u * r + 3 * u * np.abs(np.asarray(ref, np.float64))


def assert_sum_logw_close(gpu, ref, tau, sigma, what=""):
    ref = np.asarray(ref, np.float64)
    err = np.abs(np.asarray(gpu).astype(np.float64) - ref)
    tol = sum_logw_tol(tau, sigma, ref)
    bad = err > tol
    assert not bad.any(), f"{what}: {bad.sum()} particles off, worst {np.max(err - tol):.3g} above the bound"


def normalize_bounds(lw32, lz_ref):
    """(tol on log Z, relative tol on w) for a float32 log-weight vector.

    The oracle's S is within 2u of the exact sum of its terms (compensated sum),
    each term within 1 ulp of its exponential.  The GPU adds each thread's 16
    terms in order, then a tree of depth 8 per block of 4096, then scales each
    block sum by exp(m_b - m) (2 roundings) and adds the block sums, at most 2
    per thread for N <= 2^21, in another tree of depth 8: at most 36 roundings
    on the way of any term, each term within 2 ulps.  All terms are positive, so
    the two S differ by at most (36 + 2 + 2 + 1) u relative, and log S by as
    much in absolute terms; the log and m + log S round once on each side.
    Weights: the exponent l_n - log Z differs by the log Z bound plus one
    rounding of the subtraction on each side, and exp adds 2 ulps per side."""
    lw32 = np.asarray(lw32, np.float32)
    log_s = lz_ref - float(lw32.max())
    tol_lz = 41 * U64 + np.spacing(abs(log_s)) + np.spacing(abs(lz_ref))
    rtol_w = tol_lz + np.spacing(np.max(np.abs(lw32.astype(np.float64) - lz_ref))) + 4 * U64
    return tol_lz, rtol_w


def check_normalize(oracle, lw32, wq, lz=None, w=None, what=""):
    """The GPU's normalisation of the float32 log-weights lw32 against the
    oracle's on the same input.  Returns the oracle's fixed-point weights."""
    lw32 = np.ascontiguousarray(lw32, np.float32)
    w_ref, wq_ref, lz_ref = oracle.normalize(lw32.astype(np.float64))
    tol_lz, rtol_w = normalize_bounds(lw32, lz_ref)
    if lz is not None:
        assert abs(float(lz) - lz_ref) <= tol_lz, f"{what}: log Z {float(lz)} vs {lz_ref} (tol {tol_lz})"
    if w is not None:
        np.testing.assert_allclose(w, w_ref, rtol=rtol_w, atol=1e-300, err_msg=what)
    diff = np.abs(np.asarray(wq).astype(np.int64) - wq_ref.astype(np.int64))
    assert np.all(diff <= 1 + rtol_w * wq_ref.astype(np.float64)), f"{what}: fixed-point weights off"
    return wq_ref


def check_resample(oracle, wq, seed, tick, idx, poses_in=None, poses_out=None, what=""):
    """The GPU's ancestors for the fixed-point weights wq (the GPU's own, so that
    identical W go in on both sides) against the oracle's, bit for bit; the
    gathered poses must be the indexed input poses exactly."""
    idx_ref = oracle.resample_seeded(np.ascontiguousarray(wq, np.uint64), seed, tick)
    assert np.array_equal(np.asarray(idx), idx_ref), f"{what}: resampled indices differ"
    if poses_out is not None:
        assert np.array_equal(np.asarray(poses_out), np.asarray(poses_in)[:, idx_ref]), f"{what}: gathered poses differ"


def check_update(oracle, tmap, points, poses_in, sigma, logw, wq, lz, idx, seed, tick, sub,
                 poses_out=None, w=None, what="", trilinear=False):
    """One filter update (sensor, normalise, resample) against the oracle:
    log-weights of the particles `sub` (indices) within 1e-5, the whole
    normalisation within its bound on the GPU's log-weights, the whole
    resampling bit for bit on the GPU's fixed-point weights."""
    pts = np.ascontiguousarray(points, np.float32)
    ps = np.ascontiguousarray(np.asarray(poses_in)[:, sub], np.float32)
    fn = oracle.sensor_update_trilinear if trilinear else oracle.sensor_update
    ref = fn(tmap, pts, ps, sigma)
    assert_logw_close(np.asarray(logw)[sub], ref, f"{what} log-weights")
    check_normalize(oracle, logw, wq, lz, w, what)
    check_resample(oracle, wq, seed, tick, idx, poses_in, poses_out, what)


def check_estimate(g_mean, g_best, g_best_pose, w, P, what=""):
    """The GPU's pose estimate (mean [12] float64, best index, best pose [12]
    float32) of weights w and poses P against the oracle: best index and pose
    bit for bit, the mean within a bound from the float64 arithmetic.

    Both sides add the same products in different orders: the library's
    summation tree is at most 4 + 6 + 4 levels per block and 8 + 6 + 4 across
    blocks, numpy's pairwise sum at most 8 + log2(N / 8) levels, so each sum
    differs by at most 64 u sum|terms|.  A perturbation dS of S moves the
    nearest rotation by at most 2 |dS|_F / (s2 + s3') (s3' carrying the sign of
    det S), and a backward-stable 4x4 eigensolver adds a few u |K| over the same
    gap.  Where that bound is not small (S near a repeated case) the rotation
    is not unique; there both sides must reach the same value of trace(R^T S).
    Returns the oracle's mean."""
    from oracle import estimate as E
    o_mean, o_b, o_bp = E.pose_estimate(w, P)
    assert int(g_best) == o_b, (what, g_best, o_b)
    assert np.array_equal(np.asarray(g_best_pose, np.float32).view(np.uint32), o_bp.view(np.uint32)), what

    ws, S, _ = E.weighted_sums(w, P)
    Pd = np.asarray(P).astype(np.float64)
    wu = np.asarray(w, np.float64) if np.sum(w) > 0 else np.ones(Pd.shape[1])
    absS = (np.abs(Pd[0:9]) * wu).sum(axis=1)
    absT = (np.abs(Pd[9:12]) * wu).sum(axis=1)
    dS = 64 * U64 * absS                                   # per element
    s = np.linalg.svd(S, compute_uv=False)
    s3 = s[2] if np.linalg.det(S) >= 0 else -s[2]
    gap = s[1] + s3
    tol_R = (2 * np.linalg.norm(dS) + 32 * U64 * 3 * s[0]) / gap if gap > 0 else np.inf
    tol_t = 2 * 64 * U64 * absT / ws + 4 * U64 * np.abs(o_mean[9:12])
    np.testing.assert_array_less(np.abs(g_mean[9:12] - o_mean[9:12]), tol_t + 1e-300, err_msg=what)

    Rg = np.asarray(g_mean[:9]).reshape(3, 3)
    np.testing.assert_allclose(Rg @ Rg.T, np.eye(3), atol=1e-13, err_msg=what)
    assert np.linalg.det(Rg) > 0, what
    if tol_R < 1e-6:
        err = np.abs(g_mean[:9] - o_mean[:9]).max()
        assert err <= tol_R, (what, err, tol_R)
    else:
        f_o = np.trace(o_mean[:9].reshape(3, 3).T @ S)
        f_g = np.trace(Rg.T @ S)
        tol_f = 2 * math.sqrt(3) * np.linalg.norm(dS) + 64 * U64 * 3 * s[0]
        assert f_g >= f_o - tol_f, (what, f_g, f_o, tol_f)
    return o_mean
