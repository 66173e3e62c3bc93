"""Pins for the oracle's weight normalisation and low-variance resampling.

Normalisation is checked against 40-digit decimal arithmetic and closed-form
special cases; resampling against exact counting identities of systematic
resampling (the multiplicity bound, and the expectation over every offset).
"""

import math
import os
from decimal import Decimal, getcontext

import numpy as np
import pytest

SCALE = 2 ** 42


# ------------------------------------------------------------ normalisation
def _decimal_reference(logw):
    getcontext().prec = 40
    D = [Decimal(float(x)) for x in logw]
    m = max(D)
    S = sum((d - m).exp() for d in D)
    lz = m + S.ln()
    return lz, [(d - lz).exp() for d in D]


@pytest.mark.parametrize("spread", [1.0, 30.0, 700.0, 5000.0])
def test_normalize_matches_high_precision(oracle_lib, spread):
    rng = np.random.default_rng(int(spread))
    logw = -np.abs(rng.normal(0, spread, 300)) - 1e4
    w, wq, lz = oracle_lib.normalize(logw)
    lz_ref, w_ref = _decimal_reference(logw)
    assert abs(Decimal(lz) - lz_ref) <= Decimal(4e-16) * abs(lz_ref)
    for a, b in zip(w, w_ref):
        if b > Decimal(1e-300):
            assert abs(Decimal(a) - b) <= Decimal(1e-11) * b
        else:
            assert a < 1e-290
    # W is the floor of w * 2^42 (an exact power-of-two scaling of w)
    assert all(int(q) == math.floor(x * SCALE) for q, x in zip(wq, w))
    # sum w = 1 up to the rounding of log Z (relative to |log Z|) and of each exp
    assert abs(math.fsum(w) - 1.0) <= (len(w) + 2 * abs(lz) + 2) * 2.0 ** -52


def test_normalize_special_cases(oracle_lib):
    N = 1000
    w, wq, lz = oracle_lib.normalize(np.full(N, -1234.5))
    # w = 1/N up to the rounding of log Z (about |log Z| ulp(1) relative)
    assert np.all(np.abs(w - 1.0 / N) <= (2 * abs(lz) + 4) * 2.0 ** -52 / N)
    assert np.all(wq == wq[0]) and wq[0] == math.floor(SCALE / N)
    assert lz == pytest.approx(-1234.5 + math.log(N), rel=1e-15)
    # one particle dominating by more than the float64 exp range: a one-hot weight
    lw = np.random.default_rng(1).uniform(-50, 0, N)
    lw[417] = 800.0
    w, wq, lz = oracle_lib.normalize(lw)
    assert w[417] == 1.0 and wq[417] == SCALE
    assert np.count_nonzero(w) == 1 and np.count_nonzero(wq) == 1
    # shifting every l by a constant leaves w unchanged up to rounding
    lw = np.random.default_rng(2).normal(0, 20, N)
    w1, _, lz1 = oracle_lib.normalize(lw)
    w2, _, lz2 = oracle_lib.normalize(lw + 3000.0)
    np.testing.assert_allclose(w1, w2, rtol=1e-11, atol=1e-300)
    assert lz2 - lz1 == pytest.approx(3000.0, rel=1e-14)


def test_normalize_sum_is_exact_for_many_small_terms(oracle_lib):
    """log Z is defined by the exact sum S: one particle at l = 0 and 10^6 at
    l = ln(1e-17) give S = 1 + 10^6 exp(ln 1e-17), log Z = log1p of the rest.
    Each small term is below half an ulp of 1, so a plain running sum stays at
    exactly 1 (log Z = 0); the oracle must see the 1e-11."""
    n = 10 ** 6
    small = math.log(1e-17)
    lw = np.full(n + 1, small)
    lw[0] = 0.0
    w, wq, lz = oracle_lib.normalize(lw)
    term = math.exp(small)            # the float64 term both sides add
    exact = math.log1p(n * term)      # about 1e-11
    # S itself is a float64 near 1, so log S is good to about an ulp of 1
    # absolute (a plain sum would be off by the whole 1e-11)
    assert abs(lz - exact) <= 2 * 2.0 ** -52
    assert w[0] == pytest.approx(1.0 / (1.0 + n * term), rel=1e-15)


def test_normalize_single_particle(oracle_lib):
    w, wq, lz = oracle_lib.normalize(np.array([-77.25]))
    assert w[0] == 1.0 and wq[0] == SCALE and lz == -77.25


# --------------------------------------------------------------- resampling
def _u_for_offset(r, T):
    """A 64-bit draw u whose offset floor(u T / 2^64) is exactly r."""
    u = -(-(r << 64) // T)
    assert (u * T) >> 64 == r and u < 2 ** 64
    return u


def _counts(idx, N):
    return np.bincount(idx, minlength=N)


def test_resample_expectation_over_all_offsets(oracle_lib):
    """Summed over every offset r in [0, T), particle i is drawn exactly N W_i times:
    each point of [0, N T) is m T + r for exactly one (slot m, offset r)."""
    rng = np.random.default_rng(4)
    for N in (1, 2, 3, 7, 16):
        W = rng.integers(0, 40, size=N).astype(np.uint64)
        W[rng.integers(0, N)] += 1
        T = int(W.sum())
        total = np.zeros(N, np.int64)
        for r in range(T):
            idx = oracle_lib.resample(W, _u_for_offset(r, T))
            total += _counts(idx, N)
        assert np.array_equal(total, N * W.astype(np.int64))


def test_resample_multiplicity_bounds(oracle_lib):
    """For every draw, floor(N W_i / T) <= count_i <= ceil(N W_i / T); the output is
    sorted, in range, and never picks a zero-weight particle."""
    rng = np.random.default_rng(9)
    for trial in range(30):
        N = int(rng.integers(1, 3000))
        W = rng.integers(0, 2 ** 30, size=N).astype(np.uint64)
        W[rng.random(N) < 0.3] = 0
        W[rng.integers(0, N)] = 1 + int(rng.integers(0, 2 ** 20))
        u = int(rng.integers(0, 2 ** 64, dtype=np.uint64))
        idx = oracle_lib.resample(W, u)
        assert np.all(np.diff(idx) >= 0) and idx.min() >= 0 and idx.max() < N
        c = _counts(idx, N).astype(object)
        T = int(W.sum())
        Wo = W.astype(object)
        assert all((N * w) // T <= ci <= -(-(N * w) // T) for w, ci in zip(Wo, c))
        assert np.all(c[W == 0] == 0)
        assert int(c.sum()) == N


def test_resample_special_cases(oracle_lib):
    N = 64
    # equal weights with T divisible by N: the identity, for every offset
    W = np.full(N, 5, np.uint64)
    for r in range(int(W.sum())):
        assert np.array_equal(oracle_lib.resample(W, _u_for_offset(r, int(W.sum()))), np.arange(N))
    # a single non-zero weight takes every slot
    W = np.zeros(N, np.uint64)
    W[13] = 12345
    for u in (0, 2 ** 63, 2 ** 64 - 1):
        assert np.all(oracle_lib.resample(W, u) == 13)
    # every weight zero: read as equal weights
    assert np.array_equal(oracle_lib.resample(np.zeros(N, np.uint64), 99), np.arange(N))
    # largest totals the contract allows (N = 2^21, sum W = 2^42) stay exact
    N = 2 ** 21
    W = np.full(N, 2 ** 21, np.uint64)
    idx = oracle_lib.resample(W, 2 ** 64 - 1)
    assert np.array_equal(idx, np.arange(N))


# ------------------------------------------------------------- resampling draw
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "splitmix64_kat.txt")
GOLDEN_GAMMA = 0x9E3779B97F4A7C15


def _splitmix_kat():
    state, outs = None, []
    for line in open(GOLDEN):
        line = line.strip()
        if line.startswith("# state"):
            state = int(line.split()[2])
        elif line and not line.startswith("#"):
            outs.append(int(line))
    return state, outs


def test_splitmix64_known_answers(oracle_lib):
    """The published first outputs of the reference SplitMix64 from state 1234567:
    output k comes from state 1234567 + k * gamma (the generator advances first)."""
    state, outs = _splitmix_kat()
    assert len(outs) == 5
    for k, want in enumerate(outs):
        assert oracle_lib.splitmix64((state + k * GOLDEN_GAMMA) % 2 ** 64) == want, k


def test_resample_draw_properties(oracle_lib):
    """Per filter seed, distinct ticks give distinct draws (the map tick -> u is a
    bijection of 64-bit words), the draw depends on the seed, and the top bits
    of u over consecutive ticks are uniform (chi-square over 64 cells)."""
    seed = 0x0123456789ABCDEF
    us = [oracle_lib.resample_draw(seed, t) for t in range(20000)]
    assert len(set(us)) == len(us)
    assert oracle_lib.resample_draw(seed ^ 1, 5) != oracle_lib.resample_draw(seed, 5)
    # u(seed, tick) = splitmix64(seed XOR splitmix64(tick)): with seed 0 and the
    # known answers, u(0, t) for the tick whose splitmix64 is the state 1234567
    state, outs = _splitmix_kat()
    assert oracle_lib.resample_draw(state ^ oracle_lib.splitmix64(7), 7) == outs[0]
    cells = np.bincount(np.asarray([u >> 58 for u in us]), minlength=64)
    exp = len(us) / 64
    chi2 = float(((cells - exp) ** 2 / exp).sum())
    assert chi2 < 120.0, chi2   # 63 degrees of freedom: P(chi2 > 120) < 1e-5
