"""Normalisation and resampling with one workgroup per filter in one launch
(the shape mcl_normalize, mcl_resample and mcl_tick take for filters of at most
mcl_set_weights_fused_max particles), through the C ABI.

Both shapes perform the same floating-point operations in the same order, so
the contract is bit-identical outputs: every output of the one-launch shape
equals the three-launch chains' bit for bit, for sizes from one particle to the
largest limit (one 4,096-particle weight block), and the one-launch shape
meets the oracle bars by itself.
"""

import sys

import numpy as np
import pytest

from tests import checks

pytestmark = pytest.mark.gpu

FUSED_ALL = 4096


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


@pytest.fixture
def restore_limit(mcl):
    prev = mcl.get_weights_fused_max()
    yield
    mcl.set_weights_fused_max(prev)


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def log_weights(kind, rng, N):
    if kind == "spread":    # most weights underflow to a zero fixed-point weight
        lw = -np.abs(rng.normal(0, 300, N)) - 1e4
    elif kind == "narrow":
        lw = rng.normal(-50, 2, N)
    elif kind == "equal":
        lw = np.full(N, -123.25)
    else:                   # one particle far above the rest
        lw = np.full(N, -1e5)
        lw[int(rng.integers(0, N))] = -10.0
    return lw.astype(np.float32)


def run_weights(torch, mcl, lw, poses, seed, tick, limit):
    mcl.set_weights_fused_max(limit)
    w, wq, lz = mcl.normalize(dev(torch, lw))
    idx, pout = mcl.resample(wq, seed, tick, dev(torch, poses))
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (w, wq, lz, idx, pout)]


def assert_bits(a, b, what):
    for n, x, y in zip(("w", "wq", "log_z", "idx", "poses_out"), a, b):
        assert x.dtype == y.dtype and np.array_equal(x.view(np.uint8), y.view(np.uint8)), f"{what}: {n} differs"


@pytest.mark.parametrize("N", [1, 2, 63, 64, 255, 256, 257, 1000, 2048, 4095, 4096])
def test_one_launch_equals_chains(torch, mcl, restore_limit, N):
    say(f"case: one-launch weights vs chains, N={N}")
    rng = np.random.default_rng(900 + N)
    poses = rng.normal(size=(12, N)).astype(np.float32)
    for kind in ("spread", "narrow", "equal", "one"):
        lw = log_weights(kind, rng, N)
        seed, tick = int(rng.integers(0, 2 ** 63)), int(rng.integers(0, 1000))
        fused = run_weights(torch, mcl, lw, poses, seed, tick, FUSED_ALL)
        chain = run_weights(torch, mcl, lw, poses, seed, tick, 0)
        assert_bits(fused, chain, f"N={N} {kind}")
    # all-zero fixed-point weights: the identity, on both shapes
    for limit in (FUSED_ALL, 0):
        mcl.set_weights_fused_max(limit)
        idx, pout = mcl.resample(dev(torch, np.zeros(N, np.uint64)), 3, 4, dev(torch, poses))
        assert np.array_equal(idx.cpu().numpy(), np.arange(N)) and np.array_equal(pout.cpu().numpy(), poses)


def test_limit_selects_the_shape_per_size(torch, mcl, restore_limit):
    """Sizes on both sides of a limit of 1,000 give the same bits as the chains."""
    rng = np.random.default_rng(903)
    for N in (999, 1000, 1001, 4096):
        poses = rng.normal(size=(12, N)).astype(np.float32)
        lw = log_weights("narrow", rng, N)
        a = run_weights(torch, mcl, lw, poses, 9, 1, 1000)
        b = run_weights(torch, mcl, lw, poses, 9, 1, 0)
        assert_bits(a, b, f"limit 1000, N={N}")


@pytest.mark.parametrize("N", [1, 7, 1000, 4096])
def test_one_launch_against_oracle(torch, mcl, oracle_lib, restore_limit, N):
    """The one-launch shape on its own against the oracle: the normalisation
    within its float64 bound, the resampling of the oracle's fixed-point
    weights bit for bit, and the zero-weight case (ancestors are the identity)."""
    say(f"case: one-launch weights vs oracle, N={N}")
    mcl.set_weights_fused_max(FUSED_ALL)
    rng = np.random.default_rng(902 + N)
    poses = rng.normal(size=(12, N)).astype(np.float32)
    lw = log_weights("spread" if N % 2 else "narrow", rng, N)
    w, wq, lz = mcl.normalize(dev(torch, lw))
    wq_ref = checks.check_normalize(oracle_lib, lw, wq.cpu().numpy(), float(lz.cpu().numpy()[0]), w.cpu().numpy(),
                                    f"one-launch normalise N={N}")
    seed, tick = 0xDEADBEEF12345678, N
    idx, pout = mcl.resample(dev(torch, wq_ref), seed, tick, dev(torch, poses))
    checks.check_resample(oracle_lib, wq_ref, seed, tick, idx.cpu().numpy(), poses, pout.cpu().numpy(),
                          f"one-launch resample N={N}")
    idx, _ = mcl.resample(dev(torch, np.zeros(N, np.uint64)), seed, tick)
    assert np.array_equal(idx.cpu().numpy(), np.arange(N))
