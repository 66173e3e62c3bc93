"""Filter checkpoints on the CPU: save() writes plain arrays (loadable without
unpickling), load() restores poses, sigma, seed, tick and the reading, and
refuses a particle set of another size."""

import numpy as np
import pytest


@pytest.fixture(scope="module")
def mcl():
    from paper_2310_04172_amd import mcl as m
    return m


def test_filter_state_round_trip(mcl, tmp_path):
    import torch
    rng = np.random.default_rng(3)
    poses = torch.from_numpy(rng.normal(size=(12, 37)).astype(np.float32))
    seed = 2 ** 64 - 5
    f = mcl.Filter(None, None, poses, 0.125, seed, tick=9, score="sum", want_w=False)
    path = str(tmp_path / "f.npz")
    f.save(path)
    with np.load(path, allow_pickle=False) as z:
        assert set(z.files) == {"poses", "sigma", "seed", "tick", "score", "trilinear"}
    g = mcl.Filter(None, None, torch.zeros((12, 37)), 1.0, 0, want_w=False)
    g.load(path)
    assert torch.equal(g.poses, poses) and g.poses is not poses
    assert (g.sigma, g.seed, g.tick, g.score, g.trilinear) == (0.125, seed, 9, "sum", False)
    h = mcl.Filter(None, None, torch.zeros((12, 36)), 1.0, 0, want_w=False)
    with pytest.raises(ValueError):
        h.load(path)
