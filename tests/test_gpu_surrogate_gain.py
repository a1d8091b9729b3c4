"""What the trained network adds (GPU), on 300 held-out frames (6v6, one
flat pass at 4 m/s, K = 64, 5 cm answers; regret against the exact search of
the whole 5 cm lattice): the shipped network's top-64 cells re-scored
exactly, against the same search with (a) an untrained network of the same
shape and (b) no network at all (cells ranked by the robot-free terms of
Eq. 3).  All three use the same exact re-score and fallback rule.
"""
import os

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def runs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_07717_amd.surrogate import WEIGHTS, evaluate
    assert os.path.exists(WEIGHTS), "the shipped network is missing"
    out = {}
    for name in ("trained", "untrained", "no network"):
        out[name] = evaluate(WEIGHTS, 300, k=64, batch=300, random_net=(name == "untrained"),
                             proposals="geometric" if name == "no network" else "network")
    return out


def test_trained_network_beats_an_untrained_one(runs):
    t, r = runs["trained"], runs["untrained"]
    assert t["frames_with_exact_best"] == r["frames_with_exact_best"] > 250
    assert t["regret_le_1pct"] >= 0.9, t
    assert r["regret_le_1pct"] <= 0.5, r
    assert t["regret_mean"] < 0.25 * r["regret_mean"]


def test_without_a_network_most_frames_fall_back(runs):
    # the robot-free ranking proposes infeasible cells on about half of the
    # frames, which then pay for the full exact search; the network's
    # proposals are feasible on nearly all frames
    t, g = runs["trained"], runs["no network"]
    assert g["fallback_rate"] >= 0.3, g
    assert t["fallback_rate"] <= 0.05, t
