"""Invariants of the whole search, checked on the oracle (Sec. 4.2-4.3).

1. No opponents: feasible <=> reachable and some teammate intercepts, and
   the margin term is at its cap.
2. Mirror symmetry y -> -y of robots and velocities mirrors the maps (the
   lattice is exactly symmetric).
3. Permuting robots within a team changes nothing.
4. Adding an opponent never adds a feasible point and never raises a score.
5. Adding a teammate never removes a feasible point.
6. A robot 1 km away behaves exactly like an absent one.
7. Feasible scores lie in [0.3 (1 - 12.82/15) + 0.2 * 0.1, 1].
8. The best point is the brute-force argmax of the score map (ties to the
   lowest index) and is absent exactly when nothing is feasible.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1909_07717_amd.framegen import (Params, Frame, FLAT, CHIP, full_window,
                                           random_frame, variants_for)

P = Params(n_samples=32)
VARS = variants_for([2.0, 4.5], flat=True, chip=True)


def _frame(seed, n_team=6, n_opp=6, h=0.5):
    f = random_frame(np.random.default_rng(seed), n_team, n_opp)
    f.windows = [full_window(h)]
    f.variants = list(VARS)
    return f


def _maps(f):
    r = O.search_frame(f, P)
    w = f.windows[0]
    V = len(f.variants)
    return {k: (r[k].reshape(V, w[4], w[3]) if isinstance(r[k], np.ndarray) else r[k])
            for k in r}


@pytest.mark.parametrize("seed", range(3))
def test_no_opponents(seed):
    f = _frame(seed, 6, 0)
    f.opp = np.zeros((0, 4), np.float32)
    r = O.search_frame(f, P)
    pts = O.points_of_window(P, f.windows[0])
    n = pts.shape[0]
    for v, (vt, v0) in enumerate(f.variants):
        sl = slice(v * n, (v + 1) * n)
        D, sf = O.ball_range(P, vt, v0)
        d = np.hypot(pts[:, 0] - f.ball[0], pts[:, 1] - f.ball[1])
        reach = (d <= D) & (d >= 1e-9) & ((vt != CHIP) | (d >= sf))
        fin = np.isfinite(r["t_team"][sl])
        assert np.array_equal(r["mask"][sl].astype(bool), reach & fin)
        feas = r["mask"][sl].astype(bool)
        ang = np.array([O.open_angle(P, x, y, []) for x, y in pts[feas]])
        dg = np.hypot(pts[feas, 0] - 6.0, pts[feas, 1])
        want = 0.5 * ang / math.pi + 0.3 * (1 - dg / 15.0) + 0.2 * 1.0
        np.testing.assert_allclose(r["score"][sl][feas], want, rtol=0, atol=1e-14)


@pytest.mark.parametrize("seed", range(3))
def test_mirror_symmetry(seed):
    f = _frame(seed)
    g = f.copy()
    g.team[:, 1] *= -1
    g.team[:, 3] *= -1
    g.opp[:, 1] *= -1
    g.opp[:, 3] *= -1
    g.ball = g.team[g.passer, :2].copy()
    a, b = _maps(f), _maps(g)
    assert np.array_equal(a["mask"], b["mask"][:, ::-1, :])
    fa = np.isfinite(a["score"])
    np.testing.assert_allclose(a["score"][fa], b["score"][:, ::-1, :][fa], rtol=0, atol=1e-12)
    np.testing.assert_allclose(a["t_team"], b["t_team"][:, ::-1, :], rtol=0, atol=1e-12)


@pytest.mark.parametrize("seed", range(3))
def test_permutation_within_teams(seed):
    f = _frame(seed)
    rng = np.random.default_rng(100 + seed)
    g = f.copy()
    perm = rng.permutation(f.n_team)
    g.team = f.team[perm]
    g.passer = int(np.where(perm == f.passer)[0][0])
    g.opp = f.opp[rng.permutation(f.n_opp)]
    a, b = _maps(f), _maps(g)
    assert np.array_equal(a["mask"], b["mask"])
    np.testing.assert_allclose(a["score"], b["score"], rtol=0, atol=1e-13)
    assert np.array_equal(a["t_team"], b["t_team"]) and np.array_equal(a["t_opp"], b["t_opp"])


@pytest.mark.parametrize("seed", range(3))
def test_adding_robots_is_monotone(seed):
    f = _frame(seed)
    rng = np.random.default_rng(200 + seed)
    extra = np.array([[*rng.uniform([-6, -4.5], [6, 4.5]), 0.3, -0.2]], np.float32)
    more_opp = f.copy()
    more_opp.opp = np.concatenate([f.opp, extra])
    more_team = f.copy()
    more_team.team = np.concatenate([f.team, extra])
    a, b, c = _maps(f), _maps(more_opp), _maps(more_team)
    assert not np.any(b["mask"] & ~a["mask"])          # no new feasible point
    assert np.all(b["score"] <= a["score"])            # no score goes up
    assert not np.any(a["mask"] & ~c["mask"])          # no feasible point lost


@pytest.mark.parametrize("seed", range(2))
def test_far_robot_is_absent(seed):
    f = _frame(seed)
    far = np.array([[1000.0, 1000.0, 1.0, 0.5]], np.float32)
    g = f.copy()
    g.opp = np.concatenate([f.opp, far])
    g.team = np.concatenate([f.team, far])
    a, b = _maps(f), _maps(g)
    for k in ("mask", "score", "t_team", "t_opp"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("seed", range(3))
def test_score_range_and_argmax(seed):
    f = _frame(seed, h=0.3)
    r = O.search_frame(f, P)
    s = r["score"]
    feas = r["mask"].astype(bool)
    assert np.array_equal(np.isfinite(s), feas)
    lo = 0.3 * (1 - math.hypot(12.0, 4.5) / 15.0) + 0.2 * 0.1
    assert lo == pytest.approx(0.0637, abs=1e-4)
    assert np.all(s[feas] >= lo - 1e-12) and np.all(s[feas] <= 1.0)
    if feas.any():
        assert r["best"] == int(np.argmax(s)) and r["best_score"] == s.max()
    else:
        assert r["best"] == -1


def test_nothing_feasible_gives_no_best():
    # a lone passer: no teammate can receive anywhere
    f = Frame(team=np.array([[0, 0, 0, 0]], np.float32),
              opp=np.array([[1, 1, 0, 0]], np.float32), passer=0,
              ball=np.array([0, 0], np.float32), windows=[full_window(0.5)],
              variants=variants_for([3.0], True, True))
    r = O.search_frame(f, P)
    assert r["best"] == -1 and not r["mask"].any()
