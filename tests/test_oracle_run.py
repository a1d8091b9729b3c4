"""Pins for the oracle's running-point criteria (Sec. 5.2, Eq. 4): the five
criteria of a zone raster vertex and their weighted sum.

* P and Q (where the lines to the goal posts meet the defense area) against
  closed forms and against a dense walk along each segment.
* Each criterion against its closed form at chosen points: distance to the
  goal and to the ball, every branch of the angle window, the guard time of
  a resting opponent (rest-to-rest motion written here from its textbook
  form), the marking weight of an opponent nearer to the ball.
* Structure: points strictly inside the defense area are excluded, its
  boundary is not; one-hot weights give back each criterion; mirror symmetry
  of the score map; an added opponent never raises the guard or defense
  criteria; the zone best is the first maximum of the score map.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1909_07717_amd.framegen import Frame, Params, config_small, random_frame

D = O.RUN_DEFAULTS


def _frame(ball, opp):
    team = np.array([[ball[0], ball[1], 0, 0], [-5.0, -4.0, 0, 0]], np.float32)
    opp = np.asarray(opp, np.float32).reshape(-1, 4)
    return Frame(team, opp, 0, team[0, :2].copy(), [], [])


def _rest_to_rest(p, dist):
    A, V = p.amax, p.vmax
    if dist <= V * V / A:
        return 2 * math.sqrt(dist / A)
    return dist / V + V / A


@pytest.mark.parametrize("c,P,Q", [((2.0, 0.0), (4.8, 0.42), (4.8, -0.42)),
                                   ((4.5, 3.0), (5.625, 1.2), (5.25, 1.2)),
                                   ((5.5, -2.0), (5.5 + 0.5 * 0.8 / 2.6, -1.2),
                                    (5.5 + 0.5 * 0.8 / 1.4, -1.2)),
                                   # on the area's boundary: the point itself
                                   ((6.0, 0.25), (6.0, 0.25), (6.0, 0.25)),
                                   ((4.8, -0.5), (4.8, -0.5), (4.8, -0.5))])
def test_p_and_q_closed_forms(c, P, Q):
    p = Params()
    r = O.run_point(_frame((0.0, 0.0), np.zeros((0, 4))), p, *c)
    assert (r["px"], r["py"]) == pytest.approx(P, abs=1e-12)
    assert (r["qx"], r["qy"]) == pytest.approx(Q, abs=1e-12)


def test_p_and_q_against_a_dense_walk():
    p = Params()
    rng = np.random.default_rng(3)
    x0, y0, y1 = p.goal_x - D["def_depth"], -0.5 * D["def_width"], 0.5 * D["def_width"]
    for _ in range(40):
        c = (rng.uniform(-3.0, 5.9), rng.uniform(-4.4, 4.4))
        if x0 < c[0] and -1.2 < c[1] < 1.2:
            continue
        r = O.run_point(_frame((0.0, 0.0), np.zeros((0, 4))), p, *c)
        for key, post in (("p", 0.5 * p.goal_width), ("q", -0.5 * p.goal_width)):
            t = np.linspace(0.0, 1.0, 200001)
            x = c[0] + t * (p.goal_x - c[0])
            y = c[1] + t * (post - c[1])
            inside = (x >= x0) & (y >= y0) & (y <= y1)
            k = int(np.argmax(inside))
            assert r[key + "x"] == pytest.approx(x[k], abs=1e-4)
            assert r[key + "y"] == pytest.approx(y[k], abs=1e-4)


def test_criteria_closed_forms():
    p = Params()
    # ball at (-1, 1), one resting opponent at (5.4, 0.3), point c = (3, -1)
    f = _frame((-1.0, 1.0), [[5.4, 0.3, 0.0, 0.0]])
    c = (3.0, -1.0)
    r = O.run_point(f, p, *c)
    assert r["valid"] == 1
    assert r["goal"] == pytest.approx(1 - math.hypot(3.0, 1.0) / p.dist_norm, abs=1e-12)
    assert r["ball"] == pytest.approx(min(math.hypot(4.0, 2.0) / 2.0, 1.0), abs=1e-12)
    phi = math.atan2(1.0, 3.0)   # 0.3217 rad, inside [15, 45] degrees
    assert D["ang_lo"] < phi < D["ang_hi"] and r["angle"] == 1.0
    o = np.float32([5.4, 0.3]).astype(np.float64)
    tp = _rest_to_rest(p, math.hypot(r["px"] - o[0], r["py"] - o[1]) - p.robot_radius)
    tq = _rest_to_rest(p, math.hypot(r["qx"] - o[0], r["qy"] - o[1]) - p.robot_radius)
    assert r["t_p"] == pytest.approx(tp, abs=1e-12)
    assert r["t_q"] == pytest.approx(tq, abs=1e-12)
    assert r["guard"] == pytest.approx(min((tp + tq) / D["guard_norm"], 1.0), abs=1e-12)
    # the opponent is farther from the ball than c: no mark
    assert r["defense"] == 1.0
    want = (D["w_goal"] * r["goal"] + D["w_ball"] * r["ball"] + D["w_angle"] * r["angle"]
            + D["w_guard"] * r["guard"] + D["w_defense"] * r["defense"])
    assert r["score"] == pytest.approx(want, abs=1e-12)


@pytest.mark.parametrize("c,expect", [
    ((1.0, 0.0), 1 - (0.2617993877991494 - 0.0) / 0.5235987755982988),   # below the window
    ((2.0, -2.0), 1.0),                                                   # at 45 degrees
    ((5.0, 3.0), 1 - (math.atan2(3.0, 1.0) - 0.7853981633974483) / 0.5235987755982988),
    ((5.8, 4.0), 0.0),                                                    # beyond the fall
])
def test_angle_window_branches(c, expect):
    p = Params()
    r = O.run_point(_frame((0.0, 0.0), np.zeros((0, 4))), p, *c)
    assert r["angle"] == pytest.approx(max(expect, 0.0), abs=1e-12)


def test_marking_weight_of_an_opponent_nearer_the_ball():
    p = Params()
    # ball at the origin, c at (3, 0); opponent at (2.6, 0.3): 0.5 m from c,
    # 2.62 m from the ball (c is 3 m away) -> weight 1 - 0.5 / 1
    f = _frame((0.0, 0.0), [[2.6, 0.3, 0.0, 0.0]])
    r = O.run_point(f, p, 3.0, 0.0)
    o = np.float32([2.6, 0.3]).astype(np.float64)
    assert r["defense"] == pytest.approx(math.hypot(3.0 - o[0], o[1]) / D["mark_radius"],
                                         abs=1e-12)
    # the same opponent behind c (farther from the ball) does not mark it
    g = _frame((0.0, 0.0), [[3.4, 0.3, 0.0, 0.0]])
    assert O.run_point(g, p, 3.0, 0.0)["defense"] == 1.0
    # nor does a near-ball opponent beyond the mark radius
    h = _frame((0.0, 0.0), [[1.5, 0.0, 0.0, 0.0]])
    assert O.run_point(h, p, 3.0, 0.0)["defense"] == 1.0


def test_defense_area_excluded_boundary_kept():
    p = Params()
    f = _frame((0.0, 0.0), np.zeros((0, 4)))
    assert O.run_point(f, p, 5.5, 0.0)["valid"] == 0
    assert O.run_point(f, p, 5.5, 0.0)["score"] == -math.inf
    for c in ((4.8, 0.0), (5.5, 1.2), (5.5, -1.2), (6.0, 0.5)):
        assert O.run_point(f, p, *c)["valid"] == 1, c


def test_one_hot_weights_give_back_each_criterion():
    p = Params()
    f = config_small(3)
    keys = ("goal", "ball", "angle", "guard", "defense")
    base = O.run_point(f, p, 2.3, -1.7)
    for k in keys:
        w = {f"w_{q}": float(q == k) for q in keys}
        assert O.run_point(f, p, 2.3, -1.7, **w)["score"] == pytest.approx(base[k], abs=1e-15)


@pytest.mark.parametrize("seed", [0, 1])
def test_mirror_symmetry_and_zone_best(seed):
    p = Params()
    f = random_frame(np.random.default_rng(seed), 6, 8, Params())
    f.windows = [(np.float32(0.1), 60, 0, 61, 91)]   # the attacking half, full width
    g = f.copy()
    for a in (g.team, g.opp):
        a[:, 1] *= -1
        a[:, 3] *= -1
    g.ball = np.array([f.ball[0], -f.ball[1]], np.float32)
    r = O.run_search(f, p)
    q = O.run_search(g, p)
    a = r["score"].reshape(91, 61)
    b = q["score"].reshape(91, 61)[::-1]
    fin = np.isfinite(a)
    assert (fin == np.isfinite(b)).all()
    np.testing.assert_allclose(a[fin], b[fin], rtol=0, atol=1e-12)
    assert r["best"][0] == int(np.argmax(r["score"]))


def test_added_opponent_never_raises_guard_or_defense():
    p = Params()
    f = config_small(6)
    g = f.copy()
    g.opp = np.vstack([f.opp, np.array([[4.9, 0.2, 0.0, 0.0]], np.float32)])
    f.windows = g.windows = [(np.float32(0.1), 70, 20, 40, 50)]
    r, q = O.run_search(f, p), O.run_search(g, p)
    ok = r["valid"] == 1
    assert (q["guard"][ok] <= r["guard"][ok] + 1e-15).all()
    assert (q["defense"][ok] <= r["defense"][ok] + 1e-15).all()
    assert (q["guard"][ok] < r["guard"][ok]).any()
