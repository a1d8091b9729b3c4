"""Pins for the oracle's shooting decision (Sec. 4.4: the shot-angle test
fused with the interception prediction along the shot to the goal).

* Geometry: with no opponents the widest gap is the whole mouth (closed
  form from the posts); with one opponent centred on the shot line the two
  gaps are equal and the tie goes to the lower one (closed form); on random
  frames the widest gap, the total open angle and the aim agree with a dense
  scan of shot directions tested against every opponent disc by the
  perpendicular distance of the ray (a different construction from the
  oracle's interval merge).
* Interception: the shot is intercepted (slack <= 0) exactly when the
  pass search, with the ball placed at the shooter and the goal-line point as
  target, finds an opponent interception; with one opponent at rest the
  slack equals the minimum over the samples of the rest-to-rest arrival time
  minus the ball time, both written here from their textbook forms.
* Special cases and invariants: a shooter inside an opponent disc, an
  opponent behind the goal line, mirror symmetry, monotonicity of the
  decision in its thresholds, and the paper's motivating case (a far shot
  with a wide angle is intercepted, a near one on the same line is not).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1909_07717_amd.framegen import FLAT, Frame, Params, config_small, random_frame

V_SHOT = 6.5


def _frame(shooter, opp):
    team = np.array([[shooter[0], shooter[1], 0, 0], [-5.0, -4.0, 0, 0]], np.float32)
    opp = np.asarray(opp, np.float32).reshape(-1, 4)
    return Frame(team, opp, 0, team[0, :2].copy(), [], [])


def _ball_time_textbook(p, v0, s):
    """Flat kick: slide at a_s until v = ratio * v0, then roll at a_r; time
    from the quadratic s = v t - a t^2 / 2 of each phase (its smaller root)."""
    v1 = p.slide_ratio * v0
    d1 = (v0 * v0 - v1 * v1) / (2 * p.slide_decel)
    if s <= d1:
        return (v0 - math.sqrt(v0 * v0 - 2 * p.slide_decel * s)) / p.slide_decel
    t1 = (v0 - v1) / p.slide_decel
    r = s - d1
    if r > v1 * v1 / (2 * p.roll_decel):
        return math.inf
    return t1 + (v1 - math.sqrt(v1 * v1 - 2 * p.roll_decel * r)) / p.roll_decel


def _rest_to_rest(p, dist):
    """A robot at rest covering dist and stopping there: accelerate at amax,
    cruise at vmax if it gets there, brake at amax."""
    A, V = p.amax, p.vmax
    if dist <= V * V / A:
        return 2 * math.sqrt(dist / A)
    return dist / V + V / A


@pytest.mark.parametrize("c", [(0.0, 0.0), (3.0, 1.5), (-4.0, -3.0), (5.5, 0.3), (5.95, -2.0)])
def test_no_opponents_whole_mouth(c):
    p = Params(n_samples=64)
    f = _frame(c, np.zeros((0, 4)))
    c = [float(v) for v in f.ball]  # the frame holds float32 positions
    r = O.shot(f, p, v_shot=V_SHOT, min_angle=0.05)
    dx = p.goal_x - c[0]
    lo = math.atan2(-0.5 * p.goal_width - c[1], dx)
    hi = math.atan2(0.5 * p.goal_width - c[1], dx)
    assert r["n_gaps"] == 1
    assert r["gap"] == pytest.approx(hi - lo, abs=1e-12)
    assert r["open_angle"] == pytest.approx(hi - lo, abs=1e-12)
    aim = 0.5 * (lo + hi)
    assert r["aim"] == pytest.approx(aim, abs=1e-12)
    L = dx / math.cos(aim)
    assert r["length"] == pytest.approx(L, rel=1e-12)
    assert math.isinf(r["slack"])
    tg = _ball_time_textbook(p, V_SHOT, L)
    if math.isinf(tg):
        assert not r["reachable"] and math.isinf(r["t_goal"]) and not r["shoot"]
    else:
        assert r["reachable"] and r["t_goal"] == pytest.approx(tg, rel=1e-9)
        assert r["shoot"] == int(hi - lo >= 0.05)


def test_equal_gaps_tie_goes_to_the_lower_gap():
    p = Params(n_samples=64)
    f = _frame((3.0, 0.0), [[4.5, 0.0, 0.0, 0.0]])
    r = O.shot(f, p, v_shot=V_SHOT, min_angle=0.05)
    lo = -math.atan2(0.5 * p.goal_width, 3.0)
    al = math.asin(p.robot_radius / 1.5)
    assert r["n_gaps"] == 2
    assert r["gap"] == pytest.approx(-al - lo, abs=1e-12)
    assert r["second_gap"] == pytest.approx(r["gap"], abs=1e-12)
    assert r["aim"] == pytest.approx(0.5 * (lo - al), abs=1e-12)
    assert r["open_angle"] == pytest.approx(2 * (-al - lo), abs=1e-12)


def _scan(p, f, c, n=200001):
    """Free shot directions over the mouth by a dense scan: a direction is
    blocked when its ray passes within the robot radius of an opponent in
    front of the goal line (perpendicular distance, opponent ahead); a
    shooter inside such a disc has none (the reading of the open angle)."""
    dx = max(p.goal_x - c[0], p.goal_eps)
    lo = math.atan2(-0.5 * p.goal_width - c[1], dx)
    hi = math.atan2(0.5 * p.goal_width - c[1], dx)
    th = lo + (hi - lo) * (np.arange(n) + 0.5) / n
    ux, uy = np.cos(th), np.sin(th)
    free = np.ones(n, bool)
    for o in np.asarray(f.opp, np.float64):
        if o[0] >= p.goal_x:
            continue
        ox, oy = o[0] - c[0], o[1] - c[1]
        if math.hypot(ox, oy) <= p.robot_radius:
            free[:] = False
        along = ox * ux + oy * uy
        perp = np.abs(ox * uy - oy * ux)
        free &= ~((along > 0) & (perp <= p.robot_radius))
    step = (hi - lo) / n
    # widest run of free directions
    best, best_mid, run, start = 0, None, 0, 0
    for i, fr in enumerate(np.append(free, False)):
        if fr:
            if run == 0:
                start = i
            run += 1
        else:
            if run > best:
                best, best_mid = run, lo + step * (start + 0.5 * run)
            run = 0
    return free.sum() * step, best * step, best_mid, step


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4, 5])
def test_gaps_match_a_dense_scan(seed):
    p = Params(n_samples=64)
    rng = np.random.default_rng(seed)
    f = random_frame(rng, 6, 8, Params())
    # crowd the goal area so that the mouth splits into several gaps
    f.opp[:4, 0] = rng.uniform(3.5, 5.8, 4)
    f.opp[:4, 1] = rng.uniform(-0.8, 0.8, 4)
    checked = 0
    for _ in range(12):
        c = (float(rng.uniform(-2.0, 5.0)), float(rng.uniform(-3.0, 3.0)))
        r = O.shot(f, p, c[0], c[1], bands=True)
        if r["ambig"] & O.AMB_ANGLE:
            continue
        total, widest, mid, step = _scan(p, f, c)
        assert r["open_angle"] == pytest.approx(total, abs=4 * step)
        assert r["gap"] == pytest.approx(widest, abs=4 * step)
        if widest > 10 * step and r["gap"] - r["second_gap"] > 10 * step:
            assert r["aim"] == pytest.approx(mid, abs=4 * step)
        checked += 1
    assert checked >= 8


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_interception_equals_the_pass_search_to_the_goal_line(seed):
    p = Params(n_samples=64)
    rng = np.random.default_rng(100 + seed)
    f = random_frame(rng, 6, 8, Params())
    seen = {True: 0, False: 0}
    for _ in range(30):
        c = np.array([rng.uniform(-3.0, 5.0), rng.uniform(-3.5, 3.5)])
        r = O.shot(f, p, c[0], c[1], v_shot=V_SHOT)
        if not r["reachable"]:
            continue
        g = c + r["length"] * np.array([math.cos(r["aim"]), math.sin(r["aim"])])
        h = f.copy()
        h.team[h.passer, :2] = c
        h.ball = c.astype(np.float32)
        e = O.eval_point(h, p, FLAT, V_SHOT, float(g[0]), float(g[1]))
        # the ball is placed in float32 by the frame copy: use the same point
        r2 = O.shot(h, p, float(h.ball[0]), float(h.ball[1]), v_shot=V_SHOT)
        intercepted = r2["slack"] <= 0
        assert intercepted == math.isfinite(e["t_opp"])
        seen[intercepted] += 1
    assert seen[True] > 0 and seen[False] > 0


@pytest.mark.parametrize("c,o", [((-2.0, 0.0), (2.0, 0.9)), ((0.0, 1.0), (3.0, -0.4)),
                                 ((2.0, -2.0), (4.0, -1.6)),
                                 # a keeper behind the line: the goal-line sample decides
                                 ((2.0, 0.3), (6.05, 0.1))])
def test_slack_against_rest_to_rest_closed_form(c, o):
    p = Params(n_samples=64)
    f = _frame(c, [[o[0], o[1], 0.0, 0.0]])
    c = [float(v) for v in f.ball]
    o = [float(v) for v in f.opp[0, :2]]
    r = O.shot(f, p, v_shot=V_SHOT)
    aim, L = r["aim"], r["length"]
    m = math.inf
    for k in range(p.n_samples):
        s = (k + 1) / p.n_samples * L
        tb = _ball_time_textbook(p, V_SHOT, s)
        if math.isinf(tb):
            break
        px, py = c[0] + s * math.cos(aim), c[1] + s * math.sin(aim)
        dist = max(math.hypot(px - o[0], py - o[1]) - p.robot_radius, 0.0)
        m = min(m, _rest_to_rest(p, dist) - tb)
    assert r["slack"] == pytest.approx(m, abs=1e-9)


def test_shooter_inside_an_opponent_and_opponent_behind_the_goal_line():
    p = Params(n_samples=64)
    f = _frame((2.0, 0.5), [[2.05, 0.5, 0.0, 0.0]])
    r = O.shot(f, p)
    assert r["gap"] == 0 and r["open_angle"] == 0 and r["n_gaps"] == 0 and not r["shoot"]
    assert r["aim"] == pytest.approx(math.atan2(-0.5, 4.0), abs=1e-12)
    # an opponent at or behind the goal line casts no shadow (but may still
    # intercept near the line)
    g = _frame((2.0, 0.5), [[6.05, 0.2, 0.0, 0.0]])
    q = O.shot(g, p)
    dx = 4.0
    assert q["gap"] == pytest.approx(math.atan2(0.1, dx) - math.atan2(-1.1, dx), abs=1e-12)


@pytest.mark.parametrize("seed", [7, 8, 9])
def test_mirror_symmetry(seed):
    p = Params(n_samples=64)
    f = random_frame(np.random.default_rng(seed), 6, 8, Params())
    g = f.copy()
    for a in (g.team, g.opp):
        a[:, 1] *= -1
        a[:, 3] *= -1
    g.ball = np.array([f.ball[0], -f.ball[1]], np.float32)
    r, q = O.shot(f, p), O.shot(g, p)
    assert r["gap"] == pytest.approx(q["gap"], abs=1e-12)
    assert r["aim"] == pytest.approx(-q["aim"], abs=1e-12)
    for k in ("slack", "length", "t_goal", "open_angle"):
        if math.isinf(r[k]):
            assert math.isinf(q[k])
        else:
            assert r[k] == pytest.approx(q[k], abs=1e-9)
    assert r["shoot"] == q["shoot"]


def test_decision_monotone_in_its_thresholds():
    p = Params(n_samples=64)
    f = config_small(4)
    f.windows = []
    prev = 1
    for a in (0.0, 0.02, 0.05, 0.1, 0.2, 0.4):
        s = O.shot(f, p, min_angle=a)["shoot"]
        assert s <= prev
        prev = s
    prev = 1
    for m in (0.0, 0.05, 0.1, 0.3, 1.0, 3.0):
        s = O.shot(f, p, margin_s=m)["shoot"]
        assert s <= prev
        prev = s


def test_far_shot_intercepted_near_shot_not():
    # an opponent beside the shot line near the goal, clear of the mouth as
    # seen from both shooters: the far shot passes the angle test but is
    # intercepted, the near one on the same line is not
    p = Params(n_samples=128)
    opp = [[4.5, 0.9, 0.0, 0.0]]
    far = O.shot(_frame((-4.0, 0.0), opp), p, min_angle=0.05)
    near = O.shot(_frame((3.0, 0.0), opp), p, min_angle=0.05)
    assert far["gap"] >= 0.05 and far["reachable"] and far["slack"] < 0 and not far["shoot"]
    assert near["gap"] >= 0.05 and near["reachable"] and near["slack"] > 0 and near["shoot"]


def test_shot_map_equals_pointwise_decisions():
    p = Params(n_samples=64)
    f = config_small(2)
    f.windows = [(np.float32(0.2), 40, 10, 12, 9)]
    m = O.shot_search(f, p, bands=True)
    pts = O.points_of_window(p, f.windows[0])
    for i in (0, 17, 50, 107):
        r = O.shot(f, p, pts[i, 0], pts[i, 1], bands=True)
        for k in O.SHOT_FIELDS:
            a, b = m[k][i], r[k]
            assert (a == b) or (np.isinf(a) and np.isinf(b)), k
