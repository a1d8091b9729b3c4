"""Pins for the oracle's passing power (Sec. 4.1, Eq. 1-2): the kick speed of
a pass to a point, from the receiver's arrival time plus a buffer, the
distance and the rolling deceleration, clamped to the kick range.

* Inversion: the closed form of Eq. 1 equals a bisection root of the rolling
  ball's distance at the requested time (the paper's simplification, no
  sliding phase); beyond the longest time a rolling ball can take, the
  reading picks the slowest ball that still reaches the point.
* Full model: with the sliding phase kept (the forward model of Sec. 4.1),
  the ball then arrives no later than requested (it is ahead of the rolling
  ball after the slide, and faster), and it does reach the point.
* Clamping, a lone passer (no receiver), monotonicity in the receiver's
  distance, mirror symmetry of the power map.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1909_07717_amd.framegen import FLAT, Frame, Params, config_small, full_window

BUF = 0.3


def _frame(ball, recv, opp=((0.0, 4.0, 0.0, 0.0),)):
    team = np.array([[ball[0], ball[1], 0, 0], list(recv)], np.float32)
    return Frame(team, np.array(opp, np.float32), 0, team[0, :2].copy(), [], [])


def _roll_dist(v, t, a):
    return v * t - 0.5 * a * t * t if v >= a * t else v * v / (2 * a)


def _bisect_v1(d, t, a):
    lo, hi = 0.0, 200.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if _roll_dist(mid, t, a) < d:
            lo = mid
        else:
            hi = mid
    return hi


@pytest.mark.parametrize("ball,recv,c", [
    ((0.0, 0.0), (3.0, 1.0, 0.0, 0.0), (3.0, 0.0)),
    ((-4.0, 2.0), (1.0, -1.0, 0.5, 0.2), (2.0, -2.0)),
    ((1.0, 1.0), (1.5, 1.2, 0.0, 0.0), (1.6, 1.1)),
    ((0.0, 0.0), (-5.0, 4.0, -1.0, 0.0), (1.0, 0.5)),
    ((-5.0, -4.0), (4.0, 3.0, 0.0, 0.0), (4.5, 3.5)),
])
def test_power_matches_bisection_of_the_rolling_model(ball, recv, c):
    p = Params()
    f = _frame(ball, recv)
    v0, tb = O.power_speed(f, p, c[0], c[1], BUF, 0.0, 1e9)
    assert tb == pytest.approx(O.robot_time_to(p, f.team[1].astype(np.float64), c[0], c[1]),
                               abs=1e-12)
    d = math.hypot(c[0] - ball[0], c[1] - ball[1])
    t = tb + BUF
    a = p.roll_decel
    v1 = _bisect_v1(d, t, a)
    assert v0 * p.slide_ratio == pytest.approx(v1, rel=1e-9, abs=1e-9)
    # the ball of the rolling model is then at d at time t, or has just
    # stopped there when t exceeds the longest rolling time
    if t <= math.sqrt(2 * d / a):
        assert _roll_dist(v1, t, a) == pytest.approx(d, rel=1e-9)
    else:
        assert v1 == pytest.approx(math.sqrt(2 * a * d), rel=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_power_full_model_arrives_no_later_than_requested(seed):
    p = Params(n_samples=64)
    f = config_small(seed)
    rng = np.random.default_rng(seed)
    for _ in range(40):
        c = rng.uniform(-5.5, 5.5), rng.uniform(-4, 4)
        v0, tb = O.power_speed(f, p, c[0], c[1], BUF, 0.0, 1e9)
        d = math.hypot(c[0] - f.ball[0], c[1] - f.ball[1])
        t = tb + BUF
        tf = O.ball_time(p, FLAT, v0, d)
        D, _ = O.ball_range(p, FLAT, v0)
        assert D >= d and math.isfinite(tf)
        if d >= 0.5 * p.roll_decel * t * t:
            assert tf <= t + 1e-12


def test_power_clamped_to_the_kick_range_and_needs_a_receiver():
    p = Params(n_samples=64)
    f = config_small(3)
    r = O.power_search(f, p, BUF, 1.0, 6.5)
    assert (r["v0"] >= 1.0).all() and (r["v0"] <= 6.5).all()
    assert ((r["v0"] == 1.0) | (r["v0"] == 6.5)).any()
    lone = f.copy()
    lone.team = f.team[f.passer:f.passer + 1].copy()
    lone.passer = 0
    q = O.power_search(lone, p, BUF, 1.0, 6.5)
    assert (q["v0"] == 0).all() and q["mask"].sum() == 0 and q["best"] == -1


def test_power_decreases_as_the_receiver_moves_away():
    p = Params()
    c = (2.0, 0.0)
    last = math.inf
    for dist in (0.2, 0.5, 1.0, 1.5, 2.0, 3.0):
        f = _frame((-3.0, 0.0), (c[0], c[1] + dist, 0.0, 0.0))
        v0, _ = O.power_speed(f, p, c[0], c[1], BUF, 0.0, 1e9)
        assert v0 <= last + 1e-12
        last = v0


def test_power_map_mirror_symmetry():
    p = Params(n_samples=64)
    f = config_small(7)
    f.windows = [full_window(0.2)]
    g = f.copy()
    for a in (g.team, g.opp):
        a[:, 1] *= -1
        a[:, 3] *= -1
    g.ball = np.array([f.ball[0], -f.ball[1]], np.float32)
    r = O.power_search(f, p, BUF)
    q = O.power_search(g, p, BUF)
    nx, ny = 61, 46
    for key in ("v0", "t_team", "t_opp", "score"):
        a = r[key].reshape(ny, nx)
        b = q[key].reshape(ny, nx)[::-1]
        fin = np.isfinite(a)
        assert (fin == np.isfinite(b)).all()
        np.testing.assert_allclose(a[fin], b[fin], rtol=0, atol=1e-9)
    assert (r["mask"].reshape(ny, nx) == q["mask"].reshape(ny, nx)[::-1]).all()
