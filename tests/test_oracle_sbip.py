"""Pins for the oracle's interception search (SBIP, Sec. 4.2) and the team
minimum (Sec. 4.3, first teammate / first opponent).

* Dense sampling: the K-sample interception time must be the ball time at the
  first of the K samples a robot reaches in time; the K samples are a subset of
  a dense 16384-sample path, so the K result can never be earlier than the
  dense one, and it is at most one sample's ball-time step later whenever the
  robot stays ahead of the ball for that long.
* Bisection on g(s) = t_robot(s) - t_ball(s) brackets the continuous first
  crossing between two dense samples.
* Team minimum: the first crossing of the per-sample team minimum equals the
  minimum over robots of each robot's own first crossing (min commutes).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1909_07717_amd.framegen import Params, FLAT, CHIP, random_frame, Frame

KD = 16384


def _g_dense(p, ball, c, vtype, v0, robot, K):
    b = np.asarray(ball, float)
    c = np.asarray(c, float)
    d = float(np.hypot(*(c - b)))
    _, sf = O.ball_range(p, vtype, v0)
    out = []
    for k in range(K):
        f = (k + 1) / K
        s = f * d
        pt = b + f * (c - b)
        tr = O.robot_time_to(p, robot, pt[0], pt[1])
        tb = O.ball_time(p, vtype, v0, s)
        air = vtype == CHIP and s < sf
        out.append((s, tr, tb, air))
    return out, d


def _first(rows):
    for k, (s, tr, tb, air) in enumerate(rows):
        if not air and tr <= tb:
            return k
    return None


CASES = [
    # ball, target, type, v0, robot (x, y, vx, vy)
    ((0, 0), (4, 0), FLAT, 4.0, (4, 0.5, 0, 0)),
    ((0, 0), (4, 0), FLAT, 4.0, (2, 1.0, 0, -0.5)),
    ((0, 0), (4, 0), FLAT, 4.0, (2, 0.05, 0.5, 0)),
    ((-2, 1), (3, -2), FLAT, 6.5, (0.5, 0.0, -1.0, 0.4)),
    ((-2, 1), (3, -2), FLAT, 2.0, (0.5, 0.0, -1.0, 0.4)),
    ((0, 0), (4, 0), CHIP, 4.0, (1.0, 0.0, 0, 0)),
    ((0, 0), (4, 0), CHIP, 4.0, (3.0, 0.3, 0.2, 0)),
    ((1, -3), (-4, 2), CHIP, 5.0, (-2, -0.5, 0, 1.2)),
]


@pytest.mark.parametrize("case", CASES)
def test_sbip_against_dense_sampling(case):
    ball, c, vtype, v0, robot = case
    p = Params(n_samples=64)
    tau, k_hit = O.sbip_robot(p, ball, c, vtype, v0, robot)
    dense, d = _g_dense(p, ball, c, vtype, v0, robot, KD)
    step = KD // p.n_samples
    sub = [dense[(k + 1) * step - 1] for k in range(p.n_samples)]
    k_sub = _first(sub)
    if k_sub is None:
        assert tau == math.inf and k_hit == p.n_samples
    else:
        assert k_hit == k_sub
        assert tau == sub[k_sub][2]
    k_d = _first(dense)
    if k_d is None:
        assert tau == math.inf
        return
    tau_d = dense[k_d][2]
    assert tau >= tau_d
    # robot ahead of the ball for a whole sample spacing after the dense hit
    ahead = all((not a) and tr <= tb for (_, tr, tb, a) in dense[k_d:min(KD, k_d + step)])
    if ahead and k_d + step <= KD:
        assert tau <= dense[min(KD - 1, k_d + step - 1)][2]
    # bisection brackets the continuous crossing between two dense samples
    if k_d > 0 and not dense[k_d - 1][3]:
        b = np.asarray(ball, float)
        cc = np.asarray(c, float)
        lo, hi = dense[k_d - 1][0], dense[k_d][0]

        def g(s):
            pt = b + (s / d) * (cc - b)
            return O.robot_time_to(p, robot, pt[0], pt[1]) - O.ball_time(p, vtype, v0, s)
        assert g(lo) > 0 >= g(hi)
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            if g(mid) > 0:
                lo = mid
            else:
                hi = mid
        t_cont = O.ball_time(p, vtype, v0, hi)
        assert 0 <= tau_d - t_cont <= dense[k_d][2] - dense[k_d - 1][2] + 1e-12


@pytest.mark.parametrize("seed", range(6))
def test_team_min_equals_first_crossing_of_min(seed):
    # factored form: per sample the team minimum of arrival times, then the
    # first crossing; must equal the oracle's robot-by-robot minimum exactly
    p = Params(n_samples=48)
    rng = np.random.default_rng(seed)
    f = random_frame(rng, 6, 6)
    for vtype, v0 in ((FLAT, 2.0), (FLAT, 5.5), (CHIP, 4.5)):
        for _ in range(5):
            c = rng.uniform([-6, -4.5], [6, 4.5])
            r = O.eval_point(f, p, vtype, v0, c[0], c[1])
            if not r["reachable"]:
                continue
            b = f.ball.astype(float)
            d = math.sqrt((c[0] - b[0]) ** 2 + (c[1] - b[1]) ** 2)
            _, sf = O.ball_range(p, vtype, v0)
            for side, robots in (("t_team", [x for j, x in enumerate(f.team) if j != f.passer]),
                                 ("t_opp", list(f.opp))):
                got = math.inf
                for k in range(p.n_samples):
                    fr = (k + 1) / p.n_samples
                    s = fr * d
                    if vtype == CHIP and s < sf:
                        continue
                    pt = b + fr * (c - b)
                    tmin = min(O.robot_time_to(p, rb, pt[0], pt[1]) for rb in robots)
                    tb = O.ball_time(p, vtype, v0, s)
                    if tmin <= tb:
                        got = tb
                        break
                assert got == r[side]


def test_passer_is_not_an_interceptor():
    # the passer stands on the ball; if it counted it would intercept at once
    p = Params(n_samples=64)
    f = Frame(team=np.array([[0, 0, 0, 0], [3, 2, 0, 0]], np.float32),
              opp=np.zeros((0, 4), np.float32), passer=0, ball=np.array([0, 0], np.float32))
    r = O.eval_point(f, p, FLAT, 4.0, 3.0, 0.0)
    tau, _ = O.sbip_robot(p, (0, 0), (3, 0), FLAT, 4.0, (3, 2, 0, 0))
    assert r["t_team"] == tau > 0.3
    # a lone passer has nobody to pass to
    f1 = Frame(team=np.array([[0, 0, 0, 0]], np.float32), opp=np.zeros((0, 4), np.float32),
               passer=0, ball=np.array([0, 0], np.float32))
    r1 = O.eval_point(f1, p, FLAT, 4.0, 3.0, 0.0)
    assert r1["t_team"] == math.inf and not r1["feasible"]


def test_airborne_samples_are_not_interceptable():
    # an opponent standing right under the chip's flight path cannot touch it
    p = Params(n_samples=64)
    f = Frame(team=np.array([[0, 0, 0, 0], [4, 0.3, 0, 0]], np.float32),
              opp=np.array([[0.8, 0.0, 0, 0]], np.float32), passer=0,
              ball=np.array([0, 0], np.float32))
    chip = O.eval_point(f, p, CHIP, 4.0, 4.0, 0.0)
    flat = O.eval_point(f, p, FLAT, 4.0, 4.0, 0.0)
    assert flat["t_opp"] < 0.3 and not flat["feasible"]
    assert chip["t_opp"] == math.inf and chip["feasible"]
