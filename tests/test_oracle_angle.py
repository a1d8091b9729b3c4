"""Pins for the oracle's open goal angle (Sec. 4.3 shoot-angle feature,
Sec. 4.4 valid angle against opponent robots), by ray casting.

10^5 rays are cast over the goal mouth; a ray is blocked when it meets an
opponent disc ahead of the candidate.  The open fraction times the mouth's
angular width must match the oracle's interval union within a few ray
spacings.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1909_07717_amd.framegen import Params

P = Params()
NR = 100_000


def _ray_cast(cx, cy, opp, p=P):
    dx = max(p.goal_x - cx, p.goal_eps)
    lo = math.atan2(-0.5 * p.goal_width - cy, dx)
    hi = math.atan2(0.5 * p.goal_width - cy, dx)
    th = lo + (np.arange(NR) + 0.5) * (hi - lo) / NR
    ex, ey = np.cos(th), np.sin(th)
    blocked = np.zeros(NR, bool)
    for o in np.asarray(opp, float).reshape(-1, 4):
        if o[0] >= p.goal_x:
            continue
        rx, ry = o[0] - cx, o[1] - cy
        if rx * rx + ry * ry <= p.robot_radius ** 2:
            return 0.0, hi - lo
        t0 = rx * ex + ry * ey                 # closest approach along the ray
        miss2 = rx * rx + ry * ry - t0 * t0    # squared miss distance
        blocked |= (t0 > 0) & (miss2 <= p.robot_radius ** 2)
    return (hi - lo) * (1.0 - blocked.mean()), hi - lo


def test_no_opponents_is_the_mouth_angle():
    # seen from (4.5, 0) the 1.2 m mouth 1.5 m away spans 2 atan(0.6 / 1.5)
    assert O.open_angle(P, 4.5, 0.0, []) == pytest.approx(2 * math.atan(0.6 / 1.5), abs=1e-15)
    assert O.open_angle(P, 4.5, 0.0, []) == pytest.approx(0.761013, abs=1e-6)
    # on the goal line the depth is floored at 1 mm: almost a half turn
    assert O.open_angle(P, 6.0, 0.0, []) / math.pi == pytest.approx(
        2 * math.atan(0.6 / 1e-3) / math.pi, abs=1e-15)


@pytest.mark.parametrize("seed", range(12))
def test_open_angle_matches_ray_casting(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 9))
    # half the cases crowd the opponents between the candidate and the goal
    cx, cy = rng.uniform(-5, 5.5), rng.uniform(-3, 3)
    if seed % 2:
        ox = rng.uniform(cx, 6.0, n)
        oy = cy + (rng.uniform(-0.8, 0.8, n)) * (6.0 - ox) / max(6.0 - cx, 1e-3) + rng.uniform(-0.3, 0.3, n)
    else:
        ox = rng.uniform(-6, 6, n)
        oy = rng.uniform(-4.5, 4.5, n)
    opp = np.stack([ox, oy, np.zeros(n), np.zeros(n)], 1)
    got = O.open_angle(P, cx, cy, opp)
    want, width = _ray_cast(cx, cy, opp)
    assert got == pytest.approx(want, abs=4 * 2 * n * width / NR + 1e-12)


def test_overlapping_and_nested_shadows():
    # three discs on one line toward the goal: nested shadows count once
    opp = [[3, 0, 0, 0], [4, 0, 0, 0], [5, 0, 0, 0], [4.5, 0.12, 0, 0]]
    got = O.open_angle(P, 0.0, 0.0, opp)
    want, width = _ray_cast(0.0, 0.0, opp)
    assert got == pytest.approx(want, abs=16 * width / NR)
    assert got < width


def test_inside_a_disc_and_behind_the_line():
    assert O.open_angle(P, 2.0, 0.0, [[2.05, 0.0, 0, 0]]) == 0.0
    # an opponent at or beyond the goal line does not block
    assert O.open_angle(P, 4.0, 0.0, [[6.0, 0.0, 0, 0]]) == O.open_angle(P, 4.0, 0.0, [])
    # teammates never block: only the opponent list is consulted
    assert O.open_angle(P, 4.0, 0.0, []) == pytest.approx(2 * math.atan(0.6 / 2.0))
