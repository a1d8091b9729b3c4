"""Pins for the oracle's robot arrival-time model (reading of the cited,
unavailable predictor: straight-line motion with bounded acceleration and
speed that ends at rest on the point).

Independent checks: the textbook rest-to-rest minimum time (triangular and
trapezoidal profiles), and a brute-force minimum-time search that solves a
linear feasibility problem for a discretised double integrator with scipy's
HiGHS and bisects on the horizon.
"""
import math

import numpy as np
import pytest
from scipy.optimize import linprog

from oracle import oracle as O
from paper_1909_07717_amd.framegen import Params

P = Params()
A, V = P.amax, P.vmax


def _reachable_at_rest(T, delta, u, n=400):
    """Can a double integrator starting at 0 with speed u, |a| <= A, |v| <= V,
    be at rest at delta exactly at time T?  Piecewise-constant acceleration on
    n equal steps; variables are the n accelerations."""
    dt = T / n
    # v_k = u + dt * sum_{m<k} a_m ; x_n = sum_k (v_k dt + a_k dt^2 / 2)
    L = np.tril(np.ones((n, n)), -1) * dt          # v_k - u for k = 0..n-1
    x_row = (L.sum(axis=0) * dt + 0.5 * dt * dt)   # coefficient of a_m in x_n
    A_eq = np.vstack([np.full(n, dt), x_row])
    b_eq = np.array([-u, delta - u * T])
    Lv = np.tril(np.ones((n, n))) * dt             # v_{k+1} - u, k = 0..n-1
    A_ub = np.vstack([Lv, -Lv])
    b_ub = np.concatenate([np.full(n, V - u), np.full(n, V + u)])
    r = linprog(np.zeros(n), A_ub=A_ub, b_ub=b_ub, A_eq=A_eq, b_eq=b_eq,
                bounds=[(-A, A)] * n, method="highs")
    return r.status == 0


def _min_time_lp(delta, u, n=400):
    lo, hi = 0.0, 30.0
    assert _reachable_at_rest(hi, delta, u, n)
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        if _reachable_at_rest(mid, delta, u, n):
            hi = mid
        else:
            lo = mid
    return hi


def test_rest_to_rest_textbook():
    # triangular: accelerate half way, brake half way -> 2 sqrt(d / A)
    assert O.robot_time(P, 1.0, 0.0) == pytest.approx(2 * math.sqrt(1 / 3), abs=1e-12)
    # trapezoidal: d / V + V / A once d >= V^2 / A
    assert O.robot_time(P, 5.0, 0.0) == pytest.approx(5 / 3.25 + 3.25 / 3, abs=1e-12)
    assert O.robot_time(P, 0.0, 0.0) == 0.0
    # the two profiles meet at d = V^2 / A
    d = V * V / A
    assert O.robot_time(P, d * (1 - 1e-12), 0.0) == pytest.approx(O.robot_time(P, d, 0.0), abs=1e-9)


@pytest.mark.parametrize("delta,u", [
    (2.0, 1.5), (2.0, -1.5), (0.2, 1.5), (6.0, 1.0), (0.0, 1.5), (1.0, 0.0), (5.0, 0.0),
    (0.5, 3.25), (3.0, -3.0), (0.05, 0.3), (8.0, 2.5), (1.76, 0.0),
])
def test_robot_time_matches_lp_brute_force(delta, u):
    t_lp = _min_time_lp(delta, u)
    assert O.robot_time(P, delta, u) == pytest.approx(t_lp, abs=2e-4)


def test_robot_time_continuous_across_branches():
    # the closed form switches formula at u = 0, where the stopping distance
    # equals the distance left, and at the cruise threshold; evaluate on both
    # sides of each switch (the value has a square-root cusp at the second)
    e = 1e-10
    for delta in (0.05, 0.3, 1.0, 2.5, 6.0):
        assert O.robot_time(P, delta, -e) == pytest.approx(O.robot_time(P, delta, e), abs=1e-8)
        us = math.sqrt(2 * A * delta)
        if us <= V:
            assert O.robot_time(P, delta, us * (1 - e)) == pytest.approx(
                O.robot_time(P, delta, us * (1 + e)), abs=1e-4)
    for u in (0.0, 0.7, 2.0, 3.0):
        dacc = (V * V - u * u) / (2 * A) + V * V / (2 * A)
        assert O.robot_time(P, dacc * (1 - e), u) == pytest.approx(
            O.robot_time(P, dacc * (1 + e), u), abs=1e-8)
    # and it never decreases with the distance left when moving toward it
    for u in (0.0, 1.0, 3.0):
        ds = np.linspace(math.sqrt(2 * A * 0) + u * u / (2 * A) + 1e-9, 10, 2001)
        t = np.array([O.robot_time(P, x, u) for x in ds])
        assert np.all(np.diff(t) >= 0)


def test_robot_time_to_geometry():
    # at rest 2 m away: centre distance minus the radius, from rest
    r = P.robot_radius
    assert O.robot_time_to(P, (0, 0, 0, 0), 2.0, 0.0) == pytest.approx(O.robot_time(P, 2 - r, 0.0))
    # moving toward the point at 1 m/s
    assert O.robot_time_to(P, (0, 0, 1, 0), 2.0, 0.0) == pytest.approx(O.robot_time(P, 2 - r, 1.0))
    # perpendicular velocity is ignored
    assert O.robot_time_to(P, (0, 0, 0, 1.3), 2.0, 0.0) == pytest.approx(O.robot_time(P, 2 - r, 0.0))
    # inside the reach radius and at rest: already there
    assert O.robot_time_to(P, (0, 0, 0, 0), 0.05, 0.0) == 0.0
    # exactly on the point: no direction, speed along the line taken as 0
    assert O.robot_time_to(P, (1, 1, 1, 1), 1.0, 1.0) == 0.0
