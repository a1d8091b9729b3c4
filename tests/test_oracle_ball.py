"""Pins for the oracle's ball model (Sec. 4.1, ideal two-phase ball; chip reading).

The closed forms in the oracle are checked against a general-purpose ODE
integrator (scipy's RK45 with event location) driven by the equations of
motion alone, and against hand-derived constants for a 4 m/s kick.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import oracle as O
from paper_1909_07717_amd.framegen import Params, FLAT, CHIP

P = Params()


def _flat_time_by_ode(v0, s_target, p=P):
    """Integrate ds/dt = v, dv/dt = -a(v) with a = slide_decel while
    v > ratio * v0, then roll_decel until rest.  Returns the time at which
    s reaches s_target (inf if the ball stops first)."""
    v1 = p.slide_ratio * v0
    t0, y0 = 0.0, [0.0, v0]
    for decel, v_end in ((p.slide_decel, v1), (p.roll_decel, 0.0)):
        def rhs(t, y, a=decel):
            return [y[1], -a]

        def ev_target(t, y):
            return y[0] - s_target
        ev_target.terminal = True
        ev_target.direction = 1

        def ev_speed(t, y, ve=v_end):
            return y[1] - ve
        ev_speed.terminal = True
        ev_speed.direction = -1
        sol = solve_ivp(rhs, (t0, t0 + 100.0), y0, events=[ev_target, ev_speed],
                        rtol=1e-12, atol=1e-13, max_step=0.01)
        if sol.t_events[0].size:
            return float(sol.t_events[0][0])
        t0 = float(sol.t_events[1][0])
        y0 = [float(sol.y_events[1][0][0]), v_end]
    return math.inf


def _chip_time_by_ode(v0, s_target, p=P):
    """Projectile flight (no drag) from the ground at the chip angle, then a
    roll from the horizontal speed at roll_decel.  Time at which the
    horizontal distance reaches s_target, and the landing distance."""
    th = p.chip_angle

    def rhs(t, y):
        return [y[2], y[3], 0.0, -p.gravity]

    def land(t, y):
        return y[1]
    land.terminal = True
    land.direction = -1

    def target(t, y):
        return y[0] - s_target
    target.terminal = False
    target.direction = 1
    y0 = [0.0, 0.0, v0 * math.cos(th), v0 * math.sin(th)]
    sol = solve_ivp(rhs, (0.0, 100.0), y0, events=[land, target], rtol=1e-12, atol=1e-13,
                    max_step=0.01)
    t_land = float(sol.t_events[0][0])
    x_land = float(sol.y_events[0][0][0])
    if sol.t_events[1].size and sol.t_events[1][0] <= t_land:
        return float(sol.t_events[1][0]), x_land
    vh = v0 * math.cos(th)

    def rhs2(t, y):
        return [y[1], -p.roll_decel]

    def tgt2(t, y):
        return y[0] - s_target
    tgt2.terminal = True
    tgt2.direction = 1

    def stop(t, y):
        return y[1]
    stop.terminal = True
    stop.direction = -1
    sol2 = solve_ivp(rhs2, (t_land, t_land + 100.0), [x_land, vh], events=[tgt2, stop],
                     rtol=1e-12, atol=1e-13, max_step=0.01)
    if sol2.t_events[0].size:
        return float(sol2.t_events[0][0]), x_land
    return math.inf, x_land


def test_flat_constants_at_4ms():
    # v1 = 5/7 * 4 = 20/7; slide time (4 - 20/7)/5 = 8/35; slide distance
    # (16 - 400/49)/10 = 384/490; roll distance (400/49)/(2*0.5) = 400/49;
    # roll time (20/7)/0.5 = 40/7.
    D, sf = O.ball_range(P, FLAT, 4.0)
    assert sf == 0.0
    assert D == pytest.approx(384 / 490 + 400 / 49, abs=1e-12)
    assert D == pytest.approx(8.946939, abs=1e-6)
    assert O.ball_time(P, FLAT, 4.0, 384 / 490) == pytest.approx(8 / 35, abs=1e-12)
    assert O.ball_time(P, FLAT, 4.0, D) == pytest.approx(8 / 35 + 40 / 7, abs=1e-9)
    assert O.ball_time(P, FLAT, 4.0, D + 1e-6) == math.inf


@pytest.mark.parametrize("v0", [1.0, 2.5, 4.0, 6.5])
@pytest.mark.parametrize("frac", [0.01, 0.05, 0.2, 0.5, 0.9, 0.999])
def test_flat_time_matches_ode(v0, frac):
    D, _ = O.ball_range(P, FLAT, v0)
    s = frac * D
    assert O.ball_time(P, FLAT, v0, s) == pytest.approx(_flat_time_by_ode(v0, s), abs=2e-8)


def test_chip_constants_at_4ms():
    # 45 degrees: v_h = v_z = 4/sqrt(2); flight 2 v_z / g; carry v0^2 / g.
    D, sf = O.ball_range(P, CHIP, 4.0)
    assert sf == pytest.approx(16 / 9.81, abs=1e-12)
    assert D == pytest.approx(16 / 9.81 + 8 / (2 * 0.5), abs=1e-12)
    assert O.ball_time(P, CHIP, 4.0, sf) == pytest.approx(2 * (4 / math.sqrt(2)) / 9.81, abs=1e-12)


@pytest.mark.parametrize("v0", [1.0, 2.5, 4.0, 6.5])
@pytest.mark.parametrize("frac", [0.1, 0.5, 0.95, 1.05, 1.5, 3.0])
def test_chip_time_matches_ode(v0, frac):
    D, sf = O.ball_range(P, CHIP, v0)
    s = frac * sf
    if s > D:
        s = 0.99 * D
    t_ode, x_land = _chip_time_by_ode(v0, s)
    assert x_land == pytest.approx(sf, abs=1e-8)
    assert O.ball_time(P, CHIP, v0, s) == pytest.approx(t_ode, abs=2e-8)


@pytest.mark.parametrize("vtype", [FLAT, CHIP])
@pytest.mark.parametrize("v0", [1.0, 3.3, 6.5])
def test_time_increasing_and_distance_inverse(vtype, v0):
    D, sf = O.ball_range(P, vtype, v0)
    s = np.linspace(1e-3, D * (1 - 1e-9), 400)
    t = np.array([O.ball_time(P, vtype, v0, x) for x in s])
    assert np.all(np.diff(t) > 0)
    back = np.array([O.ball_dist(P, vtype, v0, x) for x in t])
    np.testing.assert_allclose(back, s, atol=1e-9)


def test_faster_kick_is_never_later():
    # the paper's ball model: a harder kick is ahead at every time
    for vtype in (FLAT, CHIP):
        for s in (0.5, 2.0, 5.0):
            ts = [O.ball_time(P, vtype, v, s) for v in np.linspace(1.0, 6.5, 23)]
            fin = [x for x in ts if math.isfinite(x)]
            assert all(a >= b for a, b in zip(fin, fin[1:]))
