"""The lower bound on a robot's arrival time over a pass path that lets the
search kernel leave robots out of the robot stage (a robot whose bound is
not below every sample's current minimum changes no minimum).

The bound is restated here as the kernel forms it: with delta the robot's
distance to the path segment less its radius, both scaled by amax, the
arrival time in the robot stage's units (amax T / 2) is at least
sqrt(delta / 2) for delta <= vmax^2 / 2 and delta / (2 vmax) + vmax / 4
beyond, whatever the velocity; and, with U the largest approach speed (in
units of 1/sqrt 2, clamped to the limit) toward any point of the segment,
at least -U / sqrt 2 + R(U^2 + delta) when U < sqrt(delta).  Both are
checked against the oracle's arrival times (seconds) at every sample of
random paths, for robots slower and faster than vmax (the kernel clamps the
approach speed of the latter), and shown tight: a robot at rest on the
path's normal, or approaching at the limit, meets the first."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1909_07717_amd.framegen import Params

P = Params()
A, V, R = P.amax, P.vmax, P.robot_radius


def bound_seconds(dseg):
    delta = np.maximum(A * (dseg - R), 0.0)
    lb = np.where(delta <= 0.5 * V * V, np.sqrt(0.5 * delta), delta / (2 * V) + V / 4)
    return lb * 2.0 / A


def cone_bound_seconds(robot, bx, by, cx, cy):
    """The velocity-aware bound, in the path frame as the kernel forms it."""
    x, y, vx, vy = robot
    L = np.hypot(cx - bx, cy - by)
    ux, uy = (cx - bx) / L, (cy - by) / L
    ax, ay = bx - x, by - y
    t = -(ax * ux + ay * uy) * A
    q = (ay * ux - ax * uy) * A
    c = 1 / np.sqrt(2.0)
    we, wn = (vx * ux + vy * uy) * c, (vy * ux - vx * uy) * c
    LA = L * A
    tc = -t if t < 0 else (t - LA if t > LA else 0.0)
    delta = max(np.hypot(q, tc) - R * A, 0.0)
    h0, h1 = -t, LA - t
    sq = -1.0 if q < 0 else 1.0
    among = (h1 * wn - q * we) * sq >= 0 and (we * q - wn * h0) * sq >= 0
    u0 = (h0 * we + q * wn) / max(np.hypot(h0, q), 1e-15)
    u1 = (h1 * we + q * wn) / max(np.hypot(h1, q), 1e-15)
    U = np.hypot(we, wn) if among else max(u0, u1)
    U = min(max(U, -V * c), V * c)
    if U * abs(U) < delta:
        D = U * U + delta
        lb = -c * U + (D / (2 * V) + V / 2 if D > V * V else np.sqrt(D))
    else:
        lb = np.sqrt(0.5 * delta) if delta <= 0.5 * V * V else delta / (2 * V) + V / 4
    return lb * 2.0 / A


def seg_dist(px, py, ax, ay, bx, by):
    ex, ey = bx - ax, by - ay
    L2 = ex * ex + ey * ey
    t = np.clip(((px - ax) * ex + (py - ay) * ey) / max(L2, 1e-30), 0.0, 1.0)
    return np.hypot(px - ax - t * ex, py - ay - t * ey)


@pytest.mark.parametrize("vscale", [0.0, 0.5, 1.0, 1.6])
def test_bound_is_below_every_sample_time(vscale):
    rng = np.random.default_rng(int(vscale * 10) + 3)
    worst = np.inf
    for _ in range(150):
        bx, by = rng.uniform(-6, 6), rng.uniform(-4.5, 4.5)
        cx, cy = rng.uniform(-6, 6), rng.uniform(-4.5, 4.5)
        x, y = rng.uniform(-6, 6), rng.uniform(-4.5, 4.5)
        ang = rng.uniform(-np.pi, np.pi)
        sp = vscale * V * np.sqrt(rng.uniform())
        robot = (x, y, sp * np.cos(ang), sp * np.sin(ang))
        lb = bound_seconds(seg_dist(x, y, bx, by, cx, cy))
        lbc = cone_bound_seconds(robot, bx, by, cx, cy)
        assert lbc >= lb * (1 - 1e-9)
        for f in (np.arange(64) + 1) / 64:
            t = O.robot_time_to(P, robot, bx + f * (cx - bx), by + f * (cy - by))
            worst = min(worst, t - lbc)
            assert t >= lbc * (1 - 1e-6), (robot, f, t, lb, lbc)
    assert np.isfinite(worst)


def test_bound_is_met():
    # at rest, straight ahead of the path: the bound is the rest-to-rest time
    for d in (0.3, 0.8, 2.0, 5.0):
        robot = (0.0, d, 0.0, 0.0)
        lb = bound_seconds(np.array(d))
        t = O.robot_time_to(P, robot, 0.0, 0.0)
        assert t >= lb
    # approaching the nearest path point at the speed limit (delta past
    # vmax^2 / 2 scaled), the time equals the bound
    d = R + 3.0 * V * V / A
    robot = (0.0, d, 0.0, -V)
    lb = float(bound_seconds(np.array(d)))
    t = O.robot_time_to(P, robot, 0.0, 0.0)
    assert t == pytest.approx(lb, rel=1e-9)
    # approaching at the best speed sqrt(delta) (below the limit): equal too
    d = R + 0.2 * V * V / A
    delta = A * (d - R)
    robot = (0.0, d, 0.0, -np.sqrt(delta) * np.sqrt(2.0))
    lb = float(bound_seconds(np.array(d)))
    t = O.robot_time_to(P, robot, 0.0, 0.0)
    assert t == pytest.approx(lb, rel=1e-6)  # the velocity is rounded to float32


def test_velocity_bound_near_and_on_the_path_line():
    """Robots close to the segment, on its line (behind the ball, past the
    point, on it), moving along, across and away from it."""
    rng = np.random.default_rng(11)
    bx, by, cx, cy = -2.0, -1.0, 3.0, 2.0
    ex, ey = (cx - bx) / np.hypot(cx - bx, cy - by), (cy - by) / np.hypot(cx - bx, cy - by)
    for along in (-0.8, 0.0, 0.3, 0.7, 1.0, 1.4):
        for off in (0.0, 0.05, 0.3, -0.3, 1.5):
            for ang in np.linspace(-np.pi, np.pi, 9)[:-1]:
                sp = V * rng.uniform(0.2, 1.5)
                x = bx + along * (cx - bx) - off * ey
                y = by + along * (cy - by) + off * ex
                robot = (x, y, sp * np.cos(ang), sp * np.sin(ang))
                lbc = cone_bound_seconds(robot, bx, by, cx, cy)
                for f in (np.arange(64) + 1) / 64:
                    t = O.robot_time_to(P, robot, bx + f * (cx - bx), by + f * (cy - by))
                    assert t >= lbc * (1 - 1e-6), (robot, f, t, lbc)
