"""Pins for the oracle's direction x power search (the paper's own DPPS form,
Sec. 4.2: every kick direction and power from the passer, the ball path
running until it stops or leaves the field, the pass received at the first
teammate's interception; Sec. 4.3 features).

* Ray length: closed forms for the distance to the field edge.
* Segment equivalence: along a ray whose ball reaches the field edge, the K
  ray samples are exactly the K samples of the segment from the ball to the
  edge point, so the first-teammate and first-opponent interception times
  must equal the ones the segment search (an independently written loop over
  the same primitives) finds for that target.
* Dense sampling: each side's sampled interception is the first of the K
  samples at which the side's earliest robot beats the ball, checked on a
  dense sub-sampled path.
* Invariants: no opponents (feasible iff a teammate intercepts, full margin
  term), mirror symmetry (y -> -y maps direction d to N - d), an added
  opponent never adds a feasible pass nor raises a score, passing points stay
  on the field, a faster kick never lets the team receive earlier on the same
  ray, and the refraction angle is 0 / pi on rays pointing at / away from the
  goal centre.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1909_07717_amd.framegen import (CHIP, FLAT, Frame, Params, random_frame,
                                           speeds_linear, variants_for)

N_DIRS = 128
W_TIME, W_REFR = 0.05, 0.1
RAY_BANDS = dict(eps_reach=1e-5)


def _frame(seed, n_team=6, n_opp=6, speeds=16, chip=True):
    f = random_frame(np.random.default_rng(seed), n_team, n_opp, Params())
    f.variants = variants_for(speeds_linear(speeds), flat=True, chip=chip)
    return f


@pytest.mark.parametrize("b,u,L", [
    ((0.0, 0.0), (1.0, 0.0), 6.0),
    ((0.0, 0.0), (0.0, -1.0), 4.5),
    ((0.0, 0.0), (math.sqrt(0.5), math.sqrt(0.5)), 4.5 / math.sqrt(0.5)),
    ((5.9, 0.0), (1.0, 0.0), 0.1),
    ((-3.0, 4.0), (-0.6, 0.8), 0.5 / 0.8),
    ((6.0, 0.0), (1.0, 0.0), 0.0),
])
def test_ray_length_closed_forms(b, u, L):
    p = Params()
    assert O.ray_length(p, b[0], b[1], u[0], u[1]) == pytest.approx(L, abs=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_ray_equals_segment_search_to_the_field_edge(seed):
    p = Params(n_samples=64)
    f = _frame(seed)
    b = np.asarray(f.ball, float)
    checked = 0
    for d in range(0, N_DIRS, 5):
        th = 2 * math.pi * d / N_DIRS
        u = np.array([math.cos(th), math.sin(th)])
        L = O.ray_length(p, b[0], b[1], u[0], u[1])
        if L < 0.5:
            continue
        c = b + L * u
        for vt, v0 in f.variants:
            D, sf = O.ball_range(p, vt, v0)
            if D < L + 1e-6 or (vt == CHIP and sf > L):
                continue
            r = O.ray_eval(f, p, N_DIRS, W_TIME, W_REFR, d, vt, v0)
            g = O.eval_point(f, p, vt, v0, c[0], c[1])
            assert r["length"] == pytest.approx(L, abs=1e-12)
            for key in ("t_team", "t_opp"):
                if math.isinf(g[key]):
                    assert math.isinf(r[key])
                else:
                    assert r[key] == pytest.approx(g[key], rel=1e-12, abs=1e-12)
            assert bool(r["feasible"]) == bool(g["feasible"])
            checked += 1
    assert checked > 20


def _side_first(p, f, d, vt, v0, robots, skip, dense):
    """First sample (of `dense` uniform samples over the ray) at which the
    side's earliest robot beats the ball, among samples the ball reaches."""
    b = np.asarray(f.ball, float)
    th = 2 * math.pi * d / N_DIRS
    u = np.array([math.cos(th), math.sin(th)])
    L = O.ray_length(p, b[0], b[1], u[0], u[1])
    D, sf = O.ball_range(p, vt, v0)
    for k in range(dense):
        s = (k + 1) / dense * L
        if s > D:
            return None, L
        if vt == CHIP and s < sf:
            continue
        tb = O.ball_time(p, vt, v0, s)
        pt = b + s * u
        tmin = min(O.robot_time_to(p, r, pt[0], pt[1])
                   for j, r in enumerate(np.asarray(robots).reshape(-1, 4)) if j != skip)
        if tmin <= tb:
            return k, L
    return None, L


@pytest.mark.parametrize("seed,d,vi", [(0, 3, 2), (0, 40, 9), (1, 77, 5), (2, 100, 14),
                                       (3, 64, 20), (4, 12, 27)])
def test_ray_crossings_against_dense_sampling(seed, d, vi):
    p = Params(n_samples=64)
    f = _frame(seed)
    vt, v0 = f.variants[vi]
    r = O.ray_eval(f, p, N_DIRS, W_TIME, W_REFR, d, vt, v0)
    mult = 32
    for robots, skip, k_or in ((f.team, f.passer, r["k_team"]), (f.opp, -1, r["k_opp"])):
        # the K samples are every mult-th sample of the dense path
        kd, _ = _side_first(p, f, d, vt, v0, robots, skip, p.n_samples * mult)
        k_sub, _ = _side_first(p, f, d, vt, v0, robots, skip, p.n_samples)
        if k_sub is None:
            assert k_or == p.n_samples
        else:
            assert k_or == k_sub
            # the dense crossing comes no later than the sampled one
            assert kd is not None and kd <= (k_sub + 1) * mult - 1


def test_ray_without_opponents():
    p = Params(n_samples=64)
    f = _frame(5)
    f.opp = np.zeros((0, 4), np.float32)
    r = O.ray_search(f, p, N_DIRS, W_TIME, W_REFR)
    fin = np.isfinite(r["t_team"])
    assert (r["mask"].astype(bool) == fin).all()
    assert np.isinf(r["t_opp"]).all()
    for d, v in zip(*np.nonzero(fin)[:2]):
        e = O.ray_eval(f, p, N_DIRS, W_TIME, W_REFR, int(d), *f.variants[int(v)])
        assert e["margin"] == math.inf
        # the margin term is at its cap
        dg = math.hypot(p.goal_x - e["x"], e["y"])
        rest = (p.w_angle * e["open_angle"] / math.pi + p.w_dist * (1 - dg / p.dist_norm)
                - W_TIME * e["t_team"] - W_REFR * e["refract"] / math.pi)
        assert e["score"] - rest == pytest.approx(p.w_margin * p.margin_cap_s, abs=1e-12)
        break


@pytest.mark.parametrize("seed", [6, 7])
def test_ray_mirror_symmetry(seed):
    p = Params(n_samples=64)
    f = _frame(seed)
    g = f.copy()
    for a in (g.team, g.opp):
        a[:, 1] *= -1
        a[:, 3] *= -1
    g.ball = np.array([f.ball[0], -f.ball[1]], np.float32)
    r = O.ray_search(f, p, N_DIRS, W_TIME, W_REFR)
    q = O.ray_search(g, p, N_DIRS, W_TIME, W_REFR)
    idx = (-np.arange(N_DIRS)) % N_DIRS
    for key in ("t_team", "t_opp", "s_recv", "score"):
        a, b = r[key], q[key][idx]
        both = np.isfinite(a) & np.isfinite(b)
        assert (np.isfinite(a) == np.isfinite(b)).all(), key
        np.testing.assert_allclose(a[both], b[both], rtol=0, atol=1e-9)
    assert (r["mask"] == q["mask"][idx]).all()


def test_ray_added_opponent_never_helps():
    p = Params(n_samples=64)
    f = _frame(8)
    r = O.ray_search(f, p, N_DIRS, W_TIME, W_REFR)
    g = f.copy()
    g.opp = np.vstack([f.opp, np.array([[1.0, 0.5, 0.0, 0.0]], np.float32)])
    q = O.ray_search(g, p, N_DIRS, W_TIME, W_REFR)
    assert (q["mask"] <= r["mask"]).all()
    ok = q["mask"].astype(bool)
    assert (q["score"][ok] <= r["score"][ok] + 1e-12).all()
    assert ((r["mask"] == 1) & (q["mask"] == 0)).any()


def test_ray_passing_points_on_the_field_and_monotone_in_power():
    p = Params(n_samples=64)
    f = _frame(9, chip=False)
    r = O.ray_search(f, p, N_DIRS, W_TIME, W_REFR)
    b = np.asarray(f.ball, float)
    th = 2 * np.pi * np.arange(N_DIRS) / N_DIRS
    s = r["s_recv"]
    fin = np.isfinite(s)
    ss = np.where(fin, s, 0.0)
    x = b[0] + ss * np.cos(th)[:, None]
    y = b[1] + ss * np.sin(th)[:, None]
    assert (np.abs(x[fin]) <= 6 + 1e-9).all() and (np.abs(y[fin]) <= 4.5 + 1e-9).all()
    # on one ray, a faster flat kick never reaches the team earlier
    for d in range(N_DIRS):
        ss = s[d][fin[d]]
        assert (np.diff(ss) >= -1e-12).all()


def test_ray_refraction_toward_and_away_from_the_goal():
    p = Params(n_samples=64)
    # ball on the x axis, a teammate further along +x and one along -x
    team = np.array([[-1.0, 0.0, 0, 0], [2.0, 0.0, 0, 0], [-4.0, 0.0, 0, 0]], np.float32)
    opp = np.array([[0.0, 4.0, 0, 0]], np.float32)
    f = Frame(team, opp, 0, team[0, :2].copy(), [], variants_for([3.0], True, False))
    fwd = O.ray_eval(f, p, N_DIRS, W_TIME, W_REFR, 0, FLAT, 3.0)
    back = O.ray_eval(f, p, N_DIRS, W_TIME, W_REFR, N_DIRS // 2, FLAT, 3.0)
    assert fwd["feasible"] and back["feasible"]
    assert fwd["refract"] == pytest.approx(0.0, abs=1e-12)
    assert back["refract"] == pytest.approx(math.pi, abs=1e-12)
    assert fwd["x"] < 2.0 and back["x"] > -4.0


def test_ray_bands_are_rare():
    # every (direction, power) entry decides up to K = 256 samples per side,
    # so it meets a crossing band more often than a lattice entry does; the
    # measured fraction on 8v8 frames is about 1.5e-3 (mostly crossing
    # bands, a quarter margin bands)
    p = Params(n_samples=256)
    fr = []
    for seed in (10, 11, 12):
        f = _frame(seed, n_team=8, n_opp=8, speeds=64, chip=False)
        r = O.ray_search(f, p, N_DIRS, W_TIME, W_REFR, bands=True, **RAY_BANDS)
        fr.append((r["ambig"] > 0).mean())
    assert max(fr) < 5e-3, fr
