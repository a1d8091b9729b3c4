"""The paper's qualitative claims about the feasible set (Sec. 4.3, figure of
feasible pass points), reproduced on the oracle.

(a) teammates each closely marked by an opponent -> few feasible points;
    nobody marked -> a dense feasible set;
(b) a pass line blocked by an opponent -> no flat pass behind it, but chip
    passes over it remain.
"""
import math

import numpy as np

from oracle import oracle as O
from paper_1909_07717_amd.framegen import Params, Frame, FLAT, CHIP, full_window, variants_for

P = Params(n_samples=64)


def _team():
    team = np.array([[-3.0, 0.0, 0, 0], [0.5, 2.5, 0, 0], [1.0, -2.0, 0, 0],
                     [3.5, 1.0, 0, 0], [3.0, -3.0, 0, 0], [-1.0, -3.5, 0, 0]], np.float32)
    return team


def _feasible_fraction(opp):
    f = Frame(team=_team(), opp=np.asarray(opp, np.float32), passer=0,
              ball=np.array([-3.0, 0.0], np.float32), windows=[full_window(0.25)],
              variants=variants_for([2.5, 4.0, 5.5], flat=True, chip=False))
    r = O.search_frame(f, P)
    return r["mask"].mean()


def test_marked_teammates_leave_few_feasible_points():
    team = _team()
    # each receiver shadowed 0.25 m away, between it and the passer
    marks = []
    for x, y, _, _ in team[1:]:
        d = np.array([-3.0 - x, 0.0 - y])
        d /= np.linalg.norm(d)
        marks.append([x + 0.25 * d[0], y + 0.25 * d[1], 0, 0])
    marked = _feasible_fraction(marks)
    # the same five opponents parked in a far corner mark nobody
    unmarked = _feasible_fraction([[-5.8, 4.3 - 0.3 * i, 0, 0] for i in range(5)])
    assert unmarked > 0.3
    assert marked < 0.5 * unmarked


def test_blocked_line_leaves_only_chip_passes():
    team = np.array([[0, 0, 0, 0], [4, 0.5, 0, 0]], np.float32)
    opp = np.array([[1.0, 0.0, 0, 0]], np.float32)
    f = Frame(team=team, opp=opp, passer=0, ball=np.array([0, 0], np.float32))
    flat = O.eval_point(f, P, FLAT, 4.0, 4.0, 0.0)
    chip = O.eval_point(f, P, CHIP, 4.0, 4.0, 0.0)
    assert not flat["feasible"] and flat["t_opp"] < flat["t_team"]
    assert chip["feasible"] and math.isinf(chip["t_opp"])
    # along the blocked line beyond the opponent no flat pass survives at any
    # speed; near the receiver (3 m and beyond, where the teammate is first to
    # the landing zone) some chip survives at every point
    for x in np.linspace(2.0, 5.5, 8):
        for v0 in np.linspace(1.0, 6.5, 16):
            assert not O.eval_point(f, P, FLAT, float(v0), float(x), 0.0)["feasible"]
        if x >= 3.0:
            assert any(O.eval_point(f, P, CHIP, float(v0), float(x), 0.0)["feasible"]
                       for v0 in np.linspace(1.0, 6.5, 16))
