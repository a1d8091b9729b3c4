"""Golden fixtures: the paper's printed constants, and a regression record of
the oracle written by ``tests/golden/make_oracle_golden.py`` (oracle only)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1909_07717_amd.framegen import Params, config_small, speeds_linear, FLAT

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _constants():
    out = {}
    with open(os.path.join(HERE, "paper_constants.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            name, val = line.split()[:2]
            out[name] = float(val)
    return out


def test_paper_constants_are_the_ones_used():
    c = _constants()
    p = Params()
    assert p.slide_ratio == pytest.approx(c["slide_ratio"], abs=1e-15)
    assert p.vmax == c["robot_top_speed_ms"]
    assert c["direction_count"] * c["power_count"] * c["robots_on_field"] == c["sbip_count"]
    assert 360.0 / c["direction_count"] == c["direction_step_deg"]
    sp = speeds_linear(16)
    assert sp[0] == c["power_min_ms"] and sp[-1] == c["power_max_ms"]
    # the slide phase ends at 5/7 of the kick speed: at 4 m/s, v1 = 20/7
    D, _ = O.ball_range(p, FLAT, 4.0)
    assert D == pytest.approx((16 - (20 / 7) ** 2) / 10 + (20 / 7) ** 2, abs=1e-12)


@pytest.mark.parametrize("rec", json.load(open(os.path.join(HERE, "oracle_small_frames.json"))))
def test_oracle_regression_record(rec):
    p = Params(n_samples=64).as_f32()
    r = O.search_frame(config_small(rec["seed"]), p)
    s = r["score"]
    assert int(r["mask"].sum()) == rec["n_feasible"]
    assert int(r["best"]) == rec["best"]
    assert float(r["best_score"]) == float(rec["best_score"])
    assert math.isclose(float(s[np.isfinite(s)].sum()), float(rec["score_sum"]), rel_tol=1e-12)
    assert int(np.isfinite(r["t_team"]).sum()) == rec["t_team_finite"]
    assert int(np.isfinite(r["t_opp"]).sum()) == rec["t_opp_finite"]
