"""GPU parity of the running-point search (Sec. 5.2, Eq. 4) against the FP64
oracle: dpps_running_points through the C ABI.

Per zone point: the same points excluded (strictly inside the defense area,
decided in FP64 on both sides), scores within 1e-5 (the criteria run in
FP32 on the device); per zone: the same found flag, the chosen point's
oracle score within 1e-5 of the oracle's best, the reported score and the
five criteria within 1e-5 of the oracle's values at that point.  The marking
criterion's "nearer to the ball" test is also taken in FP64 on both sides;
points where an opponent ties within 1e-9 m^2 are excluded (none in practice).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1909_07717_amd.framegen import Params, config_small, random_frame
from paper_1909_07717_amd.zones import front_zones

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_07717_amd import binding
    return binding


def _f32(run):
    """The device receives float32 parameters: the oracle gets the same values."""
    v = dict(O.RUN_DEFAULTS)
    v.update(run)
    return {k: float(np.float32(x)) for k, x in v.items()}


def _check_frame(B, p, f, best, score, run):
    o = O.run_search(f, p, **_f32(run))
    amb = o["ambig"] != 0
    assert amb.mean() < 1e-3
    g = score.astype(np.float64)
    ok = ~amb
    assert (np.isinf(g[ok]) == np.isinf(o["score"][ok])).all()
    fin = ok & np.isfinite(o["score"])
    assert np.abs(g[fin] - o["score"][fin]).max(initial=0.0) <= 1e-5
    off = 0
    for w, z in enumerate(f.windows):
        n = z[3] * z[4]
        b = best[w]
        ob = int(o["best"][w])
        if ob < 0:
            assert b["found"] == 0
        else:
            assert b["found"] == 1
            k = int(b["j"]) * z[3] + int(b["i"])
            osc = o["score"][off:off + n]
            assert osc[k] >= osc[ob] - 1e-5
            assert abs(float(b["score"]) - osc[k]) <= 1e-5
            for key in ("goal", "ball", "angle", "guard", "defense"):
                assert abs(float(b[key]) - o[key][off + k]) <= 1e-5, key
            pts = O.points_of_window(p, z)
            assert float(b["x"]) == pytest.approx(pts[k, 0], abs=1e-6)
            assert float(b["y"]) == pytest.approx(pts[k, 1], abs=1e-6)
        off += n


def _run(B, s, frames, **run):
    best, sc = s.running_points(frames, **run)
    torch.cuda.synchronize()
    return B.run_best_host(best), sc.cpu().numpy()


def test_running_points_front_zones(B):
    p = Params(n_samples=64).as_f32()
    s = B.Searcher(p)
    rng = np.random.default_rng(4)
    frames = []
    for _ in range(12):
        f = random_frame(rng, int(rng.integers(6, 9)), int(rng.integers(6, 9)), Params())
        f.windows = front_zones(f.ball, p)
        frames.append(f)
    best, sc = _run(B, s, frames)
    zo = po = 0
    for f in frames:
        n = sum(z[3] * z[4] for z in f.windows)
        _check_frame(B, p, f, best[zo:zo + len(f.windows)], sc[po:po + n], {})
        zo += len(f.windows)
        po += n
    s.close()


@pytest.mark.parametrize("seed", [0, 1])
def test_running_points_attacking_half(B, seed):
    # the whole attacking half at 0.1 m: the defense area and the goal line
    # are inside the window
    p = Params(n_samples=64).as_f32()
    s = B.Searcher(p)
    f = random_frame(np.random.default_rng(seed), 8, 8, Params())
    f.windows = [(np.float32(0.1), 60, 0, 61, 91)]
    run = dict(w_goal=0.2, w_ball=0.2, w_angle=0.2, w_guard=0.2, w_defense=0.2, mark_radius=1.5)
    best, sc = _run(B, s, [f], **run)
    _check_frame(B, p, f, best, sc, run)
    assert np.isinf(sc).sum() >= 11 * 23   # at least 4.9 .. 5.9 x -1.1 .. 1.1
    s.close()


def test_running_points_edge_cases_batch_and_errors(B):
    p = Params(n_samples=64).as_f32()
    s = B.Searcher(p)
    alone = config_small(2)
    alone.opp = np.zeros((0, 4), np.float32)
    alone.windows = front_zones(alone.ball, p)
    # a zone entirely inside the defense area: nothing to choose
    boxed = config_small(3)
    boxed.windows = [(np.float32(0.1), 111, 35, 8, 20)]
    near = config_small(4)
    near.windows = front_zones(near.ball, p) + [(np.float32(0.2), 0, 0, 61, 46)]
    frames = [alone, boxed, near]
    best, sc = _run(B, s, frames)
    zo = po = 0
    for f in frames:
        n = sum(z[3] * z[4] for z in f.windows)
        _check_frame(B, p, f, best[zo:zo + len(f.windows)], sc[po:po + n], {})
        b1, s1 = _run(B, s, [f])
        assert b1[:len(f.windows)].tobytes() == best[zo:zo + len(f.windows)].tobytes()
        assert s1[:n].tobytes() == sc[po:po + n].tobytes()
        zo += len(f.windows)
        po += n
    assert best[len(alone.windows)]["found"] == 0
    for bad in (dict(ball_norm=0.0), dict(ang_lo=1.0, ang_hi=0.5), dict(w_goal=float("nan")),
                dict(def_depth=-1.0), dict(mark_radius=float("inf"))):
        with pytest.raises(B.DppsError):
            s.running_points([near], **bad)
    s.close()
