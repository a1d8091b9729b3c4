"""The seeded input generator: determinism, the stated distributions, the
lattice sizes of the workloads, and the batched workload's shapes.

Distribution checks use tests whose false-failure rate at the chosen
thresholds is below 1e-6 for a correct generator (Kolmogorov-Smirnov p-value
floors on 10^5 draws)."""
import numpy as np
import pytest
from scipy import stats

from paper_1909_07717_amd.framegen import (CHIP, FLAT, Params, config_batch, config_full,
                                           config_small, full_window, lattice_dims,
                                           random_frame, random_window, speeds_linear,
                                           uniform_batch_arrays, variants_for)

P = Params()


def test_same_seed_same_frame_other_seed_other_frame():
    for make in (config_small, config_full):
        a, b, c = make(7), make(7), make(8)
        assert a.team.tobytes() == b.team.tobytes() and a.opp.tobytes() == b.opp.tobytes()
        assert a.passer == b.passer and a.windows == b.windows and a.variants == b.variants
        assert a.team.tobytes() != c.team.tobytes()
    x, y = config_batch(3, 16), config_batch(3, 16)
    assert all(f.team.tobytes() == g.team.tobytes() and f.windows == g.windows
               for f, g in zip(x, y))


def test_values_are_float32_and_the_ball_sits_on_the_passer():
    f = config_full(11)
    assert f.team.dtype == np.float32 and f.opp.dtype == np.float32
    assert f.team.shape == (8, 4) and f.opp.shape == (8, 4)
    assert np.array_equal(f.ball, f.team[f.passer, :2])


def test_lattice_sizes_of_the_workloads():
    assert lattice_dims(0.2) == (61, 46) and config_small(0).n_points() == 2806
    assert lattice_dims(0.05) == (241, 181) and config_full(0).n_points() == 43621
    assert lattice_dims(0.1) == (121, 91)
    assert full_window(0.05) == (np.float32(0.05).item(), 0, 0, 241, 181)
    with pytest.raises(ValueError):
        lattice_dims(0.07)
    f = config_full(0)
    assert f.n_evals() == 43621 * 32


def test_speeds_and_variant_order():
    s = speeds_linear(16)
    assert s[0] == 1.0 and s[-1] == np.float32(6.5) and len(s) == 16
    assert np.allclose(np.diff(s), 5.5 / 15, atol=1e-6)
    v = variants_for([5.0, 2.0], flat=True, chip=True)
    assert v == [(FLAT, 2.0), (FLAT, 5.0), (CHIP, 2.0), (CHIP, 5.0)]
    assert speeds_linear(1) == [1.0]


def test_positions_are_uniform_on_the_field_and_velocities_uniform_in_the_disc():
    team, opp, passer = uniform_batch_arrays(5, 12500, 4, 4)
    xy = np.concatenate([team[..., :2].reshape(-1, 2), opp[..., :2].reshape(-1, 2)])
    v = np.concatenate([team[..., 2:].reshape(-1, 2), opp[..., 2:].reshape(-1, 2)])
    assert xy.shape[0] == 100000
    assert stats.kstest(xy[:, 0], stats.uniform(-6, 12).cdf).pvalue > 1e-6
    assert stats.kstest(xy[:, 1], stats.uniform(-4.5, 9).cdf).pvalue > 1e-6
    sp = np.hypot(v[:, 0], v[:, 1])
    assert sp.max() <= 1.5 + 1e-6
    # uniform in the disc: the squared speed is uniform on [0, 1.5^2], the
    # heading uniform on (-pi, pi]
    assert stats.kstest(sp ** 2, stats.uniform(0, 2.25).cdf).pvalue > 1e-6
    assert stats.kstest(np.arctan2(v[:, 1], v[:, 0]), stats.uniform(-np.pi, 2 * np.pi).cdf).pvalue > 1e-6
    # passers uniform over the team
    counts = np.bincount(passer, minlength=4)
    assert stats.chisquare(counts).pvalue > 1e-6


def test_random_frame_draw_order_matches_the_array_generator():
    """random_frame and uniform_batch_arrays draw the same distributions; for
    one frame of one seed they draw the same numbers in the same order."""
    f = random_frame(np.random.default_rng(99), 6, 6)
    team, opp, passer = uniform_batch_arrays(99, 1, 6, 6)
    assert np.array_equal(f.team, team[0]) and np.array_equal(f.opp, opp[0])
    assert f.passer == int(passer[0])


def test_batched_workload_shapes():
    frames = config_batch(0, 256)
    nt = np.array([f.n_team for f in frames])
    no = np.array([f.n_opp for f in frames])
    assert set(nt) == {6, 7, 8} and set(no) == {6, 7, 8}
    for f in frames:
        h, i0, j0, nx, ny = f.windows[0]
        assert h == np.float32(0.05).item()
        assert 21 <= nx <= 241 and 21 <= ny <= 181
        assert 0 <= i0 and i0 + nx <= 241 and 0 <= j0 and j0 + ny <= 181
        assert len(f.variants) == 8 and all(t == FLAT for t, _ in f.variants)
    pts = np.array([f.n_points() for f in frames])
    # window width ~ U(1, 12) m and height ~ U(1, 9) m: mean of the point
    # count near E[nx] E[ny] = 131 * 101
    assert 0.8 * 131 * 101 < pts.mean() < 1.2 * 131 * 101
    assert pts.min() < 2000 < 30000 < pts.max()


def test_random_window_stays_on_the_lattice():
    rng = np.random.default_rng(4)
    for h in (0.05, 0.1, 0.25):
        NX, NY = lattice_dims(h)
        for _ in range(200):
            hh, i0, j0, nx, ny = random_window(rng, h)
            assert 0 <= i0 and i0 + nx <= NX and 0 <= j0 and j0 + ny <= NY and nx >= 1 and ny >= 1
