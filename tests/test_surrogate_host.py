"""Host-side helpers of the surrogate path: the 5 cm re-score windows of a
20 cm cell, the network-free geometric proposals, and packing frames with
per-frame windows.  CPU only."""
import numpy as np
import pytest

from paper_1909_07717_amd.framegen import (Params, frames_from_arrays, uniform_batch_arrays,
                                           variants_for)
from paper_1909_07717_amd.surrogate import cell_windows, geometric_cells


def test_cell_windows_cover_the_fine_points_of_each_cell():
    # every fine point of the 241 x 181 lattice lies in exactly one cell's
    # window, and cell c of an axis holds the fine points 4c-2 .. 4c+1
    cells = np.arange(61 * 46)[None, :]
    w = cell_windows(cells)[0]
    cover = np.zeros((181, 241), np.int32)
    for h, i0, j0, nx, ny in w:
        assert np.float32(h) == np.float32(0.05)
        cover[int(j0):int(j0 + ny), int(i0):int(i0 + nx)] += 1
    assert (cover == 1).all()
    c = 17 + 61 * 9
    h, i0, j0, nx, ny = w[c]
    assert (i0, j0, nx, ny) == (4 * 17 - 2, 4 * 9 - 2, 4, 4)
    # edge cells are clipped
    assert tuple(w[0][1:]) == (0, 0, 2, 2)
    assert tuple(w[61 * 46 - 1][1:]) == (238, 178, 3, 3)


def test_geometric_cells_rank_reachable_cells_by_the_robot_free_terms():
    P = Params()
    team, _, passer = uniform_batch_arrays(3, 32)
    var = variants_for([4.0], flat=True, chip=False)
    k = 64
    cells = geometric_cells(team, passer, var, k)
    assert cells.shape == (32, k)
    X = 0.2 * (np.arange(61) - 30.0)
    Y = 0.2 * (np.arange(46) - 22.5)
    v1 = P.slide_ratio * 4.0
    D = (16 - v1 * v1) / (2 * P.slide_decel) + v1 * v1 / (2 * P.roll_decel)
    for f in range(32):
        bx, by = team[f, passer[f], 0], team[f, passer[f], 1]
        cx, cy = X[cells[f] % 61], Y[cells[f] // 61]
        assert (np.hypot(cx - bx, cy - by) <= D + 0.15 + 1e-9).all()
        # priors are non-increasing along the list, ties broken by cell index
        dx = np.maximum(6.0 - cx, 1e-3)
        prior = (0.5 * (np.arctan2(0.6 - cy, dx) - np.arctan2(-0.6 - cy, dx)) / np.pi
                 + 0.3 * (1 - np.hypot(cx - 6.0, cy) / 15.0))
        assert (np.diff(prior) <= 1e-12).all()
        same = np.abs(np.diff(prior)) <= 1e-12
        assert (np.diff(cells[f])[same] > 0).all()
        # no reachable cell outside the list beats the k-th one
        AX, AY = np.meshgrid(X, Y)
        AX, AY = AX.ravel(), AY.ravel()
        reach = np.hypot(AX - bx, AY - by) <= D + 0.15
        dxa = np.maximum(6.0 - AX, 1e-3)
        pa = (0.5 * (np.arctan2(0.6 - AY, dxa) - np.arctan2(-0.6 - AY, dxa)) / np.pi
              + 0.3 * (1 - np.hypot(AX - 6.0, AY) / 15.0))
        rest = np.setdiff1d(np.flatnonzero(reach), cells[f])
        assert (pa[rest] <= prior[-1] + 1e-12).all()


def test_pack_uniform_with_per_frame_windows_matches_pack():
    B = pytest.importorskip("paper_1909_07717_amd.binding")
    try:
        B.lib()
    except Exception as e:  # pragma: no cover - library not built
        pytest.skip(f"libdpps not loadable: {e}")
    p = Params(n_samples=64).as_f32()
    team, opp, passer = uniform_batch_arrays(8, 5)
    var = variants_for([4.0], flat=True, chip=False)
    cells = geometric_cells(team, passer, var, 7)
    wins = cell_windows(cells)
    a = B.pack_uniform(team, opp, passer, wins, var, p)
    frames = frames_from_arrays(team, opp, passer, [None] * 1, var)
    for f, fr in enumerate(frames):
        fr.windows = [tuple(float(x) if c == 0 else int(x) for c, x in enumerate(w))
                      for w in wins[f]]
    b = B.pack(frames, p)
    assert a.frames.tobytes() == b.frames.tobytes()
    assert a.robots.tobytes() == b.robots.tobytes()
    assert a.windows.tobytes() == b.windows.tobytes()
    assert a.variants.tobytes() == b.variants.tobytes()
    assert a.total == b.total
