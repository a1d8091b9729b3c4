"""Pins for the FP64 surrogate reference (oracle/mlp_ref.py): gradients by
central finite differences, GELU and its derivative by closed forms and
differences, Adam by a hand-worked step, the feature encoding on a
hand-built frame, top-k against a sort."""
import math

import numpy as np
import pytest

from oracle import mlp_ref as M
from paper_1909_07717_amd.framegen import Frame


def _small_params(seed):
    rng = np.random.default_rng(seed)
    parts = []
    for (r, c) in M.DIMS:
        parts.append((rng.normal(0, 1 / math.sqrt(c), (r, c)), rng.normal(0, 0.1, r)))
    return M.join(parts)


def test_param_count():
    assert M.param_count() == 66 * 512 + 512 + 2 * (512 * 512 + 512) + 512 * 2806 + 2806
    assert M.param_count() == 1999094


def test_gelu_closed_forms():
    assert M.gelu(np.array(0.0)) == 0.0
    # Phi(1) = 0.841344746...
    assert M.gelu(np.array(1.0)) == pytest.approx(0.8413447460685429, abs=1e-15)
    x = np.linspace(-4, 4, 81)
    h = 1e-6
    fd = (M.gelu(x + h) - M.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(M.gelu_grad(x), fd, atol=1e-8)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    flat = _small_params(1)
    X = rng.normal(0, 1, (3, M.IN))
    T = rng.normal(0, 0.3, (3, M.OUT))
    T[0, :5] = -np.inf          # infeasible cells are targets of 0
    T = M.targets(T)
    _, g = M.loss_and_grad(flat, X, T)
    idx = np.concatenate([rng.choice(o, 12, replace=False) for o in
                          np.cumsum([0] + [r * c + r for r, c in M.DIMS])[1:]]) - 1
    h = 1e-6
    for i in idx:
        e = np.zeros_like(flat)
        e[i] = h
        fp = M.mse(M.forward(flat + e, X)[0], T)
        fm = M.mse(M.forward(flat - e, X)[0], T)
        fd = (fp - fm) / (2 * h)
        assert abs(g[i] - fd) <= 1e-6 * max(abs(fd), 1e-4), (i, g[i], fd)


def test_weighted_and_ranking_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(4)
    flat = _small_params(2)
    X = rng.normal(0, 1, (2, M.IN))
    T = rng.uniform(0.06, 1.0, (2, M.OUT))
    T[rng.uniform(size=T.shape) < 0.7] = -np.inf
    T[1, :] = -np.inf                       # a row with nothing feasible: no ranking term
    kw = dict(pos_weight=6.0, ce_weight=0.05, tau=0.05)
    _, g = M.loss_and_grad(flat, X, T, **kw)
    h = 1e-6
    for i in rng.choice(flat.size, 40, replace=False):
        e = np.zeros_like(flat)
        e[i] = h
        fp = M.loss_and_grad(flat + e, X, T, **kw)[0]
        fm = M.loss_and_grad(flat - e, X, T, **kw)[0]
        fd = (fp - fm) / (2 * h)
        # central-difference round-off is about eps * loss / h ~ 1e-10 here
        assert abs(g[i] - fd) <= 1e-6 * abs(fd) + 2e-9, (i, g[i], fd)


def test_cross_entropy_limits():
    # identical scaled maps over the feasible cells: the loss is the entropy
    # of the target, and its gradient vanishes when every cell is feasible
    t = np.array([[0.1, 0.3, 0.2]])
    ce, g = M.cross_entropy(t, t, 0.1)
    p = np.exp(t / 0.1) / np.exp(t / 0.1).sum()
    assert ce[0] == pytest.approx(-(p * np.log(p)).sum(), abs=1e-12)
    np.testing.assert_allclose(g, 0.0, atol=1e-12)


def test_pooling_takes_the_max_of_each_cells_fine_points():
    rng = np.random.default_rng(5)
    fine = rng.uniform(0, 1, (2, 181, 241))
    fine[fine < 0.6] = -np.inf
    c = M.pool(fine)
    for (f, cj, ci) in [(0, 0, 0), (1, 45, 60), (0, 22, 30), (1, 10, 59)]:
        pts = [fine[f, J, I] for J in range(4 * cj - 2, 4 * cj + 2) for I in range(4 * ci - 2, 4 * ci + 2)
               if 0 <= J < 181 and 0 <= I < 241]
        assert c[f, cj * 61 + ci] == max(pts)
    # the fine windows of the 61 x 46 cells cover the fine lattice exactly once
    cover = np.zeros((181, 241), int)
    for cj in range(46):
        for ci in range(61):
            cover[max(4 * cj - 2, 0):min(4 * cj + 1, 180) + 1, max(4 * ci - 2, 0):min(4 * ci + 1, 240) + 1] += 1
    assert (cover == 1).all()


def test_adam_first_step_is_lr_times_sign():
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -1e-3, 0.0])
    w1, m, v = M.adam(w, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    # bias-corrected first step: m_hat = g, v_hat = g^2 -> step lr * g / (|g| + eps)
    np.testing.assert_allclose(w1, w - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert w1[0] == pytest.approx(0.99, abs=1e-9) and w1[2] == 0.5
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_features_of_a_hand_built_frame():
    team = np.array([[1.0, 1.0, 0.5, 0.0], [0.0, 0.0, 0.0, 0.0], [3.0, 0.0, 0.0, -1.625]])
    opp = np.array([[-6.0, 4.5, 3.25, 0.0], [0.5, 0.0, 0.0, 0.0]])
    f = Frame(team.astype(np.float32), opp.astype(np.float32), 1, np.array([0, 0], np.float32))
    x = M.features(f)
    # slot 0: passer (robot 1); slot 1: robot 0 (1.41 m); slot 2: robot 2 (3 m)
    np.testing.assert_allclose(x[0:4], [0, 0, 0, 0])
    np.testing.assert_allclose(x[4:8], [1 / 6, 1 / 4.5, 0.5 / 3.25, 0])
    np.testing.assert_allclose(x[8:12], [0.5, 0, 0, -0.5])
    assert not x[12:32].any()
    # opponents by distance: (0.5, 0) first, then (-6, 4.5)
    np.testing.assert_allclose(x[32:36], [0.5 / 6, 0, 0, 0])
    np.testing.assert_allclose(x[36:40], [-1, 1, 1, 0])
    assert not x[40:64].any() and x[64] == 0 and x[65] == 0


def test_topk_order_and_ties():
    y = np.array([0.1, 0.5, 0.5, -1.0, 0.7, 0.5])
    assert list(M.topk(y, 4)) == [4, 1, 2, 5]
    rng = np.random.default_rng(2)
    z = rng.normal(size=2806)
    assert list(M.topk(z, 64)) == list(np.argsort(-z, kind="stable")[:64])
