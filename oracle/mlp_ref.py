"""FP64 reference of the learned surrogate (test infrastructure only).

The network maps a frame's 66 input features to the 2806 cells of its 20 cm
score map: three hidden layers of 512 with GELU (exact, erf form) and a
linear output; it is trained with the mean squared error against the exact
search's map (infeasible cells read as 0) and Adam.  Everything here is plain
NumPy in float64; it shares nothing with the HIP path.

Parameter vector layout (the library's real layout): W0 [512][66], b0 [512],
W1 [512][512], b1, W2 [512][512], b2, W3 [2806][512], b3 [2806].
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

IN, HID, OUT = 66, 512, 2806
DIMS = [(HID, IN), (HID, HID), (HID, HID), (OUT, HID)]


def param_count() -> int:
    return sum(o * i + o for o, i in DIMS)


def split(flat):
    """[(W, b)] views of a flat parameter vector (float64 copy)."""
    flat = np.asarray(flat, np.float64)
    out, o = [], 0
    for (r, c) in DIMS:
        W = flat[o:o + r * c].reshape(r, c)
        o += r * c
        b = flat[o:o + r]
        o += r
        out.append((W, b))
    assert o == flat.size
    return out


def join(parts) -> np.ndarray:
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in parts])


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    cdf = 0.5 * (1.0 + erf(x / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return cdf + x * pdf


def features(frame, field_len=12.0, field_wid=9.0, vmax=3.25) -> np.ndarray:
    """Input vector of one frame: team (passer first, then by distance to the
    ball, 8 slots), opponents (by distance to the ball, 8 slots), each as
    (x / (L/2), y / (W/2), vx / vmax, vy / vmax); then the ball."""
    x = np.zeros(IN)
    b = np.asarray(frame.ball, np.float64)
    for side, robots in ((0, np.asarray(frame.team, np.float64).reshape(-1, 4)),
                         (1, np.asarray(frame.opp, np.float64).reshape(-1, 4))):
        keys = []
        for r, rb in enumerate(robots):
            d2 = (rb[0] - b[0]) ** 2 + (rb[1] - b[1]) ** 2
            if side == 0 and r == frame.passer:
                d2 = -1.0
            keys.append((d2, r))
        keys.sort()
        for s, (_, r) in enumerate(keys[:8]):
            rb = robots[r]
            x[(side * 8 + s) * 4:(side * 8 + s) * 4 + 4] = (
                rb[0] * 2 / field_len, rb[1] * 2 / field_wid, rb[2] / vmax, rb[3] / vmax)
    x[64] = b[0] * 2 / field_len
    x[65] = b[1] * 2 / field_wid
    return x


def forward(flat, X):
    """Outputs [B][2806] and the cache for backward."""
    parts = split(flat)
    a = np.asarray(X, np.float64)
    cache = [a]
    for l, (W, b) in enumerate(parts):
        z = a @ W.T + b
        if l < 3:
            cache.append(z)
            a = gelu(z)
            cache.append(a)
        else:
            a = z
    return a, cache


def targets(score_maps):
    t = np.asarray(score_maps, np.float64).copy()
    t[~np.isfinite(t)] = 0.0
    return t


def weights(T, pos_weight=0.0):
    """Per-cell loss weights 1 + pos_weight * target."""
    return 1.0 + pos_weight * T


def mse(Y, T, pos_weight=0.0) -> float:
    return float(np.mean(weights(T, pos_weight) * (Y - T) ** 2))


def backward(flat, cache, dY) -> np.ndarray:
    """Gradient (flat, real layout) given dL/dY."""
    parts = split(flat)
    grads = [None] * 4
    dz = dY
    for l in (3, 2, 1, 0):
        a_in = cache[0] if l == 0 else cache[2 * l]
        W, _ = parts[l]
        grads[l] = (dz.T @ a_in, dz.sum(axis=0))
        if l > 0:
            z_prev = cache[2 * l - 1]
            dz = (dz @ W) * gelu_grad(z_prev)
    return join(grads)


def cross_entropy(Y, T_raw, tau):
    """Per-row cross-entropy between the target distribution softmax(t / tau)
    over the feasible cells (finite t) and softmax(y / tau) over all cells,
    and its gradient with respect to Y; rows with no feasible cell give 0."""
    Y = np.asarray(Y, np.float64)
    T_raw = np.asarray(T_raw, np.float64)
    ce = np.zeros(Y.shape[0])
    grad = np.zeros_like(Y)
    for r in range(Y.shape[0]):
        feas = np.isfinite(T_raw[r])
        if not feas.any():
            continue
        ly = Y[r] / tau
        ly = ly - ly.max()
        logp = ly - np.log(np.exp(ly).sum())
        lt = np.where(feas, T_raw[r] / tau, -np.inf)
        lt = lt - lt[feas].max()
        q = np.where(feas, np.exp(lt), 0.0)
        q /= q.sum()
        ce[r] = -(q * logp).sum()
        grad[r] = (np.exp(logp) - q) / tau
    return ce, grad


def loss_and_grad(flat, X, T_raw, pos_weight=0.0, ce_weight=0.0, tau=0.02):
    """Training loss (weighted squared error on targets with -inf read as 0,
    plus ce_weight times the mean cross-entropy) and its flat gradient."""
    T = targets(T_raw)
    Y, cache = forward(flat, X)
    loss = mse(Y, T, pos_weight)
    dY = 2.0 * weights(T, pos_weight) * (Y - T) / Y.size
    if ce_weight > 0.0:
        ce, g = cross_entropy(Y, T_raw, tau)
        loss += ce_weight * ce.mean()
        dY = dY + ce_weight * g / Y.shape[0]
    return loss, backward(flat, cache, dY)


def pool(fine, fnx=241, fny=181, cnx=61, cny=46):
    """Coarse labels: cell (ci, cj) takes the largest fine score over the fine
    points {4ci-2..4ci+1} x {4cj-2..4cj+1} inside the fine lattice."""
    fine = np.asarray(fine, np.float64).reshape(-1, fny, fnx)
    out = np.full((fine.shape[0], cny * cnx), -np.inf)
    for cj in range(cny):
        for ci in range(cnx):
            I0, I1 = max(4 * ci - 2, 0), min(4 * ci + 1, fnx - 1)
            J0, J1 = max(4 * cj - 2, 0), min(4 * cj + 1, fny - 1)
            out[:, cj * cnx + ci] = fine[:, J0:J1 + 1, I0:I1 + 1].reshape(fine.shape[0], -1).max(1)
    return out


def adam(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step (t counts from 1)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def topk(y, k):
    """Indices of the k largest entries, descending, ties to the lower index."""
    y = np.asarray(y)
    order = np.lexsort((np.arange(y.size), -y))
    return order[:k]
