"""Zones of the running-point search (Sec. 5.1) as lattice windows."""
from __future__ import annotations

import numpy as np


def front_zones(ball, p, h: float = 0.1):
    """Four zones of the front field that move with the ball (Sec. 5.1), as
    windows of the h lattice.  Reading (the zone figures are not available):
    x from clamp(ball_x - 1, -2, 3) to goal_x - 0.5 m, split in two halves
    (I/II behind, III/IV in front), each split at y = 0, y within 0.3 m of
    the touch lines; the more aggressive zones III and IV come last."""
    hx, hy = 0.5 * p.field_len, 0.5 * p.field_wid
    nx_all, ny_all = int(round(p.field_len / h)) + 1, int(round(p.field_wid / h)) + 1
    xa = min(max(float(ball[0]) - 1.0, -2.0), 3.0)
    xb = p.goal_x - 0.5
    xm = 0.5 * (xa + xb)
    ya, yb = -hy + 0.3, hy - 0.3

    def I(x):
        return int(round((x + hx) / h))

    def J(y):
        return int(round((y + hy) / h))

    assert I(xb) < nx_all and J(yb) < ny_all
    out = []
    for x0, x1 in ((xa, xm), (xm, xb)):
        for y0, y1 in ((ya, 0.0), (0.0, yb)):
            i0, i1, j0, j1 = I(x0), I(x1), J(y0), J(y1)
            out.append((np.float32(h), i0, j0, i1 - i0 + 1, j1 - j0 + 1))
    return out
