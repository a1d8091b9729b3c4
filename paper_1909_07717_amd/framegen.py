"""Seeded synthetic frames shaped like RoboCup SSL play.

This module is shared by the HIP path, the oracle-based tests and the
benchmark.  It draws inputs only: robot states, the passer, candidate windows
and pass variants.  It holds none of the search's arithmetic (no ball model,
no robot motion model, no lattice coordinates, no scoring).

Recipe (one ``numpy.random.Generator(PCG64(seed))`` per frame unless stated):

1. (variable-size configs only) team and opponent counts;
2. team positions, uniform on [-L/2, L/2] x [-W/2, W/2] (12 m x 9 m field);
3. team velocities, uniform in a disc of radius 1.5 m/s
   (speed = 1.5 sqrt(U), heading = 2 pi U);
4. opponent positions, then opponent velocities, drawn the same way;
5. the passer index, uniform over the team; the ball sits on the passer;
6. (variable-window configs only) the window width/height and its origin.

All values are rounded to float32 once here; the oracle receives exactly these
float32 values widened to float64, so both sides see identical inputs.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
import math

import numpy as np

FLAT = 0
CHIP = 1


@dataclass(frozen=True)
class Params:
    """Field geometry, motion limits, ball model and scoring constants.

    Defaults are the configuration values of the full-frame workloads: a
    12 m x 9 m field with a 1.2 m goal at x = +6 m, robots of radius 0.09 m
    with top speed 3.25 m/s (the paper's robot, Sec. 2.1) and acceleration
    3 m/s^2, a two-phase ball that slides at 5 m/s^2 down to 5/7 of the kick
    speed (Sec. 4.1) and then rolls at 0.5 m/s^2, 45-degree chips, a 0.1 s
    feasibility margin and the score weights 0.5 / 0.3 / 0.2.
    """

    field_len: float = 12.0
    field_wid: float = 9.0
    goal_x: float = 6.0
    goal_width: float = 1.2
    robot_radius: float = 0.09
    vmax: float = 3.25
    amax: float = 3.0
    slide_decel: float = 5.0
    roll_decel: float = 0.5
    slide_ratio: float = 5.0 / 7.0
    chip_angle: float = math.pi / 4
    gravity: float = 9.81
    n_samples: int = 64
    margin_s: float = 0.1
    margin_cap_s: float = 1.0
    w_angle: float = 0.5
    w_dist: float = 0.3
    w_margin: float = 0.2
    dist_norm: float = 15.0
    goal_eps: float = 1e-3

    def as_f32(self) -> "Params":
        """The same constants rounded to float32 (what the GPU library sees)."""
        kw = {}
        for k, v in self.__dict__.items():
            kw[k] = v if isinstance(v, int) else float(np.float32(v))
        return Params(**kw)


@dataclass
class Frame:
    """One world state plus the candidate windows and pass variants to search.

    ``team`` and ``opp`` are float32 arrays of shape (n, 4) holding
    (x, y, vx, vy).  ``windows`` is a list of (h, i0, j0, nx, ny) sub-rectangles
    of the field-centred lattice of spacing h.  ``variants`` is a list of
    (type, v0) with type FLAT or CHIP and v0 the kick speed in m/s; variants are
    ordered flat speeds ascending, then chip speeds ascending.
    """

    team: np.ndarray
    opp: np.ndarray
    passer: int
    ball: np.ndarray
    windows: list = field(default_factory=list)
    variants: list = field(default_factory=list)

    @property
    def n_team(self) -> int:
        return int(self.team.shape[0])

    @property
    def n_opp(self) -> int:
        return int(self.opp.shape[0])

    def n_points(self) -> int:
        return int(sum(w[3] * w[4] for w in self.windows))

    def n_evals(self) -> int:
        return self.n_points() * len(self.variants)

    def copy(self) -> "Frame":
        return Frame(self.team.copy(), self.opp.copy(), int(self.passer), self.ball.copy(),
                     list(self.windows), list(self.variants))


def lattice_dims(h: float, params: Params = Params()) -> tuple[int, int]:
    """Point counts of the full field lattice at spacing h (endpoints included).

    The spacing must divide both field dimensions (to within 1e-3 of a whole
    number of steps), e.g. 0.05, 0.1, 0.2, 0.25, 0.3 or 0.5 m on a 12 m x 9 m
    field.
    """
    h = float(np.float32(h))
    qx, qy = params.field_len / h, params.field_wid / h
    if abs(qx - round(qx)) > 1e-3 or abs(qy - round(qy)) > 1e-3:
        raise ValueError(f"lattice spacing {h} does not divide the field")
    return int(round(qx)) + 1, int(round(qy)) + 1


def full_window(h: float, params: Params = Params()):
    """The window covering the whole field lattice at spacing h."""
    nx, ny = lattice_dims(h, params)
    return (float(np.float32(h)), 0, 0, nx, ny)


def speeds_linear(n: int, lo: float = 1.0, hi: float = 6.5) -> list[float]:
    """n kick speeds spaced linearly over [lo, hi], both ends included."""
    if n == 1:
        return [float(np.float32(lo))]
    return [float(np.float32(v)) for v in np.linspace(lo, hi, n)]


def variants_for(speeds, flat: bool = True, chip: bool = False):
    out = []
    if flat:
        out += [(FLAT, float(np.float32(v))) for v in sorted(speeds)]
    if chip:
        out += [(CHIP, float(np.float32(v))) for v in sorted(speeds)]
    return out


def _draw_team(rng: np.random.Generator, n: int, params: Params) -> np.ndarray:
    hl, hw = params.field_len / 2, params.field_wid / 2
    pos = np.stack([rng.uniform(-hl, hl, n), rng.uniform(-hw, hw, n)], axis=1)
    return pos


def _draw_vel(rng: np.random.Generator, n: int, vdisc: float) -> np.ndarray:
    sp = vdisc * np.sqrt(rng.uniform(0.0, 1.0, n))
    hd = 2.0 * np.pi * rng.uniform(0.0, 1.0, n)
    return np.stack([sp * np.cos(hd), sp * np.sin(hd)], axis=1)


def random_frame(rng: np.random.Generator, n_team: int, n_opp: int,
                 params: Params = Params(), vdisc: float = 1.5) -> Frame:
    """Draw robots, velocities and the passer in the documented order."""
    tp = _draw_team(rng, n_team, params)
    tv = _draw_vel(rng, n_team, vdisc)
    op = _draw_team(rng, n_opp, params)
    ov = _draw_vel(rng, n_opp, vdisc)
    passer = int(rng.integers(0, n_team))
    team = np.concatenate([tp, tv], axis=1).astype(np.float32).reshape(n_team, 4)
    opp = np.concatenate([op, ov], axis=1).astype(np.float32).reshape(n_opp, 4)
    ball = team[passer, :2].copy()
    return Frame(team, opp, passer, ball)


# ---------------------------------------------------------------------------
# The workloads.  Each returns fully specified frames (windows + variants).
# ---------------------------------------------------------------------------

def config_small(seed: int) -> Frame:
    """6v6, 20 cm full lattice (61 x 46 = 2806 points), one flat pass at 4 m/s.

    Use with ``Params(n_samples=64)``.
    """
    f = random_frame(np.random.default_rng(seed), 6, 6)
    f.windows = [full_window(0.2)]
    f.variants = variants_for([4.0], flat=True, chip=False)
    return f


def config_full(seed: int) -> Frame:
    """8v8, 5 cm full lattice (241 x 181 = 43621 points), 16 speeds in
    [1, 6.5] m/s, flat and chip (32 variants).  Use with ``Params(n_samples=256)``.
    """
    f = random_frame(np.random.default_rng(seed), 8, 8)
    f.windows = [full_window(0.05)]
    f.variants = variants_for(speeds_linear(16), flat=True, chip=True)
    return f


def random_window(rng: np.random.Generator, h: float = 0.05, params: Params = Params()):
    """A random rectangle 1-12 m x 1-9 m on the lattice of spacing h."""
    NX, NY = lattice_dims(h, params)
    w = rng.uniform(1.0, params.field_len)
    g = rng.uniform(1.0, params.field_wid)
    nx = min(int(round(w / h)) + 1, NX)
    ny = min(int(round(g / h)) + 1, NY)
    i0 = int(rng.integers(0, NX - nx + 1))
    j0 = int(rng.integers(0, NY - ny + 1))
    return (float(np.float32(h)), i0, j0, nx, ny)


def config_batch_frame(rng: np.random.Generator, n_speeds: int = 8, h: float = 0.05) -> Frame:
    """One frame of the batched workload: 6-8 robots a side, a random window,
    ``n_speeds`` flat speeds in [1, 6.5] m/s.  Use with ``Params(n_samples=128)``."""
    n_team = int(rng.integers(6, 9))
    n_opp = int(rng.integers(6, 9))
    f = random_frame(rng, n_team, n_opp)
    f.windows = [random_window(rng, h)]
    f.variants = variants_for(speeds_linear(n_speeds), flat=True, chip=False)
    return f


def config_batch(seed: int, n_frames: int = 4096, n_speeds: int = 8) -> list[Frame]:
    """The batched workload: ``n_frames`` independent frames from one seed."""
    rng = np.random.default_rng(seed)
    return [config_batch_frame(rng, n_speeds) for _ in range(n_frames)]


def uniform_batch_arrays(seed: int, n: int, n_team: int = 6, n_opp: int = 6,
                         params: Params = Params(), vdisc: float = 1.5):
    """n frames of one size drawn at once (for training streams): returns
    (team [n, n_team, 4], opp [n, n_opp, 4], passer [n]) as float32 / int32.
    Same distributions as random_frame; draw order: team positions, team
    velocities, opponent positions, opponent velocities, passers."""
    rng = np.random.default_rng(seed)
    hl, hw = params.field_len / 2, params.field_wid / 2

    def pos(m):
        return np.stack([rng.uniform(-hl, hl, (n, m)), rng.uniform(-hw, hw, (n, m))], -1)

    def vel(m):
        sp = vdisc * np.sqrt(rng.uniform(0.0, 1.0, (n, m)))
        hd = 2.0 * np.pi * rng.uniform(0.0, 1.0, (n, m))
        return np.stack([sp * np.cos(hd), sp * np.sin(hd)], -1)

    tp, tv = pos(n_team), vel(n_team)
    op, ov = pos(n_opp), vel(n_opp)
    passer = rng.integers(0, n_team, n).astype(np.int32)
    team = np.concatenate([tp, tv], -1).astype(np.float32)
    opp = np.concatenate([op, ov], -1).astype(np.float32)
    return team, opp, passer


def frames_from_arrays(team, opp, passer, windows, variants) -> list:
    """Frame objects (ball on the passer) from uniform_batch_arrays output."""
    out = []
    for i in range(team.shape[0]):
        t = team[i].copy()
        out.append(Frame(t, opp[i].copy(), int(passer[i]), t[int(passer[i]), :2].copy(),
                         list(windows), list(variants)))
    return out


def with_windows(f: Frame, windows) -> Frame:
    g = f.copy()
    g.windows = list(windows)
    return g


def with_variants(f: Frame, variants) -> Frame:
    g = f.copy()
    g.variants = list(variants)
    return g


__all__ = [
    "FLAT", "CHIP", "Params", "Frame", "lattice_dims", "full_window", "speeds_linear",
    "variants_for", "random_frame", "config_small", "config_full", "random_window",
    "config_batch_frame", "config_batch", "with_windows", "with_variants", "replace",
]
