"""ctypes front end of the FP64 oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline leg of the benchmark are its only users.  It imports nothing from the
product package; frames and parameters are read by attribute (any object with
``team``, ``opp``, ``passer``, ``ball``, ``windows``, ``variants`` works).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
DEFAULT_LIB = os.path.join(HERE, "liboracle.so")
# ORACLE_LIB selects another build (e.g. one with sanitizers), loaded as is
LIB = os.environ.get("ORACLE_LIB") or DEFAULT_LIB

AMB_REACH, AMB_LAND, AMB_CROSS, AMB_MARGIN, AMB_ANGLE, AMB_RUN = 1, 2, 4, 8, 16, 32


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(DEFAULT_LIB) or os.path.getmtime(DEFAULT_LIB) < os.path.getmtime(SRC):
        tmp = DEFAULT_LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC",
                               "-shared", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, DEFAULT_LIB)
    return DEFAULT_LIB


class OrcParams(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "field_len", "field_wid", "goal_x", "goal_width", "robot_radius", "vmax", "amax",
        "slide_decel", "roll_decel", "slide_ratio", "chip_angle", "gravity", "margin_s",
        "margin_cap_s", "w_angle", "w_dist", "w_margin", "dist_norm", "goal_eps")] + [
        ("n_samples", C.c_int32), ("n_threads", C.c_int32)] + [
        (n, C.c_double) for n in ("eps_reach", "eps_land", "eps_cross_t", "eps_cross_s",
                                  "eps_margin")]


class OrcWorld(C.Structure):
    _fields_ = [("n_team", C.c_int32), ("n_opp", C.c_int32), ("passer", C.c_int32),
                ("pad", C.c_int32), ("team", C.POINTER(C.c_double)),
                ("opp", C.POINTER(C.c_double)), ("ball_x", C.c_double), ("ball_y", C.c_double)]


class OrcResult(C.Structure):
    _fields_ = [("reachable", C.c_int32), ("feasible", C.c_int32), ("ambig", C.c_int32),
                ("pad", C.c_int32), ("t_team", C.c_double), ("t_opp", C.c_double),
                ("margin", C.c_double), ("score", C.c_double), ("open_angle", C.c_double)]


class OrcRayParams(C.Structure):
    _fields_ = [("n_dirs", C.c_int32), ("pad", C.c_int32), ("w_time", C.c_double),
                ("w_refract", C.c_double)]


class OrcRayResult(C.Structure):
    _fields_ = [("feasible", C.c_int32), ("k_team", C.c_int32), ("k_opp", C.c_int32),
                ("ambig", C.c_int32)] + [(n, C.c_double) for n in (
                    "t_team", "t_opp", "margin", "score", "s_recv", "x", "y", "open_angle",
                    "refract", "length")]


class OrcShotParams(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("v_shot", "min_angle", "margin_s", "eps_angle",
                                           "eps_aim")]


class OrcShotResult(C.Structure):
    _fields_ = [("shoot", C.c_int32), ("reachable", C.c_int32), ("ambig", C.c_int32),
                ("n_gaps", C.c_int32)] + [(n, C.c_double) for n in (
                    "aim", "gap", "open_angle", "length", "t_goal", "slack", "slack_sens",
                    "second_gap", "length_sens")]


class OrcRunParams(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "w_goal", "w_ball", "w_angle", "w_guard", "w_defense", "ball_norm", "ang_lo", "ang_hi",
        "ang_fall", "guard_norm", "def_depth", "def_width", "mark_radius")]


class OrcRunResult(C.Structure):
    _fields_ = [("valid", C.c_int32), ("ambig", C.c_int32)] + [(n, C.c_double) for n in (
        "score", "goal", "ball", "angle", "guard", "defense", "px", "py", "qx", "qy", "t_p",
        "t_q")]


# Parity bands (widths of the ambiguity regions computed by the oracle).  The
# crossing band (time and ball position) is four times the largest FP32 error
# measured on the GPU's first-crossing decisions (5e-7 over the 20 cm frames
# of seeds 0-999, the 5 cm frames of seeds 0-7 and 32 frames of the batched
# workload); the margin band is the stated flag tolerance.
DEFAULT_BANDS = dict(eps_reach=1e-4, eps_land=1e-5, eps_cross_t=2e-6, eps_cross_s=2e-6,
                     eps_margin=1e-3)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.environ.get("ORACLE_LIB") and (
                not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC)):
            build(force=True)
        L = C.CDLL(LIB)
        d, i32, i64 = C.c_double, C.c_int32, C.c_int64
        P, Wp = C.POINTER(OrcParams), C.POINTER(OrcWorld)
        pd, pu8, pi32 = C.POINTER(C.c_double), C.POINTER(C.c_uint8), C.POINTER(C.c_int32)
        L.orc_ball_range.argtypes = [P, C.c_int, d, pd, pd]
        L.orc_ball_time.argtypes = [P, C.c_int, d, d]
        L.orc_ball_time.restype = d
        L.orc_ball_dist.argtypes = [P, C.c_int, d, d]
        L.orc_ball_dist.restype = d
        L.orc_robot_time.argtypes = [P, d, d]
        L.orc_robot_time.restype = d
        L.orc_robot_time_to.argtypes = [P, d, d, d, d, d, d]
        L.orc_robot_time_to.restype = d
        L.orc_sbip_robot.argtypes = [P, d, d, d, d, C.c_int, d, d, d, d, d, C.POINTER(C.c_int)]
        L.orc_sbip_robot.restype = d
        L.orc_open_angle.argtypes = [P, d, d, C.c_int, pd]
        L.orc_open_angle.restype = d
        L.orc_eval.argtypes = [P, Wp, C.c_int, d, d, d, C.c_int, C.POINTER(OrcResult)]
        L.orc_point.argtypes = [P, d, C.c_int, C.c_int, pd, pd]
        L.orc_search.argtypes = [P, Wp, C.c_int, pd, pi32, C.c_int, pi32, pd, C.c_int,
                                 pu8, pd, pd, pd, pd, pu8]
        L.orc_search.restype = i64
        L.orc_search_points.argtypes = [P, Wp, i64, pd, C.c_int, pi32, pd, C.c_int,
                                        pu8, pd, pd, pd, pd, pu8]
        L.orc_argmax.argtypes = [i64, pd]
        L.orc_argmax.restype = i64
        RP = C.POINTER(OrcRayParams)
        L.orc_ray_length.argtypes = [P, d, d, d, d]
        L.orc_ray_length.restype = d
        L.orc_ray_eval.argtypes = [P, RP, Wp, C.c_int, C.c_int, d, C.c_int,
                                   C.POINTER(OrcRayResult)]
        L.orc_ray_search.argtypes = [P, RP, Wp, C.c_int, pi32, pd, C.c_int, pu8, pd, pd, pd, pd,
                                     pu8]
        L.orc_ray_search.restype = i64
        L.orc_power_speed.argtypes = [P, Wp, d, d, d, d, d, pd]
        L.orc_power_speed.restype = d
        L.orc_power_search.argtypes = [P, Wp, C.c_int, pd, pi32, d, d, d, C.c_int, pu8, pd, pd,
                                       pd, pd, pu8]
        L.orc_power_search.restype = i64
        SP, SR = C.POINTER(OrcShotParams), C.POINTER(OrcShotResult)
        L.orc_shot.argtypes = [P, SP, Wp, d, d, C.c_int, SR]
        L.orc_shot_search.argtypes = [P, SP, Wp, C.c_int, pd, pi32, C.c_int, SR]
        L.orc_shot_search.restype = i64
        RPp, RR = C.POINTER(OrcRunParams), C.POINTER(OrcRunResult)
        L.orc_run.argtypes = [P, RPp, Wp, d, d, RR]
        L.orc_run_search.argtypes = [P, RPp, Wp, C.c_int, pd, pi32, RR, C.POINTER(i64)]
        L.orc_run_search.restype = i64
        _lib = L
    return _lib


def make_params(p, n_threads: int = 0, **bands) -> OrcParams:
    """Oracle parameters from any object with the Params attributes."""
    o = OrcParams()
    for name, _ in OrcParams._fields_:
        if name in ("n_threads",) or name.startswith("eps_"):
            continue
        setattr(o, name, getattr(p, name))
    o.n_threads = int(n_threads)
    b = dict(DEFAULT_BANDS)
    b.update(bands)
    for k, v in b.items():
        setattr(o, k, float(v))
    return o


class _WorldHolder:
    """Keeps the float64 robot arrays alive while the C side points into them."""

    def __init__(self, frame):
        self.team = np.ascontiguousarray(np.asarray(frame.team, dtype=np.float64).reshape(-1, 4))
        self.opp = np.ascontiguousarray(np.asarray(frame.opp, dtype=np.float64).reshape(-1, 4))
        if self.opp.size == 0:
            self.opp = np.zeros((1, 4))
        w = OrcWorld()
        w.n_team = int(np.asarray(frame.team).reshape(-1, 4).shape[0])
        w.n_opp = int(np.asarray(frame.opp).reshape(-1, 4).shape[0])
        w.passer = int(frame.passer)
        w.team = self.team.ctypes.data_as(C.POINTER(C.c_double))
        w.opp = self.opp.ctypes.data_as(C.POINTER(C.c_double))
        w.ball_x = float(frame.ball[0])
        w.ball_y = float(frame.ball[1])
        self.w = w


def _ptr(a, t):
    return None if a is None else a.ctypes.data_as(C.POINTER(t))


def search_frame(frame, params, bands: bool = False, n_threads: int = 0, **band_eps):
    """Run the oracle on every (window, variant, point) of a frame.

    Returns a dict of flat arrays in output order (window-major, then variant,
    then row-major [ny][nx]) plus ``best`` (index or -1) and ``best_score``.
    """
    L = lib()
    P = make_params(params, n_threads, **band_eps)
    wh = _WorldHolder(frame)
    win_h = np.array([w[0] for w in frame.windows], dtype=np.float64)
    win_i = np.array([[w[1], w[2], w[3], w[4]] for w in frame.windows], dtype=np.int32).reshape(-1)
    vt = np.array([v[0] for v in frame.variants], dtype=np.int32)
    vv = np.array([v[1] for v in frame.variants], dtype=np.float64)
    n = int(sum(w[3] * w[4] for w in frame.windows)) * len(frame.variants)
    out = dict(mask=np.zeros(n, np.uint8), score=np.zeros(n), t_team=np.zeros(n),
               t_opp=np.zeros(n), margin=np.zeros(n), ambig=np.zeros(n, np.uint8))
    L.orc_search(C.byref(P), C.byref(wh.w), len(win_h), _ptr(win_h, C.c_double),
                 _ptr(win_i, C.c_int32), len(vt), _ptr(vt, C.c_int32), _ptr(vv, C.c_double),
                 int(bands), _ptr(out["mask"], C.c_uint8), _ptr(out["score"], C.c_double),
                 _ptr(out["t_team"], C.c_double), _ptr(out["t_opp"], C.c_double),
                 _ptr(out["margin"], C.c_double), _ptr(out["ambig"], C.c_uint8))
    best = int(L.orc_argmax(n, _ptr(out["score"], C.c_double)))
    out["best"] = best
    out["best_score"] = float(out["score"][best]) if best >= 0 else float("-inf")
    return out


def search_points(frame, params, xy, bands: bool = False, n_threads: int = 0, **band_eps):
    """Oracle at explicit points ``xy`` (n, 2); outputs shaped (n, n_variants)."""
    L = lib()
    P = make_params(params, n_threads, **band_eps)
    wh = _WorldHolder(frame)
    xy = np.ascontiguousarray(np.asarray(xy, dtype=np.float64).reshape(-1, 2))
    vt = np.array([v[0] for v in frame.variants], dtype=np.int32)
    vv = np.array([v[1] for v in frame.variants], dtype=np.float64)
    n, V = xy.shape[0], len(vt)
    out = dict(mask=np.zeros((n, V), np.uint8), score=np.zeros((n, V)), t_team=np.zeros((n, V)),
               t_opp=np.zeros((n, V)), margin=np.zeros((n, V)), ambig=np.zeros((n, V), np.uint8))
    L.orc_search_points(C.byref(P), C.byref(wh.w), n, _ptr(xy, C.c_double), V,
                        _ptr(vt, C.c_int32), _ptr(vv, C.c_double), int(bands),
                        _ptr(out["mask"], C.c_uint8), _ptr(out["score"], C.c_double),
                        _ptr(out["t_team"], C.c_double), _ptr(out["t_opp"], C.c_double),
                        _ptr(out["margin"], C.c_double), _ptr(out["ambig"], C.c_uint8))
    return out


def eval_point(frame, params, vtype: int, v0: float, cx: float, cy: float, bands: bool = False):
    L = lib()
    P = make_params(params)
    wh = _WorldHolder(frame)
    r = OrcResult()
    L.orc_eval(C.byref(P), C.byref(wh.w), vtype, v0, cx, cy, int(bands), C.byref(r))
    return {k: getattr(r, k) for k, _ in OrcResult._fields_ if k != "pad"}


def points_of_window(params, win):
    """Coordinates (ny*nx, 2) of a window's points, row-major, from the oracle."""
    L = lib()
    P = make_params(params)
    h, i0, j0, nx, ny = win
    out = np.zeros((ny * nx, 2))
    x, y = C.c_double(), C.c_double()
    for j in range(ny):
        for i in range(nx):
            L.orc_point(C.byref(P), h, i0 + i, j0 + j, C.byref(x), C.byref(y))
            out[j * nx + i] = (x.value, y.value)
    return out


# scalar primitives -----------------------------------------------------------

def ball_range(params, vtype, v0):
    P = make_params(params)
    D, sf = C.c_double(), C.c_double()
    lib().orc_ball_range(C.byref(P), vtype, v0, C.byref(D), C.byref(sf))
    return D.value, sf.value


def ball_time(params, vtype, v0, s):
    return lib().orc_ball_time(C.byref(make_params(params)), vtype, v0, s)


def ball_dist(params, vtype, v0, t):
    return lib().orc_ball_dist(C.byref(make_params(params)), vtype, v0, t)


def robot_time(params, delta, u):
    return lib().orc_robot_time(C.byref(make_params(params)), delta, u)


def robot_time_to(params, robot, px, py):
    x, y, vx, vy = [float(a) for a in robot]
    return lib().orc_robot_time_to(C.byref(make_params(params)), x, y, vx, vy, px, py)


def sbip_robot(params, ball, c, vtype, v0, robot):
    k = C.c_int()
    x, y, vx, vy = [float(a) for a in robot]
    t = lib().orc_sbip_robot(C.byref(make_params(params)), float(ball[0]), float(ball[1]),
                             float(c[0]), float(c[1]), vtype, v0, x, y, vx, vy, C.byref(k))
    return t, k.value


def open_angle(params, cx, cy, opp):
    o = np.ascontiguousarray(np.asarray(opp, dtype=np.float64).reshape(-1, 4))
    n = o.shape[0]
    if n == 0:
        o = np.zeros((1, 4))
    return lib().orc_open_angle(C.byref(make_params(params)), cx, cy, n, _ptr(o, C.c_double))


# ---------------------------------------------------------------------------
# the paper's own DPPS form: every kick direction x every kick power
# ---------------------------------------------------------------------------

def _ray_params(n_dirs: int, w_time: float, w_refract: float) -> OrcRayParams:
    r = OrcRayParams()
    r.n_dirs, r.w_time, r.w_refract = int(n_dirs), float(w_time), float(w_refract)
    return r


def ray_length(params, bx, by, ux, uy) -> float:
    return float(lib().orc_ray_length(C.byref(make_params(params)), bx, by, ux, uy))


def ray_search(frame, params, n_dirs: int, w_time: float, w_refract: float,
               bands: bool = False, n_threads: int = 0, **band_eps):
    """Every (direction, variant) of a frame; arrays shaped (n_dirs, n_variants),
    plus ``best`` (flat index dir * V + v, or -1) and ``best_score``."""
    L = lib()
    P = make_params(params, n_threads, **band_eps)
    R = _ray_params(n_dirs, w_time, w_refract)
    wh = _WorldHolder(frame)
    vt = np.array([v[0] for v in frame.variants], dtype=np.int32)
    vv = np.array([v[1] for v in frame.variants], dtype=np.float64)
    V = len(vt)
    out = dict(mask=np.zeros((n_dirs, V), np.uint8), score=np.zeros((n_dirs, V)),
               t_team=np.zeros((n_dirs, V)), t_opp=np.zeros((n_dirs, V)),
               s_recv=np.zeros((n_dirs, V)), ambig=np.zeros((n_dirs, V), np.uint8))
    L.orc_ray_search(C.byref(P), C.byref(R), C.byref(wh.w), V, _ptr(vt, C.c_int32),
                     _ptr(vv, C.c_double), int(bands), _ptr(out["mask"], C.c_uint8),
                     _ptr(out["score"], C.c_double), _ptr(out["t_team"], C.c_double),
                     _ptr(out["t_opp"], C.c_double), _ptr(out["s_recv"], C.c_double),
                     _ptr(out["ambig"], C.c_uint8))
    flat = np.ascontiguousarray(out["score"].reshape(-1))
    best = int(L.orc_argmax(flat.size, _ptr(flat, C.c_double)))
    out["best"] = best
    out["best_score"] = float(flat[best]) if best >= 0 else float("-inf")
    return out


def ray_eval(frame, params, n_dirs: int, w_time: float, w_refract: float, direction: int,
             vtype: int, v0: float, bands: bool = False, **band_eps):
    """One (direction, variant): every field of the oracle's result."""
    L = lib()
    P = make_params(params, **band_eps)
    R = _ray_params(n_dirs, w_time, w_refract)
    wh = _WorldHolder(frame)
    r = OrcRayResult()
    L.orc_ray_eval(C.byref(P), C.byref(R), C.byref(wh.w), direction, vtype, v0, int(bands),
                   C.byref(r))
    return {k: getattr(r, k) for k, _ in OrcRayResult._fields_}


# ---------------------------------------------------------------------------
# passing power per point (Sec. 4.1, Eq. 1-2)
# ---------------------------------------------------------------------------

def power_speed(frame, params, cx, cy, buffer_s=0.3, v_min=1.0, v_max=6.5):
    """(kick speed, receiver arrival time) for a pass to (cx, cy)."""
    L = lib()
    P = make_params(params)
    wh = _WorldHolder(frame)
    t = C.c_double()
    v = L.orc_power_speed(C.byref(P), C.byref(wh.w), cx, cy, buffer_s, v_min, v_max,
                          C.byref(t))
    return float(v), float(t.value)


def power_search(frame, params, buffer_s=0.3, v_min=1.0, v_max=6.5, bands=False,
                 n_threads: int = 0, **band_eps):
    """Every point of the frame's windows with one flat pass at the point's
    own power; flat arrays in window-major, row-major order."""
    L = lib()
    P = make_params(params, n_threads, **band_eps)
    wh = _WorldHolder(frame)
    win_h = np.array([w[0] for w in frame.windows], dtype=np.float64)
    win_i = np.array([[w[1], w[2], w[3], w[4]] for w in frame.windows], dtype=np.int32).reshape(-1)
    n = int(sum(w[3] * w[4] for w in frame.windows))
    out = dict(mask=np.zeros(n, np.uint8), score=np.zeros(n), t_team=np.zeros(n),
               t_opp=np.zeros(n), v0=np.zeros(n), ambig=np.zeros(n, np.uint8))
    L.orc_power_search(C.byref(P), C.byref(wh.w), len(win_h), _ptr(win_h, C.c_double),
                       _ptr(win_i, C.c_int32), buffer_s, v_min, v_max, int(bands),
                       _ptr(out["mask"], C.c_uint8), _ptr(out["score"], C.c_double),
                       _ptr(out["t_team"], C.c_double), _ptr(out["t_opp"], C.c_double),
                       _ptr(out["v0"], C.c_double), _ptr(out["ambig"], C.c_uint8))
    best = int(L.orc_argmax(n, _ptr(out["score"], C.c_double)))
    out["best"] = best
    out["best_score"] = float(out["score"][best]) if best >= 0 else float("-inf")
    return out


# ---------------------------------------------------------------------------
# shooting decision (Sec. 4.4)
# ---------------------------------------------------------------------------

SHOT_FIELDS = [k for k, _ in OrcShotResult._fields_]


def _shot_params(v_shot, min_angle, margin_s, eps_angle=1e-5, eps_aim=2e-6):
    s = OrcShotParams()
    s.v_shot, s.min_angle, s.margin_s = float(v_shot), float(min_angle), float(margin_s)
    s.eps_angle, s.eps_aim = float(eps_angle), float(eps_aim)
    return s


def shot(frame, params, cx=None, cy=None, v_shot=6.5, min_angle=0.05, margin_s=0.0,
         bands=False, **band_eps):
    """Shooting decision from (cx, cy), by default from the frame's ball:
    a dict of the oracle's result fields."""
    L = lib()
    P = make_params(params, **band_eps)
    wh = _WorldHolder(frame)
    cx = float(frame.ball[0]) if cx is None else float(cx)
    cy = float(frame.ball[1]) if cy is None else float(cy)
    r = OrcShotResult()
    L.orc_shot(C.byref(P), C.byref(_shot_params(v_shot, min_angle, margin_s)), C.byref(wh.w),
               cx, cy, int(bands), C.byref(r))
    return {k: getattr(r, k) for k in SHOT_FIELDS}


def shot_search(frame, params, v_shot=6.5, min_angle=0.05, margin_s=0.0, bands=False,
                n_threads: int = 0, **band_eps):
    """The shooting decision from every point of the frame's windows (the ball
    placed there); a dict of flat arrays in window-major, row-major order."""
    L = lib()
    P = make_params(params, n_threads, **band_eps)
    wh = _WorldHolder(frame)
    win_h = np.array([w[0] for w in frame.windows], dtype=np.float64)
    win_i = np.array([[w[1], w[2], w[3], w[4]] for w in frame.windows], dtype=np.int32).reshape(-1)
    n = int(sum(w[3] * w[4] for w in frame.windows))
    res = (OrcShotResult * max(n, 1))()
    L.orc_shot_search(C.byref(P), C.byref(_shot_params(v_shot, min_angle, margin_s)),
                      C.byref(wh.w), len(win_h), _ptr(win_h, C.c_double),
                      _ptr(win_i, C.c_int32), int(bands), res)
    a = np.ctypeslib.as_array(res)[:n]
    return {k: np.array(a[k]) for k in SHOT_FIELDS}


# ---------------------------------------------------------------------------
# running points (Sec. 5.2)
# ---------------------------------------------------------------------------

RUN_FIELDS = [k for k, _ in OrcRunResult._fields_]
RUN_DEFAULTS = dict(w_goal=0.3, w_ball=0.1, w_angle=0.15, w_guard=0.25, w_defense=0.2,
                    ball_norm=2.0, ang_lo=0.2617993877991494, ang_hi=0.7853981633974483,
                    ang_fall=0.5235987755982988, guard_norm=2.0, def_depth=1.2, def_width=2.4,
                    mark_radius=1.0)


def _run_params(**kw):
    r = OrcRunParams()
    v = dict(RUN_DEFAULTS)
    v.update(kw)
    for k, x in v.items():
        setattr(r, k, float(x))
    return r


def run_point(frame, params, cx, cy, **run):
    """The five criteria and the score at (cx, cy)."""
    r = OrcRunResult()
    wh = _WorldHolder(frame)
    lib().orc_run(C.byref(make_params(params)), C.byref(_run_params(**run)), C.byref(wh.w),
                  float(cx), float(cy), C.byref(r))
    return {k: getattr(r, k) for k in RUN_FIELDS}


def run_search(frame, params, n_threads: int = 0, **run):
    """Every point of the frame's windows (the zones): a dict of flat arrays
    in window-major, row-major order, plus ``best`` (per window, the index
    within the window, or -1)."""
    L = lib()
    P = make_params(params, n_threads)
    wh = _WorldHolder(frame)
    win_h = np.array([w[0] for w in frame.windows], dtype=np.float64)
    win_i = np.array([[w[1], w[2], w[3], w[4]] for w in frame.windows], dtype=np.int32).reshape(-1)
    n = int(sum(w[3] * w[4] for w in frame.windows))
    res = (OrcRunResult * max(n, 1))()
    best = np.zeros(max(len(win_h), 1), np.int64)
    L.orc_run_search(C.byref(P), C.byref(_run_params(**run)), C.byref(wh.w), len(win_h),
                     _ptr(win_h, C.c_double), _ptr(win_i, C.c_int32), res,
                     best.ctypes.data_as(C.POINTER(C.c_int64)))
    a = np.ctypeslib.as_array(res)[:n]
    out = {k: np.array(a[k]) for k in RUN_FIELDS}
    out["best"] = best[:len(win_h)]
    return out
