"""Work model of the search: pass evaluations and FP32 VALU flops.

One *pass evaluation* is one (candidate point, pass variant) judged against
every interceptor at all K path samples.

Flops count the operations of the factored search as the kernel performs them,
per lane: an FMA is 2, every other VALU operation (add, multiply, min/max,
compare, select, square root, reciprocal) is 1.  The counts are read off the
formulation, not measured:

* robot stage, per (interceptor, sample): 26 operations of which 5 are FMAs
  -> 31 flops (offset 2, squared distance 2, clamp 1, rsq 1, distance to reach
  2, speed along the line 4, clamp 1, stopping distances 3, overshoot test and
  selects 4, sqrt 1, peak speed 1, cruise 2, total 2, team minimum 1);
* per sample, independent of speed: 7 (sample position and distance) + 2
  (time rescale) flops;
* critical kick speed, per (sample, side, kick type present): 27 operations of
  which 3 are FMAs -> 30 flops; chips add 2 per sample (airborne limit) and 1
  per side;
* first crossing, per (variant, sample): one compare per side -> 2;
* per (point, variant) finish: 40 flops (two ball times at the crossing,
  margin, feasibility, score);
* per point: 40 flops of set-up plus the open goal angle (60 + 12 per
  opponent).
"""
from __future__ import annotations

C_ROBOT = 31
C_SAMPLE = 9
C_VCRIT = 30
C_CHIP_SAMPLE = 4
C_CROSS = 2
C_FINISH = 40
C_POINT = 40
C_ANGLE = 60
C_ANGLE_OPP = 12


def point_flops(n_int: int, n_opp: int, K: int, n_flat: int, n_chip: int) -> int:
    """Flops for one candidate point: n_int interceptors (teammates other than
    the passer plus opponents), K samples, n_flat + n_chip variants."""
    types = (n_flat > 0) + (n_chip > 0)
    per_sample = C_SAMPLE + 2 * C_VCRIT * types + (C_CHIP_SAMPLE if n_chip else 0)
    V = n_flat + n_chip
    return (n_int * K * C_ROBOT + K * per_sample + V * K * C_CROSS + V * C_FINISH
            + C_POINT + C_ANGLE + C_ANGLE_OPP * n_opp)


def frame_work(frame, K: int) -> tuple[int, int]:
    """(pass evaluations, flops) of one frame."""
    n_int = frame.n_team - 1 + frame.n_opp
    n_flat = sum(1 for v in frame.variants if v[0] == 0)
    n_chip = len(frame.variants) - n_flat
    pts = frame.n_points()
    return pts * len(frame.variants), pts * point_flops(n_int, frame.n_opp, K, n_flat, n_chip)


def batch_work(frames, K: int) -> tuple[int, int]:
    ev = fl = 0
    for f in frames:
        e, x = frame_work(f, K)
        ev += e
        fl += x
    return ev, fl


# The direction x power search (the paper's own form): per direction the same
# robot stage, critical speeds and crossings as a candidate point (the ray
# plays the part of the path), a direction set-up (ray length and path frame:
# C_RAY_DIR), a per-variant finish that also forms the passing point and the
# refraction angle (C_RAY_FINISH), and one open goal angle per feasible
# passing point.
C_RAY_DIR = 60
C_RAY_FINISH = 70


def ray_frame_work(frame, K: int, n_dirs: int, n_feasible: int) -> tuple[int, int]:
    """(pass evaluations, flops) of one frame of the direction x variant
    search, given how many of its passes came out feasible."""
    n_int = frame.n_team - 1 + frame.n_opp
    n_flat = sum(1 for v in frame.variants if v[0] == 0)
    n_chip = len(frame.variants) - n_flat
    V = n_flat + n_chip
    types = (n_flat > 0) + (n_chip > 0)
    per_sample = C_SAMPLE + 2 * C_VCRIT * types + (C_CHIP_SAMPLE if n_chip else 0)
    per_dir = (n_int * K * C_ROBOT + K * per_sample + V * K * C_CROSS + V * C_RAY_FINISH
               + C_RAY_DIR)
    return n_dirs * V, n_dirs * per_dir + n_feasible * (C_ANGLE + C_ANGLE_OPP * frame.n_opp)


# MI355X peaks used for the roofline (256 CUs, 2.4 GHz)
PEAK_FP32_VECTOR_TFLOPS = 157.3   # published; assumes packed FP32 FMA every cycle
PEAK_FP32_NONPACKED_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
PEAK_HBM_GBS = 8000.0


# The shooting decision (Sec. 4.4), per shooter position: the widest-gap
# geometry (the open goal angle's terms plus C_SHOT_GAP per opponent for the
# gap scan), the aim, the shot's path frame and the ball time to the goal line
# (C_SHOT_SET), per sample its position, the float32 ball time and the slack
# (C_SHOT_SAMPLE), and the opponents' robot stage (C_ROBOT per opponent and
# sample).
C_SHOT_SET = 120
C_SHOT_GAP = 8
C_SHOT_SAMPLE = 26


def shot_flops(n_opp: int, K: int) -> int:
    """Flops of one shooting decision against n_opp opponents, K samples."""
    return (n_opp * K * C_ROBOT + K * C_SHOT_SAMPLE + C_SHOT_SET + C_ANGLE
            + (C_ANGLE_OPP + C_SHOT_GAP) * n_opp)


# Running points (Sec. 5.2), per zone point: the defense-area test, the goal
# distance, bearing and angle window, the ball distance, the two entry points
# P and Q (C_RUN_POINT), then per opponent two robot arrival times and the
# marking weight (C_RUN_OPP).
C_RUN_POINT = 90
C_RUN_OPP = 2 * C_ROBOT + 12


def run_flops(n_opp: int) -> int:
    """Flops of one running-point evaluation against n_opp opponents."""
    return C_RUN_POINT + C_RUN_OPP * n_opp


def tflops(flop: float, ms: float) -> float:
    """TFLOP/s of `flop` operations in `ms` milliseconds."""
    return flop / (ms * 1e-3) / 1e12
