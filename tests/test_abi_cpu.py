"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, and the binding's struct layouts match the header's (checked
by compiling a probe against include/dpps.h with gcc).  No GPU calls."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1909_07717_amd import binding as B
from paper_1909_07717_amd.framegen import Params, config_small, config_full, full_window

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "dpps.h")


def _declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dpps_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    L = B.lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n


def test_binding_argtypes_cover_every_declared_function():
    L = B.lib()
    for n in _declared():
        assert getattr(L, n).argtypes is not None, n


PROBE = r"""
#include <stddef.h>
#include <stdio.h>
#include "dpps.h"
#define S(t) printf(#t " %zu\n", sizeof(t))
#define O(t, f) printf(#t "." #f " %zu\n", offsetof(t, f))
int main(void) {
  S(dpps_robot); S(dpps_window); S(dpps_variant); S(dpps_frame); S(dpps_params);
  S(dpps_best); S(dpps_outputs);
  O(dpps_frame, out_off); O(dpps_frame, ball_x); O(dpps_frame, ball_y);
  O(dpps_params, n_samples); O(dpps_params, out_flags); O(dpps_params, hbm_budget_bytes);
  O(dpps_best, score); O(dpps_best, t_ball); O(dpps_outputs, best);
  S(dpps_ray_params); S(dpps_ray_best); S(dpps_ray_outputs);
  O(dpps_ray_params, w_refract); O(dpps_ray_best, theta); O(dpps_ray_best, score);
  O(dpps_ray_best, refract); O(dpps_ray_outputs, s_recv); O(dpps_ray_outputs, best);
  S(dpps_power_params); O(dpps_power_params, v_max);
  S(dpps_shot_params); S(dpps_shot); O(dpps_shot_params, margin_s); O(dpps_shot, aim);
  O(dpps_shot, t_goal); O(dpps_shot, slack);
  S(dpps_run_params); S(dpps_run_best); O(dpps_run_params, mark_radius);
  O(dpps_run_params, reserved); O(dpps_run_best, score); O(dpps_run_best, defense);
  return 0;
}
"""


def test_struct_layouts_match_header(tmp_path):
    c = tmp_path / "probe.c"
    c.write_text(PROBE)
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-std=c11", f"-I{os.path.dirname(HDR)}", "-o", str(exe), str(c)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)], text=True).splitlines())
    got = {k: int(v) for k, v in got.items()}
    assert got["dpps_robot"] == B.ROBOT_DT.itemsize
    assert got["dpps_window"] == B.WINDOW_DT.itemsize
    assert got["dpps_variant"] == B.VARIANT_DT.itemsize
    assert got["dpps_frame"] == B.FRAME_DT.itemsize
    assert got["dpps_best"] == B.BEST_DT.itemsize
    assert got["dpps_params"] == C.sizeof(B.Params_C)
    assert got["dpps_outputs"] == C.sizeof(B.Outputs_C)
    assert got["dpps_frame.out_off"] == B.FRAME_DT.fields["out_off"][1]
    assert got["dpps_frame.ball_x"] == B.FRAME_DT.fields["ball_x"][1]
    assert got["dpps_params.n_samples"] == B.Params_C.n_samples.offset
    assert got["dpps_params.out_flags"] == B.Params_C.out_flags.offset
    assert got["dpps_params.hbm_budget_bytes"] == B.Params_C.hbm_budget_bytes.offset
    assert got["dpps_best.score"] == B.BEST_DT.fields["score"][1]
    assert got["dpps_best.t_ball"] == B.BEST_DT.fields["t_ball"][1]
    assert got["dpps_outputs.best"] == B.Outputs_C.best.offset
    assert got["dpps_ray_params"] == C.sizeof(B.RayParams_C)
    assert got["dpps_ray_best"] == B.RAY_BEST_DT.itemsize
    assert got["dpps_ray_outputs"] == C.sizeof(B.RayOutputs_C)
    assert got["dpps_ray_params.w_refract"] == B.RayParams_C.w_refract.offset
    for f in ("theta", "score", "refract"):
        assert got[f"dpps_ray_best.{f}"] == B.RAY_BEST_DT.fields[f][1]
    assert got["dpps_ray_outputs.s_recv"] == B.RayOutputs_C.s_recv.offset
    assert got["dpps_ray_outputs.best"] == B.RayOutputs_C.best.offset
    assert got["dpps_power_params"] == C.sizeof(B.PowerParams_C)
    assert got["dpps_power_params.v_max"] == B.PowerParams_C.v_max.offset
    assert got["dpps_shot_params"] == C.sizeof(B.ShotParams_C)
    assert got["dpps_shot_params.margin_s"] == B.ShotParams_C.margin_s.offset
    assert got["dpps_shot"] == B.SHOT_DT.itemsize
    for f in ("aim", "t_goal", "slack"):
        assert got[f"dpps_shot.{f}"] == B.SHOT_DT.fields[f][1]
    assert got["dpps_run_params"] == C.sizeof(B.RunParams_C)
    assert got["dpps_run_params.mark_radius"] == B.RunParams_C.mark_radius.offset
    assert got["dpps_run_params.reserved"] == B.RunParams_C.reserved.offset
    assert got["dpps_run_best"] == B.RUN_BEST_DT.itemsize
    for f in ("score", "defense"):
        assert got[f"dpps_run_best.{f}"] == B.RUN_BEST_DT.fields[f][1]


def test_layout_is_host_only_and_dense():
    p = Params(n_samples=64)
    pk = B.pack([config_small(0), config_full(1), config_small(2)], p)
    assert list(pk.frame_elems) == [2806, 43621 * 32, 2806]
    assert list(pk.frames["out_off"]) == [0, 2806, 2806 + 43621 * 32]
    red = B.pack([config_full(1)], p, out_flags=B.DPPS_OUT_REDUCED)
    assert red.total == 43621


def test_layout_rejects_bad_params():
    p = Params(n_samples=64)
    pc = B.params_c(p)
    pc.n_samples = 100
    total = C.c_int64()
    fr = np.zeros(1, B.FRAME_DT)
    win = np.array([full_window(0.2)], B.WINDOW_DT)
    rc = B.lib().dpps_layout(C.byref(pc), 1, fr.ctypes.data, win.ctypes.data, C.byref(total))
    assert rc == -1
    assert b"n_samples" in B.lib().dpps_last_error()
    assert B.lib().dpps_strerror(-4) == b"device memory budget exceeded"
