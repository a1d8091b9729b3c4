"""Thin ctypes binding of libdpps (include/dpps.h).

Argument marshalling only: host inputs are packed into the C structs of the
ABI, device outputs are torch tensors whose data pointers are handed to the
library, and the stream is torch's current stream unless one is given.  Every
step of the search runs in the HIP kernels; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# DPPS_LIB selects another build of the library (e.g. one with host-side
# sanitizers); there is no fallback when the file is missing
LIB_PATH = os.environ.get("DPPS_LIB") or os.path.join(HERE, "libdpps.so")

DPPS_OK = 0
DPPS_FLAT, DPPS_CHIP = 0, 1
DPPS_OUT_REDUCED = 1
MAX_SIDE, MAX_VARIANTS = 16, 64

ROBOT_DT = np.dtype([("x", "<f4"), ("y", "<f4"), ("vx", "<f4"), ("vy", "<f4")])
WINDOW_DT = np.dtype([("h", "<f4"), ("i0", "<i4"), ("j0", "<i4"), ("nx", "<i4"), ("ny", "<i4")])
VARIANT_DT = np.dtype([("type", "<i4"), ("v0", "<f4")])
FRAME_DT = np.dtype({
    "names": ["n_team", "n_opp", "passer", "robot_off", "n_windows", "window_off", "n_variants",
              "variant_off", "out_off", "ball_x", "ball_y"],
    "formats": ["<i4"] * 8 + ["<i8", "<f4", "<f4"],
    "offsets": [0, 4, 8, 12, 16, 20, 24, 28, 32, 40, 44],
    "itemsize": 48,
})
BEST_DT = np.dtype([("found", "<i4"), ("window", "<i4"), ("variant", "<i4"), ("i", "<i4"),
                    ("j", "<i4"), ("type", "<i4"), ("x", "<f4"), ("y", "<f4"), ("v0", "<f4"),
                    ("score", "<f4"), ("t_team", "<f4"), ("t_opp", "<f4"), ("t_ball", "<f4"),
                    ("pad", "<i4")])

RAY_BEST_DT = np.dtype([("found", "<i4"), ("dir", "<i4"), ("variant", "<i4"), ("type", "<i4"),
                        ("theta", "<f4"), ("v0", "<f4"), ("x", "<f4"), ("y", "<f4"),
                        ("score", "<f4"), ("t_team", "<f4"), ("t_opp", "<f4"),
                        ("open_angle", "<f4"), ("refract", "<f4"), ("pad", "<i4")])

SHOT_DT = np.dtype([("shoot", "<i4"), ("reachable", "<i4"), ("aim", "<f4"), ("gap", "<f4"),
                    ("open_angle", "<f4"), ("length", "<f4"), ("t_goal", "<f4"),
                    ("slack", "<f4")])

RUN_BEST_DT = np.dtype([("found", "<i4"), ("i", "<i4"), ("j", "<i4"), ("reserved", "<i4"),
                        ("x", "<f4"), ("y", "<f4"), ("score", "<f4"), ("goal", "<f4"),
                        ("ball", "<f4"), ("angle", "<f4"), ("guard", "<f4"),
                        ("defense", "<f4")])

# Running-point parameters (Sec. 5.2; the paper gives no values): Eq. (4)
# weights, the ball-distance and guard-time scales, the preferred bearing
# window 15-45 degrees with a 30-degree fall-off, the SSL 2019 division A
# defense area (1.2 m deep, 2.4 m wide) and a 1 m marking radius.
RUN_DEFAULTS = dict(w_goal=0.3, w_ball=0.1, w_angle=0.15, w_guard=0.25, w_defense=0.2,
                    ball_norm=2.0, ang_lo=0.2617993877991494, ang_hi=0.7853981633974483,
                    ang_fall=0.5235987755982988, guard_norm=2.0, def_depth=1.2, def_width=2.4,
                    mark_radius=1.0)


class DppsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"dpps error {code}: {msg}")
        self.code = code


class Params_C(C.Structure):
    _fields_ = [(n, C.c_float) for n in (
        "field_len", "field_wid", "goal_x", "goal_width", "robot_radius", "vmax", "amax",
        "slide_decel", "roll_decel", "slide_ratio", "chip_angle", "gravity")] + [
        ("n_samples", C.c_int32)] + [(n, C.c_float) for n in (
            "margin_s", "margin_cap_s", "w_angle", "w_dist", "w_margin", "dist_norm",
            "goal_eps")] + [("out_flags", C.c_uint32), ("reserved", C.c_uint32),
                            ("hbm_budget_bytes", C.c_uint64)]


class Outputs_C(C.Structure):
    _fields_ = [("mask", C.c_void_p), ("score", C.c_void_p), ("t_team", C.c_void_p),
                ("t_opp", C.c_void_p), ("best", C.c_void_p)]


class RayParams_C(C.Structure):
    _fields_ = [("n_dirs", C.c_int32), ("w_time", C.c_float), ("w_refract", C.c_float),
                ("reserved", C.c_int32)]


class RunParams_C(C.Structure):
    _fields_ = [(n, C.c_float) for n in (
        "w_goal", "w_ball", "w_angle", "w_guard", "w_defense", "ball_norm", "ang_lo", "ang_hi",
        "ang_fall", "guard_norm", "def_depth", "def_width", "mark_radius")] + [
        ("reserved", C.c_int32)]


class ShotParams_C(C.Structure):
    _fields_ = [("v_shot", C.c_float), ("min_angle", C.c_float), ("margin_s", C.c_float),
                ("reserved", C.c_int32)]


class PowerParams_C(C.Structure):
    _fields_ = [("buffer_s", C.c_float), ("v_min", C.c_float), ("v_max", C.c_float),
                ("reserved", C.c_int32)]


class RayOutputs_C(C.Structure):
    _fields_ = [("mask", C.c_void_p), ("score", C.c_void_p), ("t_team", C.c_void_p),
                ("t_opp", C.c_void_p), ("s_recv", C.c_void_p), ("best", C.c_void_p)]


_lib = None


def lib():
    """Load libdpps.so; raise if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.dpps_create.argtypes = [C.POINTER(vp), C.POINTER(Params_C), C.c_int, vp]
        L.dpps_destroy.argtypes = [vp]
        L.dpps_destroy.restype = None
        L.dpps_layout.argtypes = [C.POINTER(Params_C), i32, vp, vp, C.POINTER(i64)]
        L.dpps_request_bytes.argtypes = [C.POINTER(Params_C), i32, vp, vp, i32,
                                         C.POINTER(C.c_uint64)]
        L.dpps_device_bytes.argtypes = [vp]
        L.dpps_device_bytes.restype = C.c_uint64
        L.dpps_search.argtypes = [vp, vp, vp, vp, vp, C.POINTER(Outputs_C), vp]
        L.dpps_search_batch.argtypes = [vp, i32, vp, vp, vp, vp, C.POINTER(Outputs_C), vp]
        L.dpps_search_batch_noalloc.argtypes = [vp, i32, vp, vp, vp, vp, C.POINTER(Outputs_C),
                                                vp]
        L.dpps_batch_create.argtypes = [vp, i32, vp, vp, vp, vp, C.POINTER(vp)]
        L.dpps_batch_set_robots.argtypes = [vp, vp, vp, vp]
        L.dpps_batch_run.argtypes = [vp, vp, C.POINTER(Outputs_C), vp, C.c_int]
        L.dpps_batch_destroy.argtypes = [vp]
        L.dpps_batch_destroy.restype = None
        L.dpps_batch_tiles.argtypes = [vp]
        L.dpps_batch_tiles.restype = i64
        L.dpps_batch_points.argtypes = [vp]
        L.dpps_batch_points.restype = i64
        L.dpps_set_launch.argtypes = [vp, i32, i32, i32]
        L.dpps_get_launch.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
        L.dpps_last_kernel_ms.argtypes = [vp]
        L.dpps_last_kernel_ms.restype = C.c_float
        L.dpps_autotune.argtypes = [vp, vp, C.POINTER(Outputs_C), vp, C.c_char_p, i32,
                                    C.POINTER(C.c_float)]
        pf = C.POINTER(C.c_float)
        L.dpps_mlp_param_count.argtypes = []
        L.dpps_mlp_param_count.restype = i64
        L.dpps_mlp_create.argtypes = [vp, i32, i32, C.c_uint64, C.POINTER(vp)]
        L.dpps_mlp_destroy.argtypes = [vp]
        L.dpps_mlp_destroy.restype = None
        L.dpps_mlp_set_params.argtypes = [vp, vp, i64]
        L.dpps_mlp_get_params.argtypes = [vp, vp, i64]
        L.dpps_mlp_get_grads.argtypes = [vp, vp, i64]
        L.dpps_mlp_get_adam.argtypes = [vp, vp, vp, i64, C.POINTER(i64)]
        L.dpps_mlp_set_adam.argtypes = [vp, vp, vp, i64, i64]
        L.dpps_mlp_forward.argtypes = [vp, vp, vp, i64, vp]
        f32 = C.c_float
        L.dpps_mlp_loss_grad.argtypes = [vp, vp, vp, i64, f32, f32, f32, pf, vp]
        L.dpps_pool_cells.argtypes = [vp, i32, i32, i32, vp, i32, i32, vp]
        L.dpps_mlp_adam.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float, C.c_float, vp]
        L.dpps_mlp_train_step.argtypes = [vp, vp, vp, i64, f32, f32, f32, f32, pf, vp]
        L.dpps_mlp_features.argtypes = [vp, vp, vp, vp]
        L.dpps_mlp_topk.argtypes = [vp, i32, i32, vp, vp]
        L.dpps_surrogate_search.argtypes = [vp, vp, vp, i32, vp, C.c_int, C.c_float,
                                            C.POINTER(i32), vp]
        L.dpps_surrogate_search_frames.argtypes = [vp, vp, i32, vp, vp, vp, vp, i32, vp, C.c_int,
                                                   C.c_float, C.POINTER(i32), vp, vp]
        L.dpps_ray_search.argtypes = [vp, i32, vp, vp, vp, C.POINTER(RayParams_C),
                                      C.POINTER(RayOutputs_C), vp]
        L.dpps_shot_decision.argtypes = [vp, i32, vp, vp, vp, C.POINTER(ShotParams_C), vp, vp,
                                         vp]
        L.dpps_running_points.argtypes = [vp, i32, vp, vp, vp, C.POINTER(RunParams_C), vp, vp,
                                          vp]
        L.dpps_search_power.argtypes = [vp, i32, vp, vp, vp, C.POINTER(PowerParams_C),
                                        C.POINTER(Outputs_C), vp, vp]
        L.dpps_timing_begin.argtypes = [vp, i32]
        L.dpps_timing_end.argtypes = [vp, C.POINTER(C.c_float), C.POINTER(i32)]
        L.dpps_strerror.argtypes = [C.c_int]
        L.dpps_strerror.restype = C.c_char_p
        L.dpps_last_error.argtypes = []
        L.dpps_last_error.restype = C.c_char_p
        L.dpps_version.argtypes = []
        L.dpps_version.restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != DPPS_OK:
        L = lib()
        raise DppsError(rc, f"{L.dpps_strerror(rc).decode()}: {L.dpps_last_error().decode()}")


def params_c(p, out_flags: int = 0, budget: int = 0) -> Params_C:
    """ABI parameter struct from any object with the Params attributes."""
    c = Params_C()
    for name, _ in Params_C._fields_:
        if name in ("out_flags", "reserved", "hbm_budget_bytes"):
            continue
        setattr(c, name, getattr(p, name))
    c.out_flags = out_flags
    c.reserved = 0
    c.hbm_budget_bytes = budget
    return c


@dataclass
class Packed:
    """Host arrays of a request in ABI layout."""
    frames: np.ndarray
    robots: np.ndarray
    windows: np.ndarray
    variants: np.ndarray
    total: int                      # output elements
    frame_elems: np.ndarray         # per-frame element counts


def pack(frames, p, out_flags: int = 0) -> Packed:
    """Pack framegen-style frames (team, opp, passer, ball, windows, variants)."""
    nf = len(frames)
    fr = np.zeros(nf, FRAME_DT)
    rob, win, var = [], [], []
    ro = wo = vo = 0
    for i, f in enumerate(frames):
        team = np.asarray(f.team, np.float32).reshape(-1, 4)
        opp = np.asarray(f.opp, np.float32).reshape(-1, 4)
        fr[i]["n_team"], fr[i]["n_opp"], fr[i]["passer"] = team.shape[0], opp.shape[0], f.passer
        fr[i]["robot_off"], fr[i]["window_off"], fr[i]["variant_off"] = ro, wo, vo
        fr[i]["n_windows"], fr[i]["n_variants"] = len(f.windows), len(f.variants)
        fr[i]["ball_x"], fr[i]["ball_y"] = float(f.ball[0]), float(f.ball[1])
        rob.append(np.concatenate([team, opp]))
        for w in f.windows:
            win.append(tuple(w))
        for v in f.variants:
            var.append((int(v[0]), float(v[1])))
        ro += team.shape[0] + opp.shape[0]
        wo += len(f.windows)
        vo += len(f.variants)
    robots = np.zeros(ro, ROBOT_DT)
    if ro:
        r = np.concatenate(rob).astype(np.float32)
        robots["x"], robots["y"], robots["vx"], robots["vy"] = r[:, 0], r[:, 1], r[:, 2], r[:, 3]
    windows = np.array(win, WINDOW_DT) if win else np.zeros(0, WINDOW_DT)
    variants = np.array(var, VARIANT_DT) if var else np.zeros(0, VARIANT_DT)
    total = C.c_int64()
    pc = params_c(p, out_flags)
    # frames without windows (direction x variant searches) still pass a valid array
    wl = windows if windows.size else np.zeros(1, WINDOW_DT)
    _check(lib().dpps_layout(C.byref(pc), nf, _ptr(fr), _ptr(wl), C.byref(total)))
    ends = np.append(fr["out_off"][1:], total.value) if nf else np.zeros(0, np.int64)
    return Packed(fr, robots, windows, variants, int(total.value),
                  (ends - fr["out_off"]).astype(np.int64) if nf else ends)


def _ptr(a):
    return None if a is None or a.size == 0 else a.ctypes.data


def request_bytes(pk: Packed, p, tile_points: int = 0) -> int:
    """Device bytes a search context needs for the request `pk` (host-only)."""
    pc = params_c(p)
    n = C.c_uint64()
    wl = pk.windows if pk.windows.size else np.zeros(1, WINDOW_DT)
    _check(lib().dpps_request_bytes(C.byref(pc), len(pk.frames), _ptr(pk.frames), _ptr(wl),
                                    tile_points, C.byref(n)))
    return int(n.value)


def _tptr(t):
    return None if t is None else t.data_ptr()


class DeviceOutputs:
    """torch tensors for one request's outputs (device memory)."""

    def __init__(self, total: int, n_frames: int, device, mask=True, score=True, times=False):
        import torch
        self.mask = torch.empty(total, dtype=torch.uint8, device=device) if mask else None
        self.score = torch.empty(total, dtype=torch.float32, device=device) if score else None
        self.t_team = torch.empty(total, dtype=torch.float32, device=device) if times else None
        self.t_opp = torch.empty(total, dtype=torch.float32, device=device) if times else None
        self.best = torch.empty(n_frames * BEST_DT.itemsize, dtype=torch.uint8, device=device)

    def c(self) -> Outputs_C:
        o = Outputs_C()
        o.mask, o.score = _tptr(self.mask), _tptr(self.score)
        o.t_team, o.t_opp = _tptr(self.t_team), _tptr(self.t_opp)
        o.best = _tptr(self.best)
        return o

    def best_host(self) -> np.ndarray:
        return np.frombuffer(self.best.cpu().numpy().tobytes(), BEST_DT)


class RayDeviceOutputs:
    """torch tensors for the outputs of a direction x variant search:
    [sum over frames of n_dirs * n_variants] maps and one record per frame."""

    def __init__(self, total: int, n_frames: int, device, mask=True, score=True, times=True,
                 recv=True):
        import torch
        f32 = dict(dtype=torch.float32, device=device)
        self.mask = torch.empty(total, dtype=torch.uint8, device=device) if mask else None
        self.score = torch.empty(total, **f32) if score else None
        self.t_team = torch.empty(total, **f32) if times else None
        self.t_opp = torch.empty(total, **f32) if times else None
        self.s_recv = torch.empty(total, **f32) if recv else None
        self.best = torch.empty(max(n_frames, 1) * RAY_BEST_DT.itemsize, dtype=torch.uint8,
                                device=device)

    def c(self) -> RayOutputs_C:
        o = RayOutputs_C()
        o.mask, o.score = _tptr(self.mask), _tptr(self.score)
        o.t_team, o.t_opp, o.s_recv = _tptr(self.t_team), _tptr(self.t_opp), _tptr(self.s_recv)
        o.best = _tptr(self.best)
        return o

    def best_host(self) -> np.ndarray:
        return np.frombuffer(self.best.cpu().numpy().tobytes(), RAY_BEST_DT)


def run_best_host(t) -> np.ndarray:
    """RUN_BEST_DT records of a byte tensor written by Searcher.running_points."""
    return np.frombuffer(t.cpu().numpy().tobytes(), RUN_BEST_DT)


def shots_host(t) -> np.ndarray:
    """SHOT_DT records of a byte tensor written by Searcher.shot."""
    return np.frombuffer(t.cpu().numpy().tobytes(), SHOT_DT)


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream) if hasattr(stream, "cuda_stream") else C.c_void_p(stream)


class Searcher:
    """A libdpps context on one device."""

    def __init__(self, params, device: int = 0, out_flags: int = 0, budget: int = 0, stream=None):
        import torch
        self.params = params
        self.out_flags = out_flags
        self.device = torch.device("cuda", device)
        self.pc = params_c(params, out_flags, budget)
        h = C.c_void_p()
        torch.cuda.init()
        sp = None if stream is None else _stream_ptr(stream)
        _check(lib().dpps_create(C.byref(h), C.byref(self.pc), device, sp))
        self.h = h

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().dpps_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def device_bytes(self) -> int:
        """Device memory the context holds now."""
        return int(lib().dpps_device_bytes(self.h))

    def set_launch(self, tile_points=0, waves=0, wg_per_cu=0):
        _check(lib().dpps_set_launch(self.h, tile_points, waves, wg_per_cu))

    def get_launch(self):
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().dpps_get_launch(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def outputs_for(self, pk: Packed, mask=True, score=True, times=False) -> DeviceOutputs:
        return DeviceOutputs(pk.total, len(pk.frames), self.device, mask, score, times)

    def search(self, frame, mask=True, score=True, times=False, out=None):
        """One frame (a framegen frame or a one-frame Packed request),
        synchronous.  Returns (DeviceOutputs, best record); `out` reuses the
        DeviceOutputs of an earlier call of the same size."""
        pk = frame if isinstance(frame, Packed) else pack([frame], self.params, self.out_flags)
        if len(pk.frames) != 1:
            raise ValueError("search() takes one frame")
        if out is None:
            out = self.outputs_for(pk, mask, score, times)
        oc = out.c()
        best = np.zeros(1, BEST_DT)
        _check(lib().dpps_search(self.h, _ptr(pk.frames), _ptr(pk.robots), _ptr(pk.windows),
                                 _ptr(pk.variants), C.byref(oc), best.ctypes.data))
        return out, best[0]

    def running_points(self, frames, score: bool = True, stream=None, out=None, **run):
        """Running points (Sec. 5.2) over each frame's windows as zones
        (e.g. zones.front_zones()); asynchronous on the stream.  Returns (best,
        score): best a byte tensor of RUN_BEST_DT records, one per zone in
        frame then window order (run_best_host() converts it), score a float
        tensor per zone point (None without score).  Keyword arguments
        override RUN_DEFAULTS."""
        import torch
        if isinstance(frames, Packed):
            pk = frames
        else:
            fr = []
            for f in frames:
                g = f.copy()
                g.variants = [(DPPS_FLAT, 1.0)]
                fr.append(g)
            pk = pack(fr, self.params, self.out_flags)
        n_zones = int(pk.frames["n_windows"].astype(np.int64).sum())
        if out is not None:
            best, sc = out
        else:
            best = torch.empty(max(n_zones, 1) * RUN_BEST_DT.itemsize, dtype=torch.uint8,
                               device=self.device)
            sc = torch.empty(max(pk.total, 1), dtype=torch.float32, device=self.device)
        if not score:
            sc = None
        v = dict(RUN_DEFAULTS)
        unknown = set(run) - set(v)
        if unknown:
            raise TypeError(f"unknown running-point parameters {sorted(unknown)}")
        v.update(run)
        rp = RunParams_C(*[float(v[k]) for k, _ in RunParams_C._fields_[:-1]], 0)
        _check(lib().dpps_running_points(self.h, len(pk.frames), _ptr(pk.frames), _ptr(pk.robots),
                                         _ptr(pk.windows), C.byref(rp),
                                         sc.data_ptr() if sc is not None else None,
                                         best.data_ptr(), _stream_ptr(stream)))
        return best, sc

    def pack_shots(self, frames, v_shot: float = 6.5, map: bool = True) -> "Packed":
        """Pack frames for shot(): one flat variant at v_shot per frame, and
        no windows without map."""
        fr = []
        for f in frames:
            g = f.copy()
            g.variants = [(DPPS_FLAT, float(v_shot))]
            if not map:
                g.windows = []
            fr.append(g)
        return pack(fr, self.params, self.out_flags)

    def shot(self, frames, v_shot: float = 6.5, min_angle: float = 0.05, margin_s: float = 0.0,
             map: bool = True, stream=None, out=None):
        """Shooting decisions (Sec. 4.4) from each frame's ball and, with map,
        from every point of the frames' windows; asynchronous on the stream.
        `frames` are framegen frames or a Packed from pack_shots.  Returns
        (ball, map) as byte tensors of SHOT_DT records (map None without map;
        `out` may pass tensors to reuse); shots_host() converts them."""
        import torch
        pk = frames if isinstance(frames, Packed) else self.pack_shots(frames, v_shot, map)
        n = len(pk.frames)
        if out is not None:
            ball, mp = out
        else:
            ball = torch.empty(max(n, 1) * SHOT_DT.itemsize, dtype=torch.uint8,
                               device=self.device)
            mp = None
            if map:
                mp = torch.empty(max(pk.total, 1) * SHOT_DT.itemsize, dtype=torch.uint8,
                                 device=self.device)
        if not map:
            mp = None
        sp = ShotParams_C(float(v_shot), float(min_angle), float(margin_s), 0)
        _check(lib().dpps_shot_decision(self.h, n, _ptr(pk.frames), _ptr(pk.robots),
                                        _ptr(pk.windows), C.byref(sp), ball.data_ptr(),
                                        mp.data_ptr() if mp is not None else None,
                                        _stream_ptr(stream)))
        return ball, mp

    def search_power(self, frames, buffer_s: float = 0.3, v_min: float = 1.0,
                     v_max: float = 6.5, mask=True, score=True, times=True, stream=None):
        """Every point of the frames' windows with one flat pass at the point's
        own passing power (Eq. 1-2), asynchronous on the stream.  Returns
        (DeviceOutputs, v0) with one element per point (the frames' variants
        are not used)."""
        import torch
        one = [(DPPS_FLAT, float(v_min))]
        fr = []
        for f in frames:
            g = f.copy()
            g.variants = list(one)
            fr.append(g)
        pk = pack(fr, self.params, self.out_flags)
        out = self.outputs_for(pk, mask, score, times)
        v0 = torch.empty(max(pk.total, 1), dtype=torch.float32, device=self.device)
        pp = PowerParams_C(float(buffer_s), float(v_min), float(v_max), 0)
        oc = out.c()
        _check(lib().dpps_search_power(self.h, len(fr), _ptr(pk.frames), _ptr(pk.robots),
                                       _ptr(pk.windows), C.byref(pp), C.byref(oc),
                                       v0.data_ptr(), _stream_ptr(stream)))
        return out, v0[:pk.total]

    def ray_search(self, frames, n_dirs: int = 128, w_time: float = 0.05, w_refract: float = 0.1,
                   mask=True, score=True, times=True, recv=True, stream=None, out=None):
        """The paper's direction x variant search of framegen frames (or a
        Packed request), asynchronous on the stream.  Returns RayDeviceOutputs;
        frame f's maps are [n_dirs][n_variants] starting at the sum of
        n_dirs * n_variants over the frames before it."""
        pk = frames if isinstance(frames, Packed) else pack(frames, self.params, self.out_flags)
        nf = len(pk.frames)
        total = int(n_dirs * pk.frames["n_variants"].astype(np.int64).sum())
        if out is None:
            out = RayDeviceOutputs(total, nf, self.device, mask, score, times, recv)
        rp = RayParams_C(int(n_dirs), float(w_time), float(w_refract), 0)
        oc = out.c()
        _check(lib().dpps_ray_search(self.h, nf, _ptr(pk.frames), _ptr(pk.robots),
                                     _ptr(pk.variants), C.byref(rp), C.byref(oc),
                                     _stream_ptr(stream)))
        return out

    def search_batch(self, frames, mask=True, score=True, times=False, stream=None, out=None):
        """Many frames, asynchronous on the stream.  Returns (Packed, DeviceOutputs)."""
        pk = frames if isinstance(frames, Packed) else pack(frames, self.params, self.out_flags)
        if out is None:
            out = self.outputs_for(pk, mask, score, times)
        oc = out.c()
        _check(lib().dpps_search_batch(self.h, len(pk.frames), _ptr(pk.frames), _ptr(pk.robots),
                                       _ptr(pk.windows), _ptr(pk.variants), C.byref(oc),
                                       _stream_ptr(stream)))
        return pk, out

    def search_batch_noalloc(self, frames, out, stream=None):
        """search_batch with the library's fixed device array as its only
        device state (no allocation in the call); `out` is caller-owned."""
        pk = frames if isinstance(frames, Packed) else pack(frames, self.params, self.out_flags)
        oc = out.c()
        _check(lib().dpps_search_batch_noalloc(self.h, len(pk.frames), _ptr(pk.frames),
                                               _ptr(pk.robots), _ptr(pk.windows),
                                               _ptr(pk.variants), C.byref(oc),
                                               _stream_ptr(stream)))
        return pk

    def batch(self, frames) -> "Batch":
        pk = frames if isinstance(frames, Packed) else pack(frames, self.params, self.out_flags)
        return Batch(self, pk)

    def last_kernel_ms(self) -> float:
        return float(lib().dpps_last_kernel_ms(self.h))

    def timing_begin(self, max_runs: int):
        _check(lib().dpps_timing_begin(self.h, max_runs))

    def timing_end(self):
        """(total search-kernel ms, runs recorded) since timing_begin."""
        ms, n = C.c_float(), C.c_int32()
        _check(lib().dpps_timing_end(self.h, C.byref(ms), C.byref(n)))
        return float(ms.value), int(n.value)


class Batch:
    """A device-resident batch (inputs uploaded once)."""

    def __init__(self, s: Searcher, pk: Packed):
        self.s = s
        self.pk = pk
        b = C.c_void_p()
        _check(lib().dpps_batch_create(s.h, len(pk.frames), _ptr(pk.frames), _ptr(pk.robots),
                                       _ptr(pk.windows), _ptr(pk.variants), C.byref(b)))
        self.h = b

    @property
    def tiles(self) -> int:
        return int(lib().dpps_batch_tiles(self.h))

    @property
    def points(self) -> int:
        return int(lib().dpps_batch_points(self.h))

    def run(self, out: DeviceOutputs, stream=None, graph: bool = False):
        self._oc = out.c()
        _check(lib().dpps_batch_run(self.s.h, self.h, C.byref(self._oc), _stream_ptr(stream),
                                    int(graph)))

    def autotune(self, out: DeviceOutputs, cache_path: str | None = None, reps: int = 3,
                 stream=None) -> float:
        """Pick the fastest launch shape for this batch (see dpps_autotune);
        returns its average kernel ms, or -1 when it came from the cache."""
        oc = out.c()
        ms = C.c_float()
        cp = cache_path.encode() if cache_path else None
        _check(lib().dpps_autotune(self.s.h, self.h, C.byref(oc), _stream_ptr(stream), cp, reps,
                                   C.byref(ms)))
        return float(ms.value)

    def set_robots(self, robots: np.ndarray, stream=None):
        r = np.ascontiguousarray(robots, ROBOT_DT)
        _check(lib().dpps_batch_set_robots(self.s.h, self.h, r.ctypes.data, _stream_ptr(stream)))

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().dpps_batch_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


MLP_OUT = 2806
MLP_IN = 66


class Mlp:
    """The learned surrogate network on a Searcher's context (dpps_mlp_*)."""

    def __init__(self, s: Searcher, max_frames: int, max_k: int = 64, seed: int = 0):
        self.s = s
        self.max_frames = max_frames
        h = C.c_void_p()
        _check(lib().dpps_mlp_create(s.h, max_frames, max_k, seed, C.byref(h)))
        self.h = h
        self.n = int(lib().dpps_mlp_param_count())

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().dpps_mlp_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self) -> np.ndarray:
        a = np.zeros(self.n, np.float32)
        _check(lib().dpps_mlp_get_params(self.h, a.ctypes.data, self.n))
        return a

    def set_params(self, a: np.ndarray):
        a = np.ascontiguousarray(a, np.float32)
        _check(lib().dpps_mlp_set_params(self.h, a.ctypes.data, a.size))

    def get_grads(self) -> np.ndarray:
        a = np.zeros(self.n, np.float32)
        _check(lib().dpps_mlp_get_grads(self.h, a.ctypes.data, self.n))
        return a

    def get_adam(self):
        m = np.zeros(self.n, np.float32)
        v = np.zeros(self.n, np.float32)
        st = C.c_int64()
        _check(lib().dpps_mlp_get_adam(self.h, m.ctypes.data, v.ctypes.data, self.n, C.byref(st)))
        return m, v, int(st.value)

    def set_adam(self, m, v, step: int):
        m = np.ascontiguousarray(m, np.float32)
        v = np.ascontiguousarray(v, np.float32)
        _check(lib().dpps_mlp_set_adam(self.h, m.ctypes.data, v.ctypes.data, self.n, step))

    def forward(self, batch: "Batch", out=None, stream=None):
        import torch
        nf = len(batch.pk.frames)
        if out is None:
            out = torch.empty((nf, MLP_OUT), dtype=torch.float32, device=self.s.device)
        _check(lib().dpps_mlp_forward(self.h, batch.h, out.data_ptr(), out.stride(0),
                                      _stream_ptr(stream)))
        return out

    def loss_grad(self, batch: "Batch", target, pos_weight: float = 0.0, ce_weight: float = 0.0,
                  tau: float = 0.02, stream=None) -> float:
        loss = C.c_float()
        _check(lib().dpps_mlp_loss_grad(self.h, batch.h, target.data_ptr(), target.stride(0),
                                        pos_weight, ce_weight, tau, C.byref(loss),
                                        _stream_ptr(stream)))
        return float(loss.value)

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0, stream=None):
        _check(lib().dpps_mlp_adam(self.h, lr, beta1, beta2, eps, weight_decay,
                                   _stream_ptr(stream)))

    def train_step(self, batch: "Batch", target, lr: float, pos_weight: float = 0.0,
                   ce_weight: float = 0.0, tau: float = 0.02, stream=None, want_loss=True):
        """One training step; returns the loss (synchronises), or None with
        want_loss=False (stays asynchronous on the stream)."""
        loss = C.c_float()
        _check(lib().dpps_mlp_train_step(self.h, batch.h, target.data_ptr(), target.stride(0), lr,
                                         pos_weight, ce_weight, tau,
                                         C.byref(loss) if want_loss else None,
                                         _stream_ptr(stream)))
        return float(loss.value) if want_loss else None

    def features(self, batch: "Batch", stream=None):
        """bfloat16 network inputs [n_frames][66] as a float32 torch tensor."""
        import torch
        nf = len(batch.pk.frames)
        raw = torch.empty((nf, MLP_IN), dtype=torch.int16, device=self.s.device)
        _check(lib().dpps_mlp_features(self.h, batch.h, raw.data_ptr(), _stream_ptr(stream)))
        return raw.view(torch.bfloat16).float()

    def topk(self, n_frames: int, k: int, stream=None):
        import torch
        out = torch.empty((n_frames, k), dtype=torch.int32, device=self.s.device)
        _check(lib().dpps_mlp_topk(self.h, n_frames, k, out.data_ptr(), _stream_ptr(stream)))
        return out

    def search(self, batch: "Batch", k: int = 64, fallback: bool = True, best=None, stream=None,
               fallback_below: float = float("-inf")):
        """Surrogate search; returns (best records on device as bytes tensor, fallbacks).
        With fallback, frames with no feasible proposal or a best re-scored
        score below `fallback_below` are searched exactly."""
        import torch
        nf = len(batch.pk.frames)
        if best is None:
            best = torch.empty(nf * BEST_DT.itemsize, dtype=torch.uint8, device=self.s.device)
        nfb = C.c_int32()
        _check(lib().dpps_surrogate_search(self.s.h, self.h, batch.h, k, best.data_ptr(),
                                           int(fallback), float(fallback_below), C.byref(nfb),
                                           _stream_ptr(stream)))
        return best, int(nfb.value)

    def search_frames(self, frames, k: int = 64, fallback: bool = True, best=None, stream=None,
                      fallback_below: float = float("-inf"), host=None, count: bool = True):
        """Surrogate search of host frames (a Packed request or framegen
        frames) through the context's own staging; same results as search()
        on a batch of the same frames.  With `host` (a numpy BEST_DT array of
        at least n_frames records) the records are also written there and
        the call returns when they are final.  With count=False (and no
        `host`) the call does not wait for the stream and returns -1 as the
        number of fallbacks."""
        import torch
        pk = frames if isinstance(frames, Packed) else pack(frames, self.s.params)
        nf = len(pk.frames)
        if best is None:
            best = torch.empty(nf * BEST_DT.itemsize, dtype=torch.uint8, device=self.s.device)
        if host is not None:
            assert host.dtype == BEST_DT and host.size >= nf and host.flags["C_CONTIGUOUS"]
        nfb = C.c_int32()
        _check(lib().dpps_surrogate_search_frames(
            self.s.h, self.h, nf, _ptr(pk.frames), _ptr(pk.robots), _ptr(pk.windows),
            _ptr(pk.variants), k, best.data_ptr(), int(fallback), float(fallback_below),
            C.byref(nfb) if count else None, host.ctypes.data if host is not None else None,
            _stream_ptr(stream)))
        return best, int(nfb.value) if count else -1


def pool_cells(fine, fine_nx: int, fine_ny: int, coarse_nx: int = 61, coarse_ny: int = 46,
               out=None, stream=None):
    """Coarse-cell labels (device [n][coarse_ny*coarse_nx]) from fine score
    maps (device f32, n * fine_ny * fine_nx elements)."""
    import torch
    n = fine.numel() // (fine_nx * fine_ny)
    if out is None:
        out = torch.empty((n, coarse_nx * coarse_ny), dtype=torch.float32, device=fine.device)
    _check(lib().dpps_pool_cells(fine.data_ptr(), n, fine_nx, fine_ny, out.data_ptr(), coarse_nx,
                                 coarse_ny, _stream_ptr(stream)))
    return out


def best_records(t) -> np.ndarray:
    """dpps_best records from a device byte tensor."""
    return np.frombuffer(t.cpu().numpy().tobytes(), BEST_DT)


def pack_uniform(team: np.ndarray, opp: np.ndarray, passer: np.ndarray, windows, variants, p,
                 out_flags: int = 0) -> Packed:
    """Vectorised pack of frames that share robot counts, windows and
    variants (team [n, nt, 4], opp [n, no, 4], passer [n]); the ball sits on
    the passer.  `windows` is a list shared by every frame, or an array
    [n, nw, 5] of (h, i0, j0, nx, ny) per frame."""
    n, nt, no = team.shape[0], team.shape[1], opp.shape[1]
    per_frame = isinstance(windows, np.ndarray) and windows.ndim == 3
    nw, nv = (windows.shape[1] if per_frame else len(windows)), len(variants)
    fr = np.zeros(n, FRAME_DT)
    idx = np.arange(n)
    fr["n_team"], fr["n_opp"], fr["passer"] = nt, no, passer
    fr["robot_off"] = idx * (nt + no)
    fr["n_windows"], fr["window_off"] = nw, idx * nw
    fr["n_variants"], fr["variant_off"] = nv, idx * nv
    fr["ball_x"] = team[idx, passer, 0]
    fr["ball_y"] = team[idx, passer, 1]
    r = np.concatenate([team, opp], axis=1).reshape(-1, 4).astype(np.float32)
    robots = np.zeros(r.shape[0], ROBOT_DT)
    robots["x"], robots["y"], robots["vx"], robots["vy"] = r[:, 0], r[:, 1], r[:, 2], r[:, 3]
    if per_frame:
        wa = windows.reshape(-1, 5)
        win = np.zeros(wa.shape[0], WINDOW_DT)
        win["h"] = wa[:, 0]
        for c, name in enumerate(("i0", "j0", "nx", "ny")):
            win[name] = wa[:, c + 1].astype(np.int32)
    else:
        win = np.array([tuple(w) for w in windows] * n, WINDOW_DT)
    var = np.array([(int(v[0]), float(v[1])) for v in variants] * n, VARIANT_DT)
    total = C.c_int64()
    pc = params_c(p, out_flags)
    _check(lib().dpps_layout(C.byref(pc), n, _ptr(fr), _ptr(win), C.byref(total)))
    ends = np.append(fr["out_off"][1:], total.value)
    return Packed(fr, robots, win, var, int(total.value), (ends - fr["out_off"]).astype(np.int64))
