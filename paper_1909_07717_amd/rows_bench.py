"""Timed runs of the adjacent rows (passing power per point, shooting
decisions, running points, the direction x power sweep) on one GPU: each
returns a dict of throughput, kernel time and modelled FP32 work.  Used by
the benchmark script and by the profiling runner."""
from __future__ import annotations

import time

from paper_1909_07717_amd.zones import front_zones


def power_bench(steps: int, st, launch=None):
    """Per-point passing power (Sec. 4.1, Eq. 1-2): the full frame's 8v8 robots
    and 5 cm lattice (43 621 points), one flat pass per point at the point's
    own power (receiver + 0.3 s, kick range 1-6.5 m/s), K = 256; inputs staged
    from the host on every call.  launch: (tile points, waves, workgroups per
    CU) for the search, e.g. the full frame's tuned shape (same lattice and
    K); None keeps the context's default."""
    import torch

    from paper_1909_07717_amd import binding as Bn
    from paper_1909_07717_amd.framegen import Params, config_full

    p = Params(n_samples=256).as_f32()
    f = config_full(100)
    s = Bn.Searcher(p, device=0)
    if launch is not None:
        s.set_launch(*launch)
    shape = s.get_launch()
    with torch.cuda.stream(st):
        out, v0 = s.search_power([f], stream=st)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(st):
        e0.record(st)
        for _ in range(steps):
            s.search_power([f], stream=st)
        e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / steps
    feas = int(out.mask.sum().item())
    vv = v0.cpu()
    s.close()
    return {"workload": "full frame 8v8, 5 cm lattice 241x181, one flat pass per point at its "
                        "own power (Eq. 1-2), K = 256", "points": 43621,
            "ms_per_frame": round(ms, 4), "points_per_s": round(43621 / (ms * 1e-3), 1),
            "feasible_points": feas, "v0_min": round(float(vv.min()), 4),
            "v0_max": round(float(vv.max()), 4),
            "launch": {"tile_points": shape[0], "waves_per_wg": shape[1],
                       "wg_per_cu": shape[2]}}


def shot_bench(n_frames: int, steps: int, lat_frames: int, st):
    """Shooting decision (Sec. 4.4), flat shot at 6.5 m/s, gap threshold
    0.05 rad: (a) from the ball of n_frames 8v8 frames per call, K = 128;
    (b) the shot map of a full 5 cm lattice (43 621 shooter positions, 8
    opponents), K = 256; (c) latency of one frame's decision, host inputs to
    the record on the host.  (a) and (b) pack the frames once; the library
    still stages them from the host on every call."""
    import numpy as np
    import torch

    from paper_1909_07717_amd import binding as Bn
    from paper_1909_07717_amd import flops as FL
    from paper_1909_07717_amd.framegen import Params, config_full, random_frame

    res = {}
    p = Params(n_samples=128).as_f32()
    s = Bn.Searcher(p, device=0)
    frames = [random_frame(np.random.default_rng(700 + i), 8, 8, Params())
              for i in range(n_frames)]
    pk = s.pack_shots(frames, map=False)
    with torch.cuda.stream(st):
        ball, _ = s.shot(pk, map=False, stream=st)
    torch.cuda.synchronize()
    n_shoot = int(Bn.shots_host(ball)[:n_frames]["shoot"].sum())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(st):
        e0.record(st)
        for _ in range(steps):
            s.shot(pk, map=False, stream=st, out=(ball, None))
        e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / steps
    res["ball"] = {"workload": f"{n_frames} frames of 8v8, decision from the ball, K = 128",
                   "ms_per_call": round(ms, 4),
                   "decisions_per_s": round(n_frames / (ms * 1e-3), 1),
                   "shoot_fraction": round(n_shoot / n_frames, 4)}
    lat = []
    b1 = torch.empty(Bn.SHOT_DT.itemsize, dtype=torch.uint8, device=ball.device)
    host = torch.empty(Bn.SHOT_DT.itemsize, dtype=torch.uint8, pin_memory=True)
    for i in range(100 + lat_frames):
        a = time.perf_counter()
        with torch.cuda.stream(st):
            s.shot([frames[i % n_frames]], map=False, stream=st, out=(b1, None))
            host.copy_(b1, non_blocking=True)
        st.synchronize()
        if i >= 100:
            lat.append(time.perf_counter() - a)
    lat = np.array(lat) * 1e3
    res["latency_ms"] = {"p50": round(float(np.percentile(lat, 50)), 4),
                         "p99": round(float(np.percentile(lat, 99)), 4), "frames": int(lat.size),
                         "path": "one frame per call, host inputs to the decision on the host"}
    s.close()
    p = Params(n_samples=256).as_f32()
    s = Bn.Searcher(p, device=0)
    f = config_full(100)
    pk = s.pack_shots([f])
    with torch.cuda.stream(st):
        bm, mp = s.shot(pk, stream=st)
    torch.cuda.synchronize()
    n = 43621
    n_shoot = int(Bn.shots_host(mp)[:n]["shoot"].sum())
    with torch.cuda.stream(st):
        e0.record(st)
        for _ in range(steps):
            s.shot(pk, stream=st, out=(bm, mp))
        e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / steps
    fl = n * FL.shot_flops(int(np.asarray(f.opp).shape[0]), 256)
    res["map"] = {"workload": "shot map of the full 5 cm lattice 241x181, 8 opponents, K = 256",
                  "ms_per_frame": round(ms, 4), "positions_per_s": round(n / (ms * 1e-3), 1),
                  "tflops": round(fl / (ms * 1e-3) / 1e12, 3),
                  "frac": round(FL.tflops(fl, ms) / FL.PEAK_FP32_VECTOR_TFLOPS, 4),
                  "frac_of_nonpacked": round(FL.tflops(fl, ms) / FL.PEAK_FP32_NONPACKED_TFLOPS, 4),
                  "shoot_fraction": round(n_shoot / n, 4)}
    s.close()
    return res


def run_bench(n_frames: int, steps: int, lat_frames: int, st):
    """Running points (Sec. 5.2): n_frames 8v8 frames, each with the four
    front-field zones at 0.1 m that follow its ball, per call (frames packed
    once, staged from the host on every call); latency of one frame's four
    zone bests, host inputs to the records on the host."""
    import numpy as np
    import torch

    from paper_1909_07717_amd import binding as Bn
    from paper_1909_07717_amd import flops as FL
    from paper_1909_07717_amd.framegen import Params, random_frame

    p = Params(n_samples=64).as_f32()
    s = Bn.Searcher(p, device=0)
    frames = []
    for i in range(n_frames):
        f = random_frame(np.random.default_rng(800 + i), 8, 8, Params())
        f.windows = front_zones(f.ball, p)
        f.variants = [(Bn.DPPS_FLAT, 1.0)]
        frames.append(f)
    pk = Bn.pack(frames, p)
    pts = int(pk.total)
    with torch.cuda.stream(st):
        best, sc = s.running_points(pk, stream=st)
    torch.cuda.synchronize()
    found = float(Bn.run_best_host(best)["found"][:4 * n_frames].mean())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(st):
        e0.record(st)
        for _ in range(steps):
            s.running_points(pk, stream=st, out=(best, sc))
        e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / steps
    lat = []
    b1 = torch.empty(4 * Bn.RUN_BEST_DT.itemsize, dtype=torch.uint8, device=best.device)
    s1 = torch.empty(8192, dtype=torch.float32, device=best.device)
    host = torch.empty(4 * Bn.RUN_BEST_DT.itemsize, dtype=torch.uint8, pin_memory=True)
    for i in range(100 + lat_frames):
        a = time.perf_counter()
        with torch.cuda.stream(st):
            s.running_points([frames[i % n_frames]], score=False, stream=st, out=(b1, s1))
            host.copy_(b1, non_blocking=True)
        st.synchronize()
        if i >= 100:
            lat.append(time.perf_counter() - a)
    lat = np.array(lat) * 1e3
    s.close()
    fl = pts * FL.run_flops(8)
    return {"workload": f"{n_frames} frames of 8v8, four front-field zones at 0.1 m each "
                        f"({pts // n_frames} points per frame)",
            "ms_per_call": round(ms, 4), "points_per_s": round(pts / (ms * 1e-3), 1),
            "zones_per_s": round(4 * n_frames / (ms * 1e-3), 1),
            "tflops": round(fl / (ms * 1e-3) / 1e12, 3),
            "frac": round(FL.tflops(fl, ms) / FL.PEAK_FP32_VECTOR_TFLOPS, 4),
            "frac_of_nonpacked": round(FL.tflops(fl, ms) / FL.PEAK_FP32_NONPACKED_TFLOPS, 4),
            "found_fraction": round(found, 4),
            "score_map_bytes": 4 * pts,
            "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                           "p99": round(float(np.percentile(lat, 99)), 4),
                           "frames": int(lat.size),
                           "path": "one frame per call, host inputs to the zone bests on the host"}}


def ray_bench(n_frames: int, steps: int, lat_frames: int, st):
    """The paper's own DPPS form: 8v8 frames, 128 kick directions x 64 flat
    powers in [1, 6.5] m/s, K = 256 samples per ray.  Batched: n_frames frames
    per call (host inputs staged by the library), timed over `steps` calls;
    latency: one frame per call, host inputs to the best pass on the host."""
    import numpy as np
    import torch

    from paper_1909_07717_amd import binding as Bn
    from paper_1909_07717_amd import flops as FL
    from paper_1909_07717_amd.framegen import Params, random_frame, speeds_linear, variants_for

    n_dirs, speeds = 128, 64
    p = Params(n_samples=256).as_f32()
    var = variants_for(speeds_linear(speeds), flat=True, chip=False)
    frames = []
    for i in range(n_frames):
        f = random_frame(np.random.default_rng(500 + i), 8, 8, Params())
        f.variants = var
        frames.append(f)
    s = Bn.Searcher(p, device=0)
    pk = Bn.pack(frames, p)
    with torch.cuda.stream(st):
        out = s.ray_search(pk, n_dirs, stream=st)
    torch.cuda.synchronize()
    n_feas = out.mask.view(n_frames, -1).sum(1).cpu().numpy()
    evals = fl = 0
    for f, nf in zip(frames, n_feas):
        e, x = FL.ray_frame_work(f, p.n_samples, n_dirs, int(nf))
        evals += e
        fl += x
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.timing_begin(steps)
    with torch.cuda.stream(st):
        e0.record(st)
        for _ in range(steps):
            s.ray_search(pk, n_dirs, stream=st, out=out)
        e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / steps
    kms, kn = s.timing_end()
    kms /= max(kn, 1)
    # latency, one frame at a time
    one = s.ray_search(frames[:1], n_dirs, stream=st, mask=False, score=False, times=False,
                       recv=False)
    host = torch.empty(Bn.RAY_BEST_DT.itemsize, dtype=torch.uint8, pin_memory=True)
    lat = []
    for i in range(100 + lat_frames):
        a = time.perf_counter()
        with torch.cuda.stream(st):
            s.ray_search([frames[i % n_frames]], n_dirs, stream=st, out=one)
            host.copy_(one.best[:Bn.RAY_BEST_DT.itemsize], non_blocking=True)
        st.synchronize()
        if i >= 100:
            lat.append(time.perf_counter() - a)
    lat = np.array(lat) * 1e3
    s.close()
    return {"workload": f"{n_frames} frames of 8v8, {n_dirs} directions x {speeds} flat powers "
                        f"1.0-6.5 m/s, K = 256 samples per ray",
            "evals_per_call": evals, "ms_per_call": round(ms, 4),
            "frames_per_s": round(n_frames / (ms * 1e-3), 1),
            "pass_evals_per_s": round(evals / (ms * 1e-3), 1),
            # the roofline of the direction-sweep kernel alone (HIP events
            # around it); ms_per_call also stages the frames from the host
            "kernel_ms": round(kms, 4),
            "tflops": round(fl / (kms * 1e-3) / 1e12, 3),
            "frac": round(FL.tflops(fl, kms) / FL.PEAK_FP32_VECTOR_TFLOPS, 4),
            "frac_of_nonpacked": round(FL.tflops(fl, kms) / FL.PEAK_FP32_NONPACKED_TFLOPS, 4),
            "feasible_fraction": round(float(n_feas.sum()) / (n_frames * n_dirs * speeds), 4),
            "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                           "p99": round(float(np.percentile(lat, 99)), 4),
                           "frames": int(lat.size),
                           "path": "one frame per call, host inputs to the best pass on the host"}}
