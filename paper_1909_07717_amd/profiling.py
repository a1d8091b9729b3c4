"""Workloads to run under rocprofv3.

    python3 -m paper_1909_07717_amd.profiling search --steps 20
        the full-frame search of the benchmark (8v8, 5 cm, 32 variants,
        K = 256), inputs resident, `steps` launches;
    python3 -m paper_1909_07717_amd.profiling copy --mib 512 --reps 4
        a plain device-to-device copy of known size, to calibrate the HBM
        byte counters (FETCH_SIZE / WRITE_SIZE) against bytes actually moved;
    python3 -m paper_1909_07717_amd.profiling mlp --batch 4096 --steps 20
        the surrogate network: `steps` forward passes, then `steps` training
        steps (forward, loss, backward, Adam) on one batch of 6 v 6 frames
        with synthetic labels;
    python3 -m paper_1909_07717_amd.profiling rows --steps 5
        the benchmark's workloads of the next rows, `steps` calls each: the
        passing-power search of the full frame, the shot decisions and map,
        the running points, the direction x power sweep;
    python3 -m paper_1909_07717_amd.profiling latency --frames 300
        one frame per call (6 v 6, one flat pass at 4 m/s, K = 64, 5 cm):
        the exact search, then the surrogate search with fallback, host
        inputs to the best record on the host.
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def run_search(steps: int, seed: int = 100, reduced: bool = False, launch=None):
    """The full frame of the benchmark (8v8, 5 cm, 32 variants, K = 256),
    inputs resident, `steps` launches; `launch` = (tile_points, waves per
    workgroup, workgroups per CU) or None for the context's default."""
    import torch

    from paper_1909_07717_amd import binding as Bn
    from paper_1909_07717_amd.framegen import Params, config_full

    p = Params(n_samples=256).as_f32()
    s = Bn.Searcher(p, out_flags=Bn.DPPS_OUT_REDUCED if reduced else 0)
    if launch:
        s.set_launch(*launch)
    bt = s.batch([config_full(seed)])
    out = s.outputs_for(bt.pk)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        for _ in range(steps):
            bt.run(out, stream=st)
    torch.cuda.synchronize()
    print(f"search: {steps} launches, {bt.points} points, {bt.tiles} tiles", flush=True)
    bt.close()
    s.close()


MLP_FWD_FLOP = 2 * (66 * 512 + 2 * 512 * 512 + 512 * 2806)  # per frame
# backward: weight gradients of every layer, input gradients of all but the first
MLP_STEP_FLOP = 3 * MLP_FWD_FLOP - 2 * 66 * 512


def mlp_timing(batch: int, steps: int, stream=None):
    """Average forward and training-step times (ms) of the surrogate network
    at `batch` frames, from CUDA events on the stream the kernels run on."""
    import torch

    from paper_1909_07717_amd import binding as Bn
    from paper_1909_07717_amd.framegen import Params, full_window, uniform_batch_arrays, variants_for

    p = Params(n_samples=64).as_f32()
    s = Bn.Searcher(p)
    net = Bn.Mlp(s, batch, seed=1)
    team, opp, passer = uniform_batch_arrays(4242, batch)
    bt = s.batch(Bn.pack_uniform(team, opp, passer, [full_window(0.2)],
                                 variants_for([4.0], flat=True, chip=False), p))
    g = torch.Generator(device="cpu").manual_seed(0)
    lab = torch.rand((batch, 2806), generator=g).to(s.device)
    st = stream or torch.cuda.current_stream()
    out = torch.empty((batch, 2806), dtype=torch.float32, device=s.device)
    res = {}
    with torch.cuda.stream(st):
        for name, fn in (("forward", lambda: net.forward(bt, out=out, stream=st)),
                         ("train_step", lambda: net.train_step(bt, lab, 1e-4, 8.0, 0.2, 0.02,
                                                               stream=st, want_loss=False))):
            for _ in range(3):
                fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(steps):
                fn()
            e1.record(st)
            e1.synchronize()
            res[name + "_ms"] = e0.elapsed_time(e1) / steps
    bt.close()
    net.close()
    s.close()
    fl_f, fl_s = MLP_FWD_FLOP * batch, MLP_STEP_FLOP * batch
    res.update({"batch": batch,
                "forward_tflops": fl_f / (res["forward_ms"] * 1e-3) / 1e12,
                "train_step_tflops": fl_s / (res["train_step_ms"] * 1e-3) / 1e12,
                "bf16_mfma_peak_tflops": 2500.0})
    return res


def run_copy(mib: int, reps: int):
    import torch

    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copy: {reps} x {mib} MiB read + {mib} MiB written", flush=True)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("search")
    a.add_argument("--steps", type=int, default=20)
    a.add_argument("--seed", type=int, default=100)
    a.add_argument("--reduced", action="store_true")
    a.add_argument("--launch", type=int, nargs=3, default=None,
                   metavar=("TILE", "WAVES", "WG_PER_CU"))
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=512)
    c.add_argument("--reps", type=int, default=4)
    m = sub.add_parser("mlp")
    m.add_argument("--batch", type=int, default=4096)
    m.add_argument("--steps", type=int, default=20)
    w = sub.add_parser("rows")
    w.add_argument("--steps", type=int, default=5)
    w.add_argument("--power-launch", type=int, nargs=3, default=None,
                   metavar=("TILE", "WAVES", "WG_PER_CU"))
    q = sub.add_parser("latency")
    q.add_argument("--frames", type=int, default=300)
    q.add_argument("--warmup", type=int, default=50)
    args = ap.parse_args()
    if args.cmd == "search":
        run_search(args.steps, args.seed, args.reduced, args.launch)
    elif args.cmd == "copy":
        run_copy(args.mib, args.reps)
    elif args.cmd == "rows":
        import json

        import torch

        from paper_1909_07717_amd import rows_bench as R
        st = torch.cuda.Stream()
        out = {"power": R.power_bench(args.steps, st, launch=args.power_launch),
               "shots": R.shot_bench(4096, args.steps, 20, st),
               "running": R.run_bench(4096, args.steps, 20, st),
               "rays": R.ray_bench(512, args.steps, 20, st)}
        print(json.dumps({k: v.get("workload", "") for k, v in out.items()}), flush=True)
    elif args.cmd == "latency":
        import json

        from paper_1909_07717_amd.surrogate import WEIGHTS, latency
        print(json.dumps(latency(WEIGHTS, frames=args.frames, warmup=args.warmup)), flush=True)
    else:
        import json
        print(json.dumps(mlp_timing(args.batch, args.steps)), flush=True)


if __name__ == "__main__":
    main()
