"""Workloads to run under rocprofv3.

    python3 -m paper_1909_07717_amd.profiling search --steps 20
        the full-frame search of the benchmark (8v8, 5 cm, 32 variants,
        K = 256), inputs resident, `steps` launches;
    python3 -m paper_1909_07717_amd.profiling copy --mib 512 --reps 4
        a plain device-to-device copy of known size, to calibrate the HBM
        byte counters (FETCH_SIZE / WRITE_SIZE) against bytes actually moved.
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def run_search(steps: int, seed: int = 100, reduced: bool = False):
    import torch

    from paper_1909_07717_amd import binding as Bn
    from paper_1909_07717_amd.framegen import Params, config_full

    p = Params(n_samples=256).as_f32()
    s = Bn.Searcher(p, out_flags=Bn.DPPS_OUT_REDUCED if reduced else 0)
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
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=512)
    c.add_argument("--reps", type=int, default=4)
    args = ap.parse_args()
    if args.cmd == "search":
        run_search(args.steps, args.seed, args.reduced)
    else:
        run_copy(args.mib, args.reps)


if __name__ == "__main__":
    main()
