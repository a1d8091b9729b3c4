"""Training and evaluation of the learned surrogate (on the GPU, through the
library's own kernels).

    python3 -m paper_1909_07717_amd.surrogate train --frames 2000000 --out W.npz
    python3 -m paper_1909_07717_amd.surrogate eval --weights W.npz --frames 2000

Training frames are 6 v 6 robot states drawn in batches (one generator per
batch, seed = 1 000 000 + batch index), one flat pass at 4 m/s with K = 64
samples.  A frame's label is a 61 x 46 map over the 20 cm cells: by default
("pooled") each cell holds the best exact score among the 5 cm points that
the re-score of that cell visits, from the exact search of the whole 5 cm
lattice on the same device; "center" labels take the exact 20 cm map
instead.  Infeasible points count as score 0.  Loss: squared error weighted
by (1 + pos_weight * label), plus ce_weight times the cross-entropy between
the softmax of the labels and of the outputs at temperature tau (a listwise
term that rewards ranking the best cells first).  Optimiser: Adam with a
cosine-decayed rate.  Labels are computed once per batch and kept in device
memory for later epochs.

Evaluation compares, on frames from a disjoint seed range (20 000 000 + i),
the surrogate search (top-k cells re-scored exactly at 5 cm, exact fallback)
with the exact search of the whole 5 cm lattice: score regret
(S*_exact - S_chosen) / S*_exact, chosen-point match rate and fallback rate.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "surrogate.npz")
TUNE_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.jsonl")


def _tune(s, B, pk, cache):
    """Set the context's launch shape from the autotuner for requests like
    pk (cached per request class in `cache`; None keeps the default)."""
    if cache is None:
        return
    bt = s.batch(pk)
    bt.autotune(s.outputs_for(pk, mask=False, score=False), cache, reps=5)
    bt.close()
TRAIN_SEED = 1_000_000
EVAL_SEED = 20_000_000


def _params():
    from paper_1909_07717_amd.framegen import Params
    return Params(n_samples=64).as_f32()


def _label_setup():
    from paper_1909_07717_amd.framegen import full_window, variants_for
    return [full_window(0.2)], variants_for([4.0], flat=True, chip=False)


def mirror_arrays(team: np.ndarray, opp: np.ndarray):
    """The frames reflected about the field's long axis (y -> -y, vy -> -vy).
    The field, the goal and the lattice are symmetric about it, so the exact
    score map of a reflected frame is the reflected map."""
    t, o = team.copy(), opp.copy()
    for a in (t, o):
        a[..., 1] *= -1.0
        a[..., 3] *= -1.0
    return t, o


def mirror_cells(y):
    """Reflect [n, 2806] maps over the 20 cm cells (row cj <-> 45 - cj)."""
    return y.reshape(y.shape[0], 46, 61).flip(1).reshape(y.shape[0], 2806)


def cell_windows(cells: np.ndarray) -> np.ndarray:
    """5 cm windows [n, k, 5] = (h, i0, j0, nx, ny) of 20 cm cells [n, k]:
    the fine points {4c-2 .. 4c+1} of each axis, clipped to the lattice."""
    ci, cj = cells % 61, cells // 61
    i0, i1 = np.maximum(4 * ci - 2, 0), np.minimum(4 * ci + 1, 240)
    j0, j1 = np.maximum(4 * cj - 2, 0), np.minimum(4 * cj + 1, 180)
    out = np.zeros(cells.shape + (5,), np.float64)
    out[..., 0] = np.float32(0.05)
    out[..., 1], out[..., 2] = i0, j0
    out[..., 3], out[..., 4] = i1 - i0 + 1, j1 - j0 + 1
    return out


def geometric_cells(team: np.ndarray, passer: np.ndarray, variants, k: int,
                    params=None) -> np.ndarray:
    """The proposals of the method without a network: 20 cm cells ranked by
    the terms of the Eq. (3) score that need no robot (open goal angle with
    no blockers, distance to the goal), among the cells within the ball's
    reach of the fastest variant (plus the cell's half-diagonal); ties to
    the lower cell.  Returns [n, k] cell indices."""
    from paper_1909_07717_amd.framegen import Params
    P = params or Params()
    cx = 0.2 * (np.arange(61) - 30.0)
    cy = 0.2 * (np.arange(46) - 22.5)
    X, Y = np.meshgrid(cx, cy)
    X, Y = X.ravel(), Y.ravel()
    hw = P.goal_width / 2
    dx = np.maximum(P.goal_x - X, P.goal_eps)
    ang = np.arctan2(hw - Y, dx) - np.arctan2(-hw - Y, dx)
    prior = (P.w_angle * ang / np.pi
             + P.w_dist * (1.0 - np.hypot(X - P.goal_x, Y) / P.dist_norm))
    reach = 0.0
    for typ, v0 in variants:
        if typ == 0:
            v1 = P.slide_ratio * v0
            D = (v0 * v0 - v1 * v1) / (2 * P.slide_decel) + v1 * v1 / (2 * P.roll_decel)
        else:
            vh = v0 * np.cos(P.chip_angle)
            D = v0 * v0 * np.sin(2 * P.chip_angle) / P.gravity + vh * vh / (2 * P.roll_decel)
        reach = max(reach, D)
    idx = np.arange(team.shape[0])
    bx, by = team[idx, passer, 0], team[idx, passer, 1]
    d = np.hypot(X[None, :] - bx[:, None], Y[None, :] - by[:, None])
    score = np.where(d <= reach + 0.15, prior[None, :], -np.inf)
    return np.argsort(-score, axis=1, kind="stable")[:, :k]


def save_checkpoint(path, net, step: int, extra: dict, params_only: bool = False):
    """Parameters, Adam state and data position (for resume); with
    params_only, the parameters and the metadata alone (8 MB)."""
    tmp = path + ".tmp.npz"
    meta = np.frombuffer(json.dumps(extra).encode(), np.uint8)
    if params_only:
        np.savez(tmp, params=net.get_params(), data_step=np.int64(step), meta=meta)
    else:
        m, v, st = net.get_adam()
        np.savez(tmp, params=net.get_params(), adam_m=m, adam_v=v, adam_step=np.int64(st),
                 data_step=np.int64(step), meta=meta)
    os.replace(tmp, path)


def load_checkpoint(path):
    with np.load(path, allow_pickle=False) as z:
        out = {k: z[k] for k in z.files}
    out["meta"] = json.loads(out["meta"].tobytes().decode()) if "meta" in out else {}
    return out


def train(frames: int, batch: int, lr: float, out: str, resume: str | None = None,
          log_every: int = 20, seed: int = 0, epochs: int = 1, pos_weight: float = 0.0,
          ce_weight: float = 0.0, tau: float = 0.02, labels: str = "pooled",
          params_only: bool = False, mirror: bool = False, init: str | None = None,
          data_seed: int = TRAIN_SEED):
    """`frames` distinct frames (frames // batch seeded batches) seen `epochs`
    times, batch order reshuffled every epoch.  With mirror, every batch also
    appears reflected about the field's long axis (its labels computed
    exactly on the reflected frames), doubling the batches of an epoch.

    labels = "pooled": each 20 cm cell's label is the best exact score over
    the 5 cm points its re-score would visit (exact search of the 5 cm
    lattice, then dpps_pool_cells); "center": the exact score at the cell's
    centre (the 20 cm search).  Labels are computed once per batch by the
    exact kernel and kept in device memory for later epochs.

    init: start from the parameters of a checkpoint (fresh Adam state, the
    schedule from the start); data_seed: the seed of the first training
    batch (batch b uses data_seed + b)."""
    import torch

    from paper_1909_07717_amd import binding as B
    from paper_1909_07717_amd.framegen import full_window, uniform_batch_arrays

    p = _params()
    windows, variants = _label_setup()
    fine = [full_window(0.05)]
    s = B.Searcher(p)
    net = B.Mlp(s, batch, seed=seed)
    n_batches = max(1, frames // batch)
    n_virt = n_batches * (2 if mirror else 1)
    order = np.concatenate([np.random.default_rng(seed + e).permutation(n_virt)
                            for e in range(epochs)])
    steps = len(order)
    start = 0
    if init and not resume:
        net.set_params(load_checkpoint(init)["params"])
    if resume:
        ck = load_checkpoint(resume)
        net.set_params(ck["params"])
        net.set_adam(ck["adam_m"], ck["adam_v"], int(ck["adam_step"]))
        start = int(ck["data_step"])
    st = torch.cuda.Stream()
    cache = torch.empty((n_virt, batch, 2806), dtype=torch.float32, device=s.device)
    have = np.zeros(n_virt, bool)
    tables = {}  # device tables of each batch, kept for later epochs
    fine_out = None
    log = []
    t0 = time.time()
    for step in range(start, steps):
        bi = int(order[step])
        if bi not in tables:
            team, opp, passer = uniform_batch_arrays(data_seed + bi % n_batches, batch)
            if bi >= n_batches:
                team, opp = mirror_arrays(team, opp)
            tables[bi] = s.batch(B.pack_uniform(team, opp, passer, windows, variants, p))
        bt = tables[bi]
        with torch.cuda.stream(st):
            if not have[bi]:
                if labels == "pooled":
                    pkf = B.pack_uniform(team, opp, passer, fine, variants, p)
                    btf = s.batch(pkf)
                    if fine_out is None:
                        fine_out = s.outputs_for(pkf, mask=False)
                    btf.run(fine_out, stream=st)
                    B.pool_cells(fine_out.score, 241, 181, out=cache[bi], stream=st)
                    st.synchronize()
                    btf.close()
                else:
                    lab = s.outputs_for(pk, mask=False)
                    bt.run(lab, stream=st)
                    cache[bi].copy_(lab.score.view(batch, 2806))
                have[bi] = True
            rate = lr * 0.5 * (1.0 + math.cos(math.pi * step / steps)) + 1e-5
            logged = step % log_every == 0 or step == steps - 1
            loss = net.train_step(bt, cache[bi], rate, pos_weight, ce_weight, tau, stream=st,
                                  want_loss=logged)
        if logged:
            rec = {"step": step, "presented": (step + 1) * batch, "loss": loss, "lr": rate,
                   "elapsed_s": round(time.time() - t0, 2)}
            log.append(rec)
            print(json.dumps(rec), flush=True)
    meta = {"frames": n_batches * batch, "epochs": epochs, "batch": batch, "lr": lr,
            "pos_weight": pos_weight, "ce_weight": ce_weight, "tau": tau, "labels": labels,
            "steps": steps, "train_seed": data_seed, "mirror": mirror, "log": log,
            "init": os.path.basename(init) if init else None}
    for t in tables.values():
        t.close()
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    save_checkpoint(out, net, steps, meta, params_only)
    net.close()
    s.close()
    return log


def evaluate(weights: str | None, frames: int, k: int = 64, batch: int = 512, random_net=False,
             seed0: int = EVAL_SEED, dump: str | None = None, proposals: str = "network",
             fallback_below: float = -math.inf, tune_cache: str | None = TUNE_CACHE):
    """Regret statistics of the surrogate search against the exact 5 cm search.

    proposals = "network": the trained (or, with random_net, untrained)
    network's top-k cells; "mirror": the top-k cells of the network's map
    averaged with its (reflected back) map of the reflected frame;
    "geometric": the method without a network (geometric_cells).  All are
    re-scored by the same exact kernel with the same fallback rule.  Frames whose best re-scored pass is infeasible or scores
    below `fallback_below` take the exact search.

    With `dump`, also writes per-frame arrays (npz): the exact best score,
    the surrogate's best re-scored score before any fallback (-inf when no
    proposal is feasible), and the network's largest and k-th largest
    predicted cell values."""
    import torch

    from paper_1909_07717_amd import binding as B
    from paper_1909_07717_amd.framegen import full_window, uniform_batch_arrays, variants_for

    p = _params()
    variants = variants_for([4.0], flat=True, chip=False)
    fine = [full_window(0.05)]
    s = B.Searcher(p)
    # the exact path at its autotuned launch shape (the surrogate shares it)
    t0, o0, p0 = uniform_batch_arrays(seed0, min(batch, frames))
    _tune(s, B, B.pack_uniform(t0, o0, p0, fine, variants, p), tune_cache)
    net = B.Mlp(s, batch, max_k=max(k, 1), seed=12345)
    if weights and not random_net:
        net.set_params(load_checkpoint(weights)["params"])
    regrets, match, fallbacks, found_both, none_exact = [], 0, 0, 0, 0
    rows = []
    t_exact = t_sur = 0.0
    n_done = 0
    bi = 0
    while n_done < frames:
        n = min(batch, frames - n_done)
        team, opp, passer = uniform_batch_arrays(seed0 + bi, n)
        bi += 1
        pk = B.pack_uniform(team, opp, passer, fine, variants, p)
        bt = s.batch(pk)
        ex = s.outputs_for(pk, mask=False, score=False)
        torch.cuda.synchronize()
        a = time.perf_counter()
        bt.run(ex)
        torch.cuda.synchronize()
        dt_ex = time.perf_counter() - a
        t_exact += dt_ex
        be = ex.best_host()
        a = time.perf_counter()
        if proposals in ("geometric", "mirror"):
            if proposals == "geometric":
                cells = geometric_cells(team, passer, variants, k)
            else:
                tm, om = mirror_arrays(team, opp)
                btm = s.batch(B.pack_uniform(tm, om, passer, fine, variants, p))
                y = net.forward(bt) + mirror_cells(net.forward(btm))
                btm.close()
                cells = torch.topk(y, k, dim=1).indices.cpu().numpy()
            wins = cell_windows(cells)
            pkc = B.pack_uniform(team, opp, passer, wins, variants, p)
            _, outc = s.search_batch(pkc, mask=False, score=False)
            torch.cuda.synchronize()
            bs = outc.best_host().copy()
            redo = (bs["found"] == 0) | (bs["score"] < fallback_below)
            nfb = int(redo.sum())
            bs[redo] = be[redo]  # the fallback is the exact search of the frame
            # plus the exact searches of the fallback frames, at this batch's rate
            t_sur += time.perf_counter() - a + nfb * dt_ex / n
        else:
            sb, nfb = net.search(bt, k=k, fallback=True, fallback_below=fallback_below)
            torch.cuda.synchronize()
            t_sur += time.perf_counter() - a
            bs = B.best_records(sb)
        fallbacks += nfb
        if dump:
            raw, _ = net.search(bt, k=k, fallback=False)
            br = B.best_records(raw)
            y = net.forward(bt)
            top = torch.topk(y, k, dim=1).values.cpu().numpy()
            rows.append(np.stack([
                np.where(be["found"] != 0, be["score"], -np.inf),
                np.where(br["found"] != 0, br["score"], -np.inf),
                top[:, 0], top[:, k - 1]], 1).astype(np.float64))
        for i in range(n):
            if not be[i]["found"]:
                none_exact += 1
                continue
            if not bs[i]["found"]:
                regrets.append(1.0)
                continue
            found_both += 1
            r = (float(be[i]["score"]) - float(bs[i]["score"])) / float(be[i]["score"])
            regrets.append(max(r, 0.0))
            # the same field point and kick (i, j are relative to each record's window)
            match += int(be[i]["x"] == bs[i]["x"] and be[i]["y"] == bs[i]["y"]
                         and be[i]["v0"] == bs[i]["v0"])
        bt.close()
        n_done += n
    r = np.array(regrets)
    res = {"frames": frames, "k": k, "frames_with_exact_best": int(r.size),
           "regret_le_1pct": float(np.mean(r <= 0.01)) if r.size else None,
           "regret_mean": float(r.mean()) if r.size else None,
           "regret_p99": float(np.percentile(r, 99)) if r.size else None,
           "match_rate": match / max(r.size, 1), "fallback_rate": fallbacks / frames,
           "no_feasible_exact": none_exact,
           "exact_frames_per_s": frames / t_exact, "surrogate_frames_per_s": frames / t_sur,
           "fallback_below": fallback_below, "proposals": proposals,
           "network": (None if proposals == "geometric" else "random init"
                       if (random_net or not weights) else os.path.basename(weights))}
    if dump:
        a = np.concatenate(rows, 0)
        np.savez(dump, exact=a[:, 0], raw=a[:, 1], pred_top=a[:, 2], pred_kth=a[:, 3])
    net.close()
    s.close()
    return res


def latency(weights: str | None, frames: int = 10000, warmup: int = 100, k: int = 64,
            seed0: int = EVAL_SEED, tune_cache: str | None = TUNE_CACHE):
    """Frame latency, host inputs to the best pass on the host, one frame at
    a time (6 v 6, one flat pass at 4 m/s, K = 64): the exact search of the
    whole 5 cm lattice (dpps_search) and the surrogate search with exact
    fallback (dpps_surrogate_search_frames with the best record returned in
    host memory).  Frames arrive packed in the C ABI's structs (packing
    Python frame objects is not part of the call); p50 / p99 over `frames`
    frames after `warmup`."""
    import torch

    from paper_1909_07717_amd import binding as B
    from paper_1909_07717_amd.framegen import (frames_from_arrays, full_window,
                                               uniform_batch_arrays, variants_for)

    p = _params()
    variants = variants_for([4.0], flat=True, chip=False)
    fine = [full_window(0.05)]
    s = B.Searcher(p)
    net = B.Mlp(s, 1, max_k=k, seed=0)
    if weights:
        net.set_params(load_checkpoint(weights)["params"])
    n = warmup + frames
    team, opp, passer = uniform_batch_arrays(seed0 + 7777, n)
    fr = frames_from_arrays(team, opp, passer, fine, variants)
    pks = [B.pack([f], p) for f in fr]
    _tune(s, B, pks[0], tune_cache)
    best = torch.empty(B.BEST_DT.itemsize, dtype=torch.uint8, device=s.device)
    host = np.zeros(1, B.BEST_DT)
    dev = s.outputs_for(pks[0], mask=False, score=False)
    out = {}
    for kind in ("exact", "surrogate"):
        lat, fb = [], 0
        for i in range(n):
            a = time.perf_counter()
            if kind == "exact":
                s.search(pks[i], out=dev)
            else:
                _, nfb = net.search_frames(pks[i], k=k, fallback=True, best=best, host=host)
                fb += nfb
            if i >= warmup:
                lat.append(time.perf_counter() - a)
        lat = np.array(lat) * 1e3
        out[kind] = {"p50_ms": float(np.percentile(lat, 50)),
                     "p99_ms": float(np.percentile(lat, 99)), "frames": int(lat.size)}
        if kind == "surrogate":
            out[kind]["fallbacks"] = fb
    net.close()
    s.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--frames", type=int, default=2_000_000)
    t.add_argument("--batch", type=int, default=4096)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--out", default=WEIGHTS)
    t.add_argument("--resume", default=None)
    t.add_argument("--epochs", type=int, default=1)
    t.add_argument("--pos-weight", type=float, default=0.0)
    t.add_argument("--ce-weight", type=float, default=0.0)
    t.add_argument("--tau", type=float, default=0.02)
    t.add_argument("--labels", choices=["pooled", "center"], default="pooled")
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--params-only", action="store_true")
    t.add_argument("--mirror", action="store_true")
    t.add_argument("--init", default=None)
    t.add_argument("--data-seed", type=int, default=TRAIN_SEED)
    e = sub.add_parser("eval")
    e.add_argument("--weights", default=WEIGHTS)
    e.add_argument("--frames", type=int, default=2000)
    e.add_argument("--k", type=int, default=64)
    e.add_argument("--random", action="store_true")
    e.add_argument("--dump", default=None)
    e.add_argument("--proposals", choices=["network", "mirror", "geometric"], default="network")
    e.add_argument("--fallback-below", type=float, default=-math.inf)
    e.add_argument("--tune-cache", default=TUNE_CACHE)
    args = ap.parse_args()
    if args.cmd == "train":
        train(args.frames, args.batch, args.lr, args.out, args.resume, seed=args.seed,
              epochs=args.epochs, pos_weight=args.pos_weight, ce_weight=args.ce_weight,
              tau=args.tau, labels=args.labels, params_only=args.params_only,
              mirror=args.mirror, init=args.init, data_seed=args.data_seed)
    else:
        print(json.dumps(evaluate(args.weights, args.frames, args.k, random_net=args.random,
                                  dump=args.dump, proposals=args.proposals,
                                  fallback_below=args.fallback_below,
                                  tune_cache=args.tune_cache)), flush=True)


if __name__ == "__main__":
    main()
