"""Continuous-batching serving loop for the passing-point search.

Simulated matches issue one search request per tick (60 Hz each, phases
staggered); requests carry the match's current robot states, a candidate grid
(20 / 10 / 5 cm, whole field) and 4-16 flat kick speeds.  The loop:

* keeps S slots, each an independent executor with its own HIP stream (one
  library context per slot), so batches admitted to different slots overlap
  on the device;
* whenever a slot is free, admits the requests that have arrived (oldest
  first) into one batch, up to `max_batch` requests and the device-memory
  budget of the slot (the library's own arena estimate for the request);
* polls slot completion without blocking, hands the results back and records
  the latency from the request's arrival to its result on the host.

Executors: `ExactExecutor` (dpps_search_batch), `SurrogateExecutor` (network
proposals re-scored exactly; a frame with no feasible proposal goes back to
the queue as an exact follow-up request) and `MockExecutor` (CPU, injected
delays) for the scheduler's own tests.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from paper_1909_07717_amd.framegen import (FLAT, Frame, Params, full_window, speeds_linear,
                                           variants_for)

TICK = 1.0 / 60.0
GRIDS = (0.2, 0.1, 0.05)


# ---------------------------------------------------------------------------
# workload: matches with random-walk robots
# ---------------------------------------------------------------------------

class MatchSim:
    """n_matches matches; each robot's acceleration per axis per tick is
    N(0, accel_sd) (m/s^2), speed capped at vmax, positions reflected at the
    field edges.  One numpy Generator per simulator (seeded)."""

    def __init__(self, n_matches: int = 64, seed: int = 0, params: Params = Params(),
                 accel_sd: float = 3.0):
        self.p = params
        self.rng = np.random.default_rng(seed)
        self.accel_sd = accel_sd
        self.n = n_matches
        hl, hw = params.field_len / 2, params.field_wid / 2
        self.n_team = self.rng.integers(6, 9, n_matches)
        self.n_opp = self.rng.integers(6, 9, n_matches)
        self.state = []
        for m in range(n_matches):
            k = int(self.n_team[m] + self.n_opp[m])
            pos = np.stack([self.rng.uniform(-hl, hl, k), self.rng.uniform(-hw, hw, k)], 1)
            vel = np.zeros((k, 2))
            self.state.append(np.concatenate([pos, vel], 1))
        self.phase = self.rng.uniform(0.0, TICK, n_matches)
        self.ticks = np.zeros(n_matches, np.int64)

    def step(self, m: int):
        s = self.state[m]
        hl, hw = self.p.field_len / 2, self.p.field_wid / 2
        acc = self.rng.normal(0.0, self.accel_sd, (s.shape[0], 2))
        v = s[:, 2:] + acc * TICK
        sp = np.linalg.norm(v, axis=1, keepdims=True)
        v = np.where(sp > self.p.vmax, v * (self.p.vmax / np.maximum(sp, 1e-12)), v)
        x = s[:, :2] + v * TICK
        for a, lim in ((0, hl), (1, hw)):
            hi = x[:, a] > lim
            lo = x[:, a] < -lim
            x[hi, a] = 2 * lim - x[hi, a]
            x[lo, a] = -2 * lim - x[lo, a]
            v[hi | lo, a] *= -1
        s[:, :2], s[:, 2:] = x, v
        self.ticks[m] += 1

    def request_frame(self, m: int) -> Frame:
        """The match's current state as a request: a random passer, a random
        grid and 4-16 flat speeds."""
        s = self.state[m].astype(np.float32)
        nt = int(self.n_team[m])
        passer = int(self.rng.integers(0, nt))
        h = float(GRIDS[int(self.rng.integers(0, len(GRIDS)))])
        nv = int(self.rng.integers(4, 17))
        team, opp = s[:nt].copy(), s[nt:].copy()
        return Frame(team, opp, passer, team[passer, :2].copy(), [full_window(h)],
                     variants_for(speeds_linear(nv), flat=True, chip=False))


@dataclass(order=True)
class Request:
    arrival: float
    rid: int = field(compare=False)
    match: int = field(compare=False)
    frame: Frame = field(compare=False, repr=False)
    kind: str = field(default="primary", compare=False)
    result: object = field(default=None, compare=False, repr=False)
    done: float = field(default=math.nan, compare=False)
    slot: int = field(default=-1, compare=False)


def request_schedule(sim: MatchSim, duration: float):
    """All requests of `duration` seconds of play, in arrival order."""
    ev = []
    rid = 0
    for m in range(sim.n):
        t = sim.phase[m]
        while t < duration:
            ev.append((t, m))
            t += TICK
    ev.sort()
    reqs = []
    for t, m in ev:
        sim.step(m)
        reqs.append(Request(float(t), rid, m, sim.request_frame(m)))
        rid += 1
    return reqs


# ---------------------------------------------------------------------------
# executors
# ---------------------------------------------------------------------------

def request_bytes(frame: Frame, tile_points: int = 8) -> int:
    """Device bytes a request needs in a slot (tables, tile records, best):
    mirrors the library's arena layout closely enough for admission."""
    pts = frame.n_points()
    tiles = sum(math.ceil(w[3] * w[4] / tile_points) for w in frame.windows)
    return (48 + 16 * (frame.n_team + frame.n_opp) + 40 * len(frame.windows)
            + 8 * len(frame.variants) + 24 * tiles + 56 + 0 * pts)


class MockExecutor:
    """CPU stand-in: a batch 'runs' for fixed + per-request time and returns
    the request ids; used to test the scheduler."""

    def __init__(self, fixed_s=1e-4, per_req_s=2e-5, budget=1 << 40):
        self.fixed_s, self.per_req_s, self.budget = fixed_s, per_req_s, budget
        self.busy_until = None
        self.batch = None
        self.history = []

    def start(self, batch, now):
        self.batch = batch
        self.busy_until = now + self.fixed_s + self.per_req_s * len(batch)
        self.history.append((now, [r.rid for r in batch]))

    def poll(self, now):
        if self.batch is None or now < self.busy_until:
            return None
        out = [(r, {"found": 1, "rid": r.rid}) for r in self.batch]
        self.batch = None
        return out

    @property
    def idle(self):
        return self.batch is None


class ExactExecutor:
    """One library context and stream; dpps_search_batch, best records only."""

    def __init__(self, params: Params, budget: int = 1 << 34, device: int = 0):
        import torch

        from paper_1909_07717_amd import binding as B
        self.B = B
        self.torch = torch
        self.stream = torch.cuda.Stream()
        self.s = B.Searcher(params, device=device, budget=budget, stream=self.stream)
        self.budget = budget
        self.batch = None
        self.event = None
        self.out = None
        self.host = None

    def start(self, batch, now):
        B, torch = self.B, self.torch
        frames = [r.frame for r in batch]
        pk = B.pack(frames, self.s.params)
        n = len(frames)
        self.out = B.DeviceOutputs(0, n, self.s.device, mask=False, score=False)
        self.host = torch.empty(n * B.BEST_DT.itemsize, dtype=torch.uint8, pin_memory=True)
        self.s.search_batch(pk, out=self.out, stream=self.stream)
        with torch.cuda.stream(self.stream):
            self.host.copy_(self.out.best, non_blocking=True)
            self.event = torch.cuda.Event()
            self.event.record(self.stream)
        self.batch = batch

    def poll(self, now):
        if self.batch is None or not self.event.query():
            return None
        recs = np.frombuffer(self.host.numpy().tobytes(), self.B.BEST_DT)
        out = [(r, recs[i].copy()) for i, r in enumerate(self.batch)]
        self.batch = None
        return out

    @property
    def idle(self):
        return self.batch is None

    def close(self):
        self.s.close()


class SurrogateExecutor(ExactExecutor):
    """Network proposals re-scored exactly (5 cm).  A primary request whose
    proposals are all infeasible is returned as None, and the loop re-queues
    it as a follow-up, which this executor then serves with the exact search
    (in the same launch sequence as the next batch's proposals)."""

    def __init__(self, params: Params, weights: str | None, max_batch: int, budget: int = 1 << 34,
                 k: int = 64, device: int = 0):
        super().__init__(params, budget, device)
        self.k = k
        self.net = self.B.Mlp(self.s, max_batch, max_k=k, seed=0)
        if weights:
            from paper_1909_07717_amd.surrogate import load_checkpoint
            self.net.set_params(load_checkpoint(weights)["params"])
        self.n_primary = 0

    def start(self, batch, now):
        B, torch = self.B, self.torch
        prim = [r for r in batch if r.kind != "followup"]
        foll = [r for r in batch if r.kind == "followup"]
        ordered = prim + foll
        n = len(ordered)
        self.host = torch.empty(n * B.BEST_DT.itemsize, dtype=torch.uint8, pin_memory=True)
        sz = B.BEST_DT.itemsize
        with torch.cuda.stream(self.stream):
            if prim:
                best, _ = self.net.search_frames(B.pack([r.frame for r in prim], self.s.params),
                                                 k=self.k, fallback=False, stream=self.stream)
                self.host[:len(prim) * sz].copy_(best, non_blocking=True)
            if foll:
                pk = B.pack([r.frame for r in foll], self.s.params)
                self.out = B.DeviceOutputs(0, len(foll), self.s.device, mask=False, score=False)
                self.s.search_batch(pk, out=self.out, stream=self.stream)
                self.host[len(prim) * sz:].copy_(self.out.best, non_blocking=True)
            self.event = torch.cuda.Event()
            self.event.record(self.stream)
        self.n_primary = len(prim)
        self.batch = ordered

    def poll(self, now):
        out = super().poll(now)
        if out is None:
            return None
        return [(r, rec if (rec["found"] or i >= self.n_primary) else None)
                for i, (r, rec) in enumerate(out)]

    def close(self):
        self.net.close()
        super().close()


# ---------------------------------------------------------------------------
# the loop
# ---------------------------------------------------------------------------

class Scheduler:
    """Continuous batching over executors (slots)."""

    def __init__(self, slots, max_batch: int = 64, fallback_executor_index=None):
        self.slots = list(slots)
        self.max_batch = max_batch
        self.queue = deque()
        self.done = []
        self.inflight_bytes = [0] * len(self.slots)
        self.admitted = set()
        self.followups = 0
        self.max_queue = 0

    def _admit(self, si, now):
        ex = self.slots[si]
        batch, used = [], 0
        while self.queue and len(batch) < self.max_batch:
            r = self.queue[0]
            b = request_bytes(r.frame)
            if b > ex.budget:
                # can never fit: fail it rather than block the queue
                self.queue.popleft()
                r.result, r.done = "budget", now
                self.done.append(r)
                continue
            if used + b > ex.budget:
                break
            self.queue.popleft()
            assert r.rid not in self.admitted or r.kind == "followup"
            self.admitted.add(r.rid)
            r.slot = si
            batch.append(r)
            used += b
        if batch:
            self.inflight_bytes[si] = used
            ex.start(batch, now)

    def run(self, requests, clock=None, sleep=None, realtime=True, horizon=None):
        """Serve `requests` (sorted by arrival).  With realtime, arrivals follow
        the wall clock from the start; otherwise a virtual clock jumps to the
        next event (for mock executors)."""
        reqs = sorted(requests)
        clock = clock or time.perf_counter
        t0 = clock()
        nxt = 0
        pending = len(reqs)
        virtual = 0.0
        while pending > 0:
            now = (clock() - t0) if realtime else virtual
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                self.queue.append(reqs[nxt])
                nxt += 1
            self.max_queue = max(self.max_queue, len(self.queue))
            for si, ex in enumerate(self.slots):
                res = ex.poll(now)
                if res is None:
                    continue
                self.inflight_bytes[si] = 0
                for r, out in res:
                    if out is None:
                        # no feasible proposal: back to the queue for the exact path
                        f = Request(r.arrival, r.rid, r.match, r.frame, "followup")
                        self.followups += 1
                        self.queue.appendleft(f)
                        continue
                    r.result, r.done = out, now
                    self.done.append(r)
                    pending -= 1
            for si, ex in enumerate(self.slots):
                if ex.idle and self.queue:
                    self._admit(si, now)
            if not realtime:
                cand = [reqs[nxt].arrival] if nxt < len(reqs) else []
                cand += [ex.busy_until for ex in self.slots if not ex.idle]
                if not cand:
                    break
                virtual = max(virtual, min(cand))
            elif sleep:
                sleep()
            if horizon is not None and now > horizon:
                break
        return self.done


def latency_stats(done):
    lat = np.array([(r.done - r.arrival) * 1e3 for r in done if isinstance(r.done, float)
                    and not math.isnan(r.done)])
    if lat.size == 0:
        return {"n": 0}
    return {"n": int(lat.size), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "max_ms": float(lat.max())}


def run_serving(kind: str = "exact", duration: float = 1.0, n_matches: int = 64, slots: int = 4,
                max_batch: int = 64, weights: str | None = None, seed: int = 0,
                budget: int = 1 << 34, params: Params | None = None):
    """Serve `duration` seconds of `n_matches` simulated matches on the GPU in
    real time; returns (stats, done requests)."""
    import torch

    p = params or Params(n_samples=128).as_f32()
    reqs = request_schedule(MatchSim(n_matches, seed=seed), duration)
    if kind == "exact":
        ex = [ExactExecutor(p, budget) for _ in range(slots)]
    else:
        ex = [SurrogateExecutor(p, weights, max_batch, budget) for _ in range(slots)]
    # warm every slot once (first launches compile nothing but allocate)
    warm = Scheduler(ex, max_batch=max_batch)
    warm.run([Request(0.0, -1 - i, 0, reqs[i].frame) for i in range(min(slots, len(reqs)))],
             realtime=True)
    torch.cuda.synchronize()
    sch = Scheduler(ex, max_batch=max_batch)
    t0 = time.perf_counter()
    done = sch.run(reqs, realtime=True)
    wall = time.perf_counter() - t0
    st = latency_stats(done)
    st.update({"kind": kind, "requests": len(reqs), "wall_s": wall, "duration_s": duration,
               "frames_per_s": len(done) / wall, "offered_per_s": len(reqs) / duration,
               "slots": slots, "max_batch": max_batch, "followups": sch.followups,
               "max_queue": sch.max_queue,
               "evals": int(sum(r.frame.n_evals() for r in reqs))})
    for e in ex:
        e.close()
    return st, done
