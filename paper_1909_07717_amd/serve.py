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
proposals re-scored exactly, with the exact fallback on the device) and
`MockExecutor` (CPU, injected delays) for the scheduler's own tests.  An
executor may also hand a request back (result None) to be queued again as an
exact follow-up.
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
    nbytes: int = field(default=-1, compare=False)  # device bytes (admission)


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
        f = sim.request_frame(m)
        reqs.append(Request(float(t), rid, m, f, nbytes=request_bytes(f, sim.p)))
        rid += 1
    return reqs


# ---------------------------------------------------------------------------
# executors
# ---------------------------------------------------------------------------

# bytes of one best record (dpps_best), the only output a served request writes
BEST_BYTES = 56


def request_bytes(frame: Frame, params: Params = Params(), tile_points: int = 8) -> int:
    """Device bytes a request needs in a slot: the search library's own
    figure for its tables, tile records and best record (dpps_request_bytes),
    plus the record the executor writes out for it."""
    from paper_1909_07717_amd import binding as B
    return B.request_bytes(B.pack([frame], params.as_f32()), params.as_f32(), tile_points) + BEST_BYTES


def library_budget(slot_budget: int) -> int:
    """The search context's own device-memory cap for a slot that admits up
    to slot_budget bytes of requests at once: its memory may grow a quarter
    beyond the largest request and round up to 64 KiB in each of its two
    regions, so the cap is a backstop the admitted batches never reach."""
    return int(slot_budget * 1.25) + (1 << 18)


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
    """One library context and stream; dpps_search_batch, best records only.
    The device best records, their pinned host copy and the completion event
    are allocated once for max_batch requests."""

    def __init__(self, params: Params, budget: int = 1 << 26, device: int = 0,
                 max_batch: int = 64, library_cap: bool = True):
        import torch

        from paper_1909_07717_amd import binding as B
        self.B = B
        self.torch = torch
        self.stream = torch.cuda.Stream()
        self.s = B.Searcher(params, device=device,
                            budget=library_budget(budget) if library_cap else 0,
                            stream=self.stream)
        self.budget = budget
        self.max_batch = max_batch
        self.batch = None
        self.sz = B.BEST_DT.itemsize
        self.out = B.DeviceOutputs(0, max_batch, self.s.device, mask=False, score=False)
        self.host = torch.empty(max_batch * self.sz, dtype=torch.uint8, pin_memory=True)
        self.event = torch.cuda.Event()

    def start(self, batch, now):
        torch = self.torch
        n = len(batch)
        assert n <= self.max_batch
        pk = self.B.pack([r.frame for r in batch], self.s.params)
        self.s.search_batch(pk, out=self.out, stream=self.stream)
        with torch.cuda.stream(self.stream):
            self.host[:n * self.sz].copy_(self.out.best[:n * self.sz], non_blocking=True)
            self.event.record(self.stream)
        self.batch = batch

    def poll(self, now):
        if self.batch is None or not self.event.query():
            return None
        n = len(self.batch)
        recs = np.frombuffer(self.host[:n * self.sz].numpy().tobytes(), self.B.BEST_DT)
        out = [(r, recs[i].copy()) for i, r in enumerate(self.batch)]
        self.batch = None
        return out

    @property
    def idle(self):
        return self.batch is None

    def device_bytes(self) -> int:
        return self.s.device_bytes()

    def close(self):
        self.s.close()


class SurrogateExecutor(ExactExecutor):
    """Network proposals re-scored exactly (5 cm); a frame whose proposals
    are all infeasible takes the exact search of its whole 5 cm lattice in
    the same launch sequence (picked on the device, no host round trip)."""

    def __init__(self, params: Params, weights: str | None, max_batch: int, budget: int = 1 << 26,
                 k: int = 64, device: int = 0):
        # the network's memory counts against the context, not the slot
        super().__init__(params, budget, device, max_batch, library_cap=False)
        self.k = k
        self.net = self.B.Mlp(self.s, max_batch, max_k=k, seed=0)
        if weights:
            from paper_1909_07717_amd.surrogate import load_checkpoint
            self.net.set_params(load_checkpoint(weights)["params"])
        self.prop = self.torch.empty(max_batch * self.sz, dtype=self.torch.uint8,
                                     device=self.s.device)

    def start(self, batch, now):
        B, torch = self.B, self.torch
        n, sz = len(batch), self.sz
        assert n <= self.max_batch
        with torch.cuda.stream(self.stream):
            self.net.search_frames(B.pack([r.frame for r in batch], self.s.params), k=self.k,
                                   fallback=True, best=self.prop[:n * sz], stream=self.stream,
                                   count=False)
            self.host[:n * sz].copy_(self.prop[:n * sz], non_blocking=True)
            self.event.record(self.stream)
        self.batch = batch

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
        self.budget_cuts = 0      # batches closed by the budget with requests waiting
        self.batches = []         # (slot, requests, admitted bytes) of every batch

    def _admit(self, si, now):
        ex = self.slots[si]
        batch, used = [], 0
        while self.queue and len(batch) < self.max_batch:
            r = self.queue[0]
            b = r.nbytes if r.nbytes >= 0 else request_bytes(r.frame)
            if b > ex.budget:
                # can never fit: fail it rather than block the queue
                self.queue.popleft()
                r.result, r.done = "budget", now
                self.done.append(r)
                continue
            if used + b > ex.budget:
                self.budget_cuts += 1
                break
            self.queue.popleft()
            assert r.rid not in self.admitted or r.kind == "followup"
            self.admitted.add(r.rid)
            r.slot = si
            batch.append(r)
            used += b
        if batch:
            self.inflight_bytes[si] = used
            self.batches.append((si, len(batch), used))
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
                        f = Request(r.arrival, r.rid, r.match, r.frame, "followup",
                                    nbytes=r.nbytes)
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


def warm_batch(sim_params: Params, n: int, budget: int):
    """Requests of the largest kind (5 cm whole field, 16 speeds, 8v8) that a
    slot admits at once: serving them first grows every slot's memory to
    what any later batch needs, so no allocation happens while serving."""
    from paper_1909_07717_amd.framegen import random_frame
    f = random_frame(np.random.default_rng(12345), 8, 8)
    f.windows = [full_window(0.05)]
    f.variants = variants_for(speeds_linear(16), flat=True, chip=False)
    b = request_bytes(f, sim_params)
    k = max(1, min(n, budget // b))
    return [Request(0.0, -1 - i, 0, f, nbytes=b) for i in range(k)]


def run_serving(kind: str = "exact", duration: float = 1.0, n_matches: int = 64, slots: int = 4,
                max_batch: int = 64, weights: str | None = None, seed: int = 0,
                budget: int = 1 << 26, params: Params | None = None):
    """Serve `duration` seconds of `n_matches` simulated matches on the GPU in
    real time; returns (stats, done requests, scheduler).  `budget` is each
    slot's device-memory budget for the requests it holds at once."""
    import torch

    p = params or Params(n_samples=128).as_f32()
    reqs = request_schedule(MatchSim(n_matches, seed=seed, params=p), duration)
    if kind == "exact":
        ex = [ExactExecutor(p, budget, max_batch=max_batch) for _ in range(slots)]
    else:
        ex = [SurrogateExecutor(p, weights, max_batch, budget) for _ in range(slots)]
    # warm every slot with its largest admissible batch (device memory grows
    # here, not while serving)
    for e in ex:
        e.start(warm_batch(p, max_batch, budget), 0.0)
        while e.poll(0.0) is None:
            pass
    torch.cuda.synchronize()
    sch = Scheduler(ex, max_batch=max_batch)
    t0 = time.perf_counter()
    done = sch.run(reqs, realtime=True)
    wall = time.perf_counter() - t0
    st = latency_stats(done)
    st.update({"kind": kind, "requests": len(reqs), "wall_s": wall, "duration_s": duration,
               "frames_per_s": len(done) / wall, "offered_per_s": len(reqs) / duration,
               "slots": slots, "max_batch": max_batch, "followups": sch.followups,
               "max_queue": sch.max_queue, "budget_bytes": budget,
               "budget_cuts": sch.budget_cuts, "batches": len(sch.batches),
               "max_batch_bytes": max((b for _, _, b in sch.batches), default=0),
               "slot_device_bytes": [e.device_bytes() for e in ex],
               "evals": int(sum(r.frame.n_evals() for r in reqs))})
    for e in ex:
        e.close()
    return st, done, sch
