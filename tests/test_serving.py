"""Serving loop on the CPU: the match simulator and the continuous-batching
scheduler driven by a mock executor on a virtual clock."""
import math

import numpy as np
import pytest

from paper_1909_07717_amd.serve import (TICK, MatchSim, MockExecutor, Request, Scheduler,
                                        latency_stats, request_bytes, request_schedule)
from paper_1909_07717_amd.framegen import Params, config_small


def test_match_sim_is_seeded_and_physical():
    a = request_schedule(MatchSim(8, seed=3), 0.5)
    b = request_schedule(MatchSim(8, seed=3), 0.5)
    assert len(a) == len(b) and all(x.frame.team.tobytes() == y.frame.team.tobytes()
                                    for x, y in zip(a, b))
    # 60 Hz per match
    assert abs(len(a) - 8 * 0.5 / TICK) <= 8
    p = Params()
    for r in a:
        allr = np.concatenate([r.frame.team, r.frame.opp])
        assert np.all(np.abs(allr[:, 0]) <= p.field_len / 2 + 1e-4)
        assert np.all(np.abs(allr[:, 1]) <= p.field_wid / 2 + 1e-4)
        assert np.all(np.hypot(allr[:, 2], allr[:, 3]) <= p.vmax + 1e-4)
        assert 6 <= r.frame.n_team <= 8 and 6 <= r.frame.n_opp <= 8
        assert 4 <= len(r.frame.variants) <= 16
        assert r.frame.windows[0][0] in (np.float32(0.2), np.float32(0.1), np.float32(0.05))
    arr = [r.arrival for r in a]
    assert arr == sorted(arr)


def _run(n_matches=16, duration=0.3, slots=3, max_batch=8, budget=1 << 40, fixed=2e-3, per=1e-4):
    reqs = request_schedule(MatchSim(n_matches, seed=1), duration)
    ex = [MockExecutor(fixed, per, budget) for _ in range(slots)]
    sch = Scheduler(ex, max_batch=max_batch)
    done = sch.run(reqs, realtime=False)
    return reqs, ex, sch, done


def test_every_request_served_once_in_fifo_order():
    reqs, ex, sch, done = _run()
    assert sorted(r.rid for r in done) == sorted(r.rid for r in reqs)
    starts = sorted((t, rids) for e in ex for t, rids in e.history)
    order = [rid for _, rids in starts for rid in rids]
    assert order == sorted(order)           # admitted oldest first
    assert len(order) == len(set(order))    # never twice
    for e in ex:
        for _, rids in e.history:
            assert len(rids) <= 8


def test_budget_is_never_exceeded_and_oversize_fails_alone():
    reqs = request_schedule(MatchSim(12, seed=2), 0.2)
    sizes = {r.rid: request_bytes(r.frame) for r in reqs}
    budget = int(np.percentile(list(sizes.values()), 90) * 2)
    ex = [MockExecutor(1e-3, 1e-4, budget) for _ in range(2)]
    sch = Scheduler(ex, max_batch=16)
    done = sch.run(reqs, realtime=False)
    for e in ex:
        for _, rids in e.history:
            assert sum(sizes[i] for i in rids) <= budget
    failed = [r for r in done if r.result == "budget"]
    assert all(sizes[r.rid] > budget for r in failed)
    assert len(done) == len(reqs)


def test_no_starvation_and_latency_accounting():
    reqs, ex, sch, done = _run(n_matches=32, duration=0.5, slots=2, max_batch=16, fixed=3e-3)
    st = latency_stats(done)
    assert st["n"] == len(reqs)
    lat = np.array([(r.done - r.arrival) for r in done])
    # every request waits at least one batch execution and no more than a
    # few: the service capacity exceeds the arrival rate
    assert lat.min() >= 3e-3 - 1e-12
    assert lat.max() < 0.05
    assert st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]


def test_overload_queues_but_serves_everything():
    # service slower than arrivals: the queue grows, nothing is dropped
    reqs, ex, sch, done = _run(n_matches=32, duration=0.2, slots=1, max_batch=4, fixed=5e-3)
    assert len(done) == len(reqs)
    assert sch.max_queue > 10
    lat = [(r.done - r.arrival) for r in done]
    assert max(lat) > 0.05
