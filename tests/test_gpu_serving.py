"""Serving on the GPU.

* Results in the continuous-batching mix equal the same requests searched
  alone (exact path bitwise; the surrogate path, exact fallback included,
  bitwise as well, its network and re-score being per-frame computations).
* Served exact results are the oracle's best pass (Sec. 4.2-4.3 search) on
  sampled 20 cm and 10 cm requests; served surrogate results are feasible in
  the oracle with the reported score.
* A slot budget that binds: batches are cut by it, never exceed it, every
  request is still served, and the contexts' memory stays within the
  library cap derived from the budget.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1909_07717_amd.framegen import Params
from tests.parity import S_FLOOR, S_REL, check_best

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _serve(kind, n_matches=16, slots=3, **kw):
    from paper_1909_07717_amd.serve import run_serving
    p = Params(n_samples=128).as_f32()
    print(f"[serve] {kind} {kw}", flush=True)
    st, done, sch = run_serving(kind, duration=0.25, n_matches=n_matches, slots=slots, max_batch=16,
                                params=p, **kw)
    print(f"[serve] {st}", flush=True)
    assert st["n"] == st["requests"]
    return p, st, done, sch


def _elem(frame, best):
    win = frame.windows[0]
    return best["variant"] * win[3] * win[4] + best["j"] * win[3] + best["i"]


@pytest.mark.parametrize("kind", ["exact", "surrogate"])
def test_alone_equals_mix(kind):
    from paper_1909_07717_amd import binding as B
    p, st, done, _ = _serve(kind)
    s = B.Searcher(p)
    net = None
    if kind == "surrogate":
        net = B.Mlp(s, 1, seed=0)
    rng = np.random.default_rng(0)
    for r in [done[i] for i in rng.choice(len(done), 24, replace=False)]:
        if kind == "exact":
            _, alone = s.search(r.frame)
        else:
            bt = s.batch([r.frame])
            best, _ = net.search(bt, k=64, fallback=True)
            alone = B.best_records(best)[0]
            bt.close()
        assert np.asarray(r.result).tobytes() == alone.tobytes(), (kind, r.rid)
    if net:
        net.close()
    s.close()


def test_served_exact_results_are_the_oracle_best():
    p, st, done, _ = _serve("exact")
    rng = np.random.default_rng(1)
    picked = []
    for h, n in ((0.2, 10), (0.1, 6)):
        cand = [r for r in done if abs(r.frame.windows[0][0] - h) < 1e-6]
        picked += [cand[i] for i in rng.choice(len(cand), min(n, len(cand)), replace=False)]
    assert len(picked) >= 16
    for r in picked:
        print(f"[serve] oracle check rid {r.rid} h {r.frame.windows[0][0]:.2f}", flush=True)
        o = O.search_frame(r.frame, p, bands=True)
        b = r.result
        check_best(b, o, _elem(r.frame, b) if b["found"] else -1, f"rid {r.rid}")


def test_served_surrogate_results_are_feasible_with_their_score():
    p, st, done, _ = _serve("surrogate")
    rng = np.random.default_rng(2)
    found = [r for r in done if r.result["found"]]
    for r in [found[i] for i in rng.choice(len(found), 16, replace=False)]:
        b = r.result
        f = r.frame.copy()
        f.variants = [r.frame.variants[int(b["variant"])]]
        o = O.search_points(f, p, np.array([[float(b["x"]), float(b["y"])]]), bands=True)
        amb = int(o["ambig"][0, 0]) & 7
        assert o["mask"][0, 0] == 1 or amb, r.rid
        if not amb:
            sc = o["score"][0, 0]
            assert abs(float(b["score"]) - sc) <= S_REL * max(abs(sc), S_FLOOR), (r.rid, b["score"], sc)


def test_a_binding_budget_cuts_batches_and_serves_everything():
    from paper_1909_07717_amd.serve import library_budget, request_bytes
    from paper_1909_07717_amd.framegen import full_window, random_frame, speeds_linear, variants_for
    f = random_frame(np.random.default_rng(0), 8, 8)
    f.windows = [full_window(0.05)]
    f.variants = variants_for(speeds_linear(16), flat=True)
    big = request_bytes(f, Params(n_samples=128))
    budget = 2 * big
    # the full 64-match load on one slot: requests queue while a batch runs,
    # and two of the largest requests fill the budget
    p, st, done, sch = _serve("exact", n_matches=64, slots=1, budget=budget)
    assert st["budget_cuts"] > 0
    assert all(b <= budget for _, _, b in sch.batches)
    assert all(0 < d <= library_budget(budget) for d in st["slot_device_bytes"])
    assert all(isinstance(r.result, np.void) for r in done)
