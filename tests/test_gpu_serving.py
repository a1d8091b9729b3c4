"""Serving on the GPU: results in the continuous-batching mix equal the same
requests searched alone (exact path bitwise; the surrogate path bitwise as
well, its network and re-score being per-frame computations)."""
import numpy as np
import pytest

from paper_1909_07717_amd.framegen import Params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["exact", "surrogate"])
def test_alone_equals_mix(kind):
    from paper_1909_07717_amd import binding as B
    from paper_1909_07717_amd.serve import run_serving
    p = Params(n_samples=128).as_f32()
    print(f"[serve] {kind}", flush=True)
    st, done = run_serving(kind, duration=0.25, n_matches=16, slots=3, max_batch=16, params=p)
    print(f"[serve] {st}", flush=True)
    assert st["n"] == st["requests"]
    s = B.Searcher(p)
    net = None
    if kind == "surrogate":
        net = B.Mlp(s, 1, seed=0)
    rng = np.random.default_rng(0)
    for r in [done[i] for i in rng.choice(len(done), 24, replace=False)]:
        if kind == "exact" or r.kind == "followup":
            _, alone = s.search(r.frame)
        else:
            bt = s.batch([r.frame])
            best, _ = net.search(bt, k=64, fallback=False)
            alone = B.best_records(best)[0]
            bt.close()
        assert np.asarray(r.result).tobytes() == alone.tobytes(), (kind, r.rid)
    if net:
        net.close()
    s.close()
