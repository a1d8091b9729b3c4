"""The batched workload at full size: 4096 frames with 6-8 robots a side,
random windows on the 5 cm lattice (uneven point counts), 8 flat speeds,
K = 128, in one persistent launch with the autotuned shape, replayed from a
HIP graph.  Checked against the oracle on sampled frames and points, and
bitwise against the default launch shape."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1909_07717_amd.framegen import Params, config_batch
from tests.parity import compare_maps

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_full_batch_autotuned_graph(tmp_path):
    from paper_1909_07717_amd import binding as B
    p = Params(n_samples=128).as_f32()
    print("[batch] generating 4096 frames", flush=True)
    frames = config_batch(0, n_frames=4096)
    s = B.Searcher(p)
    bt = s.batch(frames)
    assert bt.points == sum(f.n_points() for f in frames)
    ref = s.outputs_for(bt.pk)
    st = torch.cuda.Stream()
    print(f"[batch] default launch {s.get_launch()}, {bt.points} points", flush=True)
    with torch.cuda.stream(st):
        bt.run(ref, stream=st)
    st.synchronize()
    cache = str(tmp_path / "tune.jsonl")
    out = s.outputs_for(bt.pk)
    ms = bt.autotune(out, cache, reps=1, stream=st)
    shape = s.get_launch()
    print(f"[batch] autotuned {shape} {ms:.3f} ms", flush=True)
    assert ms > 0
    assert bt.autotune(out, cache, reps=1, stream=st) == -1.0 and s.get_launch() == shape
    for rep in range(2):
        with torch.cuda.stream(st):
            out.score.fill_(3.0)
            bt.run(out, stream=st, graph=True)
        st.synchronize()
        assert torch.equal(out.mask, ref.mask) and torch.equal(out.score, ref.score), rep
        assert torch.equal(out.best, ref.best), rep
    bests = out.best_host()
    rng = np.random.default_rng(1)
    for fi in sorted(rng.choice(len(frames), 12, replace=False)):
        f = frames[fi]
        a = int(bt.pk.frames["out_off"][fi])
        win = f.windows[0]
        npts = win[3] * win[4]
        idx = np.sort(rng.choice(npts, min(npts, 40), replace=False))
        V = len(f.variants)
        sel = torch.as_tensor((a + np.arange(V)[None, :] * npts + idx[:, None]).reshape(-1),
                              device=out.mask.device)
        g = dict(mask=out.mask[sel].cpu().numpy().reshape(-1, V),
                 score=out.score[sel].cpu().numpy().reshape(-1, V))
        o = O.search_points(f, p, O.points_of_window(p, win)[idx], bands=True)
        compare_maps(g, o, f"batch frame {fi}")
        # the frame's best equals the argmax of its own score map
        sc = out.score[a:a + npts * V]
        if bests[fi]["found"]:
            e = int(torch.argmax(sc).item())
            assert float(sc[e].item()) == float(bests[fi]["score"])
            assert e == bests[fi]["variant"] * npts + bests[fi]["j"] * win[3] + bests[fi]["i"]
        else:
            assert not torch.isfinite(sc).any()
    bt.close()
    s.close()
