"""The surrogate's kernels through the C ABI against the FP64 reference
(oracle/mlp_ref.py): features, forward pass, loss and parameter gradients
(BF16 operands, FP32 accumulation: relative L2 tolerances), Adam, top-k, the
surrogate search against the exact search on the same windows, the
fallback, and checkpoint/resume determinism of training."""
import numpy as np
import pytest

from oracle import mlp_ref as M
from oracle import oracle as O
from paper_1909_07717_amd.framegen import (Params, Frame, config_small, full_window,
                                           random_frame, variants_for)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P = Params(n_samples=64).as_f32()


@pytest.fixture(scope="module")
def B():
    from paper_1909_07717_amd import binding
    assert torch.cuda.is_available()
    return binding


def _frames(n, base=0):
    return [config_small(base + i) for i in range(n)]


def _labels(B, s, frames):
    """Exact 20 cm score maps of the frames (device, [n][2806])."""
    bt = s.batch(frames)
    out = s.outputs_for(bt.pk, mask=False)
    bt.run(out)
    torch.cuda.synchronize()
    bt.close()
    return out.score.view(len(frames), 2806)


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def test_features(B):
    s = B.Searcher(P)
    frames = _frames(40)
    net = B.Mlp(s, 64)
    bt = s.batch(frames)
    x = net.features(bt).cpu().numpy()
    for i, f in enumerate(frames):
        want = torch.tensor(M.features(f)).to(torch.bfloat16).float().numpy()
        assert np.array_equal(x[i], want), i
    bt.close(); net.close(); s.close()


def test_forward_loss_and_gradients(B):
    s = B.Searcher(P)
    frames = _frames(37, 100)
    net = B.Mlp(s, 64, seed=3)
    bt = s.batch(frames)
    T = _labels(B, s, frames)
    y = net.forward(bt).cpu().numpy()
    w = net.get_params().astype(np.float64)
    X = np.stack([M.features(f) for f in frames])
    Yref, _ = M.forward(w, X)
    e_fwd = _rel_l2(y, Yref)
    kw = dict(pos_weight=4.0, ce_weight=0.05, tau=0.05)
    loss = net.loss_grad(bt, T, **kw)
    g = net.get_grads().astype(np.float64)
    lref, gref = M.loss_and_grad(w, X, T.cpu().numpy(), **kw)
    print(f"[mlp] forward rel L2 {e_fwd:.2e}, loss {loss:.6f} vs {lref:.6f}", flush=True)
    assert e_fwd <= 2e-2
    assert abs(loss - lref) <= 2e-2 * lref
    o = 0
    for l, (r, c) in enumerate(M.DIMS):
        for name, n in (("W", r * c), ("b", r)):
            e = _rel_l2(g[o:o + n], gref[o:o + n])
            print(f"[mlp] grad {name}{l} rel L2 {e:.2e}", flush=True)
            assert e <= 3e-2, (name, l, e)
            o += n
    # one Adam step from these gradients matches the reference update
    net.adam(1e-3)
    w1 = net.get_params().astype(np.float64)
    wref, _, _ = M.adam(w, g, np.zeros_like(w), np.zeros_like(w), 1, 1e-3)
    assert np.max(np.abs(w1 - wref)) <= 1e-6
    m, v, step = net.get_adam()
    assert step == 1
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-6, atol=1e-12)
    bt.close(); net.close(); s.close()


def test_forward_and_gradients_large_batch(B):
    # 2048 frames: the output layer runs on the 128 x 128 tiles and the
    # weight gradients reduce over the batch in split slices
    from paper_1909_07717_amd.framegen import (frames_from_arrays, uniform_batch_arrays,
                                               variants_for)
    s = B.Searcher(P)
    team, opp, passer = uniform_batch_arrays(777, 2048)
    frames = frames_from_arrays(team, opp, passer, [full_window(0.2)],
                                variants_for([4.0], flat=True, chip=False))
    net = B.Mlp(s, 2048, seed=9)
    bt = s.batch(frames)
    T = _labels(B, s, frames)
    y = net.forward(bt).cpu().numpy()
    w = net.get_params().astype(np.float64)
    X = np.stack([M.features(f) for f in frames])
    Yref, _ = M.forward(w, X)
    assert _rel_l2(y, Yref) <= 2e-2
    kw = dict(pos_weight=8.0, ce_weight=0.2, tau=0.02)
    loss = net.loss_grad(bt, T, **kw)
    g = net.get_grads().astype(np.float64)
    lref, gref = M.loss_and_grad(w, X, T.cpu().numpy(), **kw)
    assert abs(loss - lref) <= 2e-2 * lref
    o = 0
    for l, (r, c) in enumerate(M.DIMS):
        for name, n in (("W", r * c), ("b", r)):
            e = _rel_l2(g[o:o + n], gref[o:o + n])
            print(f"[mlp 2048] grad {name}{l} rel L2 {e:.2e}", flush=True)
            assert e <= 3e-2, (name, l, e)
            o += n
    # the split reduction is deterministic
    net.loss_grad(bt, T, **kw)
    assert np.array_equal(net.get_grads(), g.astype(np.float32))
    bt.close(); net.close(); s.close()


def test_pooled_labels(B):
    s = B.Searcher(P)
    frames = _frames(3, 400)
    for f in frames:
        f.windows = [full_window(0.05)]
    bt = s.batch(frames)
    out = s.outputs_for(bt.pk, mask=False)
    bt.run(out)
    c = B.pool_cells(out.score, 241, 181)
    torch.cuda.synchronize()
    want = M.pool(out.score.cpu().numpy())
    assert np.array_equal(c.cpu().numpy().astype(np.float64), want)
    bt.close(); s.close()


def test_topk_matches_sort(B):
    s = B.Searcher(P)
    frames = _frames(20, 200)
    net = B.Mlp(s, 32, seed=5)
    bt = s.batch(frames)
    y = net.forward(bt).cpu().numpy()
    cells = net.topk(len(frames), 64).cpu().numpy()
    for i in range(len(frames)):
        assert list(cells[i]) == list(M.topk(y[i], 64)), i
    bt.close(); net.close(); s.close()


def test_topk_ties_take_the_lower_indices(B):
    # a zero output layer: every frame's map is the bias, 7 levels over 2806
    # cells, so the k-th largest value is shared by hundreds of cells
    s = B.Searcher(P)
    net = B.Mlp(s, 8, max_k=256, seed=5)
    parts = M.split(net.get_params())
    W3, b3 = parts[3]
    rng = np.random.default_rng(9)
    parts[3] = (np.zeros_like(W3), rng.integers(-3, 4, b3.size).astype(np.float64) * 0.25)
    net.set_params(M.join(parts).astype(np.float32))
    frames = _frames(3, 500)
    bt = s.batch(frames)
    y = net.forward(bt).cpu().numpy()
    assert (y == y[0]).all() and np.unique(y[0]).size == 7
    for k in (1, 17, 64, 100, 128, 200, 256):
        cells = net.topk(len(frames), k).cpu().numpy()
        for i in range(len(frames)):
            assert list(cells[i]) == list(M.topk(y[i], k)), (k, i)
    bt.close(); net.close(); s.close()


def test_small_batch_forward_is_bit_identical_to_the_tiled_forward(B):
    # up to 64 frames run through the few-row GEMM, larger batches through
    # the tiled one: the same frames give the same outputs bit for bit
    s = B.Searcher(P)
    net = B.Mlp(s, 80, seed=11)
    frames = _frames(70, 600)
    big = s.batch(frames)
    yb = net.forward(big).cpu().numpy()
    for n in (1, 5, 16, 17, 64):
        small = s.batch(frames[:n])
        ys = net.forward(small).cpu().numpy()
        assert ys.tobytes() == yb[:n].tobytes(), n
        small.close()
    big.close(); net.close(); s.close()


def _windows_of_cells(cells):
    wins = []
    for c in cells:
        ci, cj = int(c) % 61, int(c) // 61
        a0, a1 = max(4 * ci - 2, 0), min(4 * ci + 1, 240)
        b0, b1 = max(4 * cj - 2, 0), min(4 * cj + 1, 180)
        wins.append((float(np.float32(0.05)), a0, b0, a1 - a0 + 1, b1 - b0 + 1))
    return wins


def test_surrogate_search_equals_exact_search_on_its_windows(B):
    s = B.Searcher(P)
    frames = _frames(12, 300)
    net = B.Mlp(s, 16, seed=7)
    bt = s.batch(frames)
    best_t, nfb = net.search(bt, k=64, fallback=False)
    best = B.best_records(best_t)
    net.forward(bt)
    cells = net.topk(len(frames), 64).cpu().numpy()
    for i, f in enumerate(frames):
        g = f.copy()
        g.windows = _windows_of_cells(cells[i])
        _, ref = s.search(g)
        assert best[i].tobytes() == ref.tobytes(), i
    bt.close(); net.close(); s.close()


def test_surrogate_search_of_host_frames_equals_batch_search(B):
    # two calls in a row through the context's own staging (the second
    # smaller), with and without fallback, against batches of the same frames
    s = B.Searcher(P)
    net = B.Mlp(s, 16, seed=5)
    for n, base, fb in ((12, 700, True), (5, 900, False), (9, 1100, True)):
        frames = _frames(n, base)
        host = np.zeros(n, B.BEST_DT)
        got_t, nfb_a = net.search_frames(frames, k=64, fallback=fb, host=host)
        got = B.best_records(got_t).copy()
        # the records returned in host memory are the device ones
        assert host.tobytes() == got.tobytes()
        bt = s.batch(frames)
        ref_t, nfb_b = net.search(bt, k=64, fallback=fb)
        ref = B.best_records(ref_t)
        bt.close()
        assert nfb_a == nfb_b
        assert got.tobytes() == ref.tobytes()
    net.close(); s.close()


def test_single_frames_through_staging_match_batch_search(B):
    # one frame per call through the context's staging, alternating fallback,
    # each against the batch search of the same frame
    s = B.Searcher(P)
    net = B.Mlp(s, 16, seed=7)
    host = np.zeros(1, B.BEST_DT)
    for rep, f in enumerate(_frames(6, 1300)):
        fb = rep % 2 == 0
        got_t, nfb_a = net.search_frames([f], k=64, fallback=fb, host=host)
        torch.cuda.synchronize()
        got = B.best_records(got_t).copy()
        assert host.tobytes() == got.tobytes()
        bt = s.batch([f])
        ref_t, nfb_b = net.search(bt, k=64, fallback=fb)
        torch.cuda.synchronize()
        ref = B.best_records(ref_t)
        bt.close()
        assert nfb_a == nfb_b, rep
        assert got.tobytes() == ref.tobytes(), rep
    net.close(); s.close()


def test_fallback_when_no_proposal_is_feasible(B):
    s = B.Searcher(P)
    net = B.Mlp(s, 8, seed=1)
    net.set_params(np.zeros(net.n, np.float32))  # every cell ties: the first 64 cells win
    # passer at the centre, one teammate far from the bottom edge, opponents
    # lined up along it: every proposal (bottom row) is intercepted
    team = np.array([[0, 0, 0, 0], [3, 3, 0, 0]], np.float32)
    opp = np.array([[x, -3.8, 0, 0] for x in (-5, -3, -1, 1, 3, 5)], np.float32)
    f = Frame(team, opp, 0, np.array([0, 0], np.float32), [full_window(0.2)],
              variants_for([4.0], True, False))
    bt = s.batch([f])
    best_t, nfb = net.search(bt, k=64, fallback=True)
    best = B.best_records(best_t)[0]
    assert nfb == 1
    g = f.copy()
    g.windows = [full_window(0.05)]
    _, ref = s.search(g)
    assert ref["found"] == 1 and best.tobytes() == ref.tobytes()
    bt.close(); net.close(); s.close()


def test_fallback_below_a_score_threshold(B):
    s = B.Searcher(P)
    frames = _frames(12, 500)
    net = B.Mlp(s, 16, seed=3)
    bt = s.batch(frames)
    raw = B.best_records(net.search(bt, k=64, fallback=False)[0]).copy()
    found = raw["found"] != 0
    assert found.any()
    thr = float(np.median(raw["score"][found]))
    got_t, nfb = net.search(bt, k=64, fallback=True, fallback_below=thr)
    got = B.best_records(got_t)
    redo = 0
    for i, f in enumerate(frames):
        if raw[i]["found"] and raw[i]["score"] >= thr:
            assert got[i].tobytes() == raw[i].tobytes(), i
            continue
        redo += 1
        g = f.copy()
        g.windows = [full_window(0.05)]
        _, ref = s.search(g)
        assert got[i].tobytes() == ref.tobytes(), i
    assert nfb == redo and 0 < redo < len(frames)
    with pytest.raises(B.DppsError):
        net.search(bt, k=64, fallback=True, fallback_below=float("nan"))
    bt.close(); net.close(); s.close()


def test_device_fallback_over_several_chunks_of_frames(B):
    """300 frames (two chunks of the device's frame compaction), half of them
    below the threshold: each fallback record equals the exact search of the
    frame's whole 5 cm lattice, the others the raw proposals."""
    s = B.Searcher(P)
    frames = _frames(300, 900)
    net = B.Mlp(s, 320, seed=4)
    bt = s.batch(frames)
    raw = B.best_records(net.search(bt, k=64, fallback=False)[0]).copy()
    found = raw["found"] != 0
    thr = float(np.median(raw["score"][found]))
    got = B.best_records(net.search(bt, k=64, fallback=True, fallback_below=thr)[0])
    fine = []
    for f in frames:
        g = f.copy()
        g.windows = [full_window(0.05)]
        fine.append(g)
    _, ex = s.search_batch(fine, mask=False, score=False)
    torch.cuda.synchronize()
    ref = ex.best_host()
    redo = ~found | (raw["score"] < thr)
    assert 100 < int(redo.sum()) < 200
    for i in range(len(frames)):
        want = ref[i] if redo[i] else raw[i]
        assert got[i].tobytes() == want.tobytes(), i
    # asynchronous call (no fallback count): the same records
    pk = B.pack(frames, P)
    best = torch.empty(len(frames) * B.BEST_DT.itemsize, dtype=torch.uint8, device=s.device)
    _, n = net.search_frames(pk, k=64, fallback=True, fallback_below=thr, best=best, count=False)
    torch.cuda.synchronize()
    assert n == -1 and B.best_records(best).tobytes() == got.tobytes()
    bt.close(); net.close(); s.close()


def test_training_resume_is_deterministic(B):
    s = B.Searcher(P)
    data = [_frames(64, 1000 + 64 * i) for i in range(6)]
    batches = [s.batch(fr) for fr in data]
    labels = [_labels(B, s, fr) for fr in data]
    a = B.Mlp(s, 64, seed=11)
    losses = [a.train_step(batches[i], labels[i], 1e-3) for i in range(6)]
    assert losses[-1] < losses[0]
    b = B.Mlp(s, 64, seed=11)
    for i in range(3):
        b.train_step(batches[i], labels[i], 1e-3)
    w, (m, v, st) = b.get_params(), b.get_adam()
    c = B.Mlp(s, 64, seed=99)
    c.set_params(w)
    c.set_adam(m, v, st)
    for i in range(3, 6):
        c.train_step(batches[i], labels[i], 1e-3)
    assert np.array_equal(c.get_params(), a.get_params())
    for x in batches:
        x.close()
    a.close(); b.close(); c.close(); s.close()
