"""dpps_search_batch_noalloc (the batched search on the library's fixed
device array) against dpps_search_batch on the same inputs: two calls in a
row, the second with a smaller request, every output bitwise equal; a
request larger than the array is refused before anything runs."""
import numpy as np
import pytest

from paper_1909_07717_amd.framegen import (Params, config_full, config_small, full_window,
                                           random_frame, random_window, variants_for)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_1909_07717_amd import binding
    assert torch.cuda.is_available()
    return binding


def _host(out):
    return {k: getattr(out, k).cpu().numpy() for k in ("mask", "score", "t_team", "t_opp", "best")}


def _same(a, b, label):
    for k in a:
        assert a[k].tobytes() == b[k].tobytes(), (label, k)


def _frames_large():
    rng = np.random.default_rng(41)
    fs = [config_small(s) for s in range(6)]
    f = random_frame(rng, 8, 7)
    f.windows = [random_window(rng, 0.05), (0.25, 3, 4, 0, 5), (0.1, 37, 11, 13, 7)]
    f.variants = variants_for([1.5, 3.25, 5.0], flat=True, chip=True)
    fs.append(f)
    fs.append(config_full(3))
    return fs


def _frames_small():
    f = random_frame(np.random.default_rng(42), 5, 6)
    f.windows = [full_window(0.5)]
    f.variants = variants_for([2.0, 4.5], flat=True, chip=False)
    return [config_small(100), f]


@pytest.mark.parametrize("K", [64, 256])
def test_noalloc_equals_batch_twice_then_smaller(B, K):
    p = Params(n_samples=K).as_f32()
    s = B.Searcher(p)
    for label, frames in (("first", _frames_large()), ("second, smaller", _frames_small())):
        print(f"[noalloc] K={K} {label}: {len(frames)} frames", flush=True)
        pk, ref = s.search_batch(frames, times=True)
        torch.cuda.synchronize()
        want = _host(ref)
        out = s.outputs_for(pk, times=True)
        out.mask.fill_(7)
        out.score.fill_(3.0)
        out.t_team.fill_(-1.0)
        out.t_opp.fill_(-1.0)
        out.best.fill_(0)
        s.search_batch_noalloc(pk, out)
        torch.cuda.synchronize()
        _same(want, _host(out), label)
        assert np.isfinite(want["score"]).any()
    s.close()


def test_noalloc_on_another_context_and_stream(B):
    """A second context on the same GPU uses the same array; a call on a
    caller's stream gives the same results."""
    p = Params(n_samples=128).as_f32()
    frames = _frames_small()
    s1, s2 = B.Searcher(p), B.Searcher(p)
    pk, ref = s1.search_batch(frames, times=True)
    torch.cuda.synchronize()
    want = _host(ref)
    st = torch.cuda.Stream()
    for s in (s2, s1):
        out = s.outputs_for(pk, times=True)
        with torch.cuda.stream(st):
            s.search_batch_noalloc(pk, out, stream=st)
        st.synchronize()
        _same(want, _host(out), "context")
    s1.close()
    s2.close()


def test_noalloc_refuses_a_request_larger_than_the_array(B):
    p = Params(n_samples=64).as_f32()
    s = B.Searcher(p)
    frames = [config_full(s_) for s_ in range(30)]
    pk = B.pack(frames, p)
    out = B.DeviceOutputs(1, len(frames), s.device, mask=False, score=False)
    with pytest.raises(B.DppsError) as e:
        s.search_batch_noalloc(pk, out)
    assert e.value.code == -4
    # the array is untouched by the refusal: a fitting request still matches
    frames = _frames_small()
    pk, ref = s.search_batch(frames, times=True)
    torch.cuda.synchronize()
    out = s.outputs_for(pk, times=True)
    s.search_batch_noalloc(pk, out)
    torch.cuda.synchronize()
    _same(_host(ref), _host(out), "after refusal")
    s.close()
