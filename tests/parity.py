"""Comparison of HIP-path outputs with the oracle (test helper).

Tolerances (FP32 GPU vs FP64 oracle):
  * interception times: 1e-4 s absolute on entries outside the oracle's
    ambiguity bands, infinities matching exactly;
  * feasibility flags: identical outside the bands (reach edge, chip landing
    edge, first-crossing flips, and |margin - threshold| < 1e-3 s);
  * scores: 1e-5 relative where both sides are feasible;
  * best pass: found flags agree, and the oracle's score at the GPU's choice is
    at least (1 - 1e-5) times the oracle's best;
  * ambiguous fraction below 1e-3.
"""
import numpy as np

T_ABS = 1e-4
S_REL = 1e-5
AMB_MAX = 1e-3


def compare_maps(gpu: dict, orc: dict, label: str = "", check_times: bool = True) -> dict:
    amb = orc["ambig"] != 0
    n = amb.size
    gm = gpu["mask"].astype(bool)
    om = orc["mask"].astype(bool)
    bad = (gm != om) & ~amb
    assert not bad.any(), (f"{label}: {int(bad.sum())} feasibility mismatches outside the bands, "
                           f"first at {np.flatnonzero(bad)[:5]}")
    both = gm & om
    if both.any():
        gs = gpu["score"][both].astype(np.float64)
        os_ = orc["score"][both]
        rel = np.abs(gs - os_) / np.abs(os_)
        assert rel.max() <= S_REL, f"{label}: score rel err {rel.max():.3e}"
    assert np.all(np.isneginf(gpu["score"][~gm])), f"{label}: infeasible score not -inf"
    if check_times and gpu.get("t_team") is not None:
        for k in ("t_team", "t_opp"):
            g = gpu[k].astype(np.float64)
            o = orc[k]
            ok = ~amb
            gi, oi = np.isinf(g) & ok, np.isinf(o) & ok
            assert np.array_equal(gi, oi), f"{label}: {k} infinity mismatch at {np.flatnonzero(gi != oi)[:5]}"
            fin = ok & ~oi
            if fin.any():
                err = np.abs(g[fin] - o[fin])
                assert err.max() <= T_ABS, f"{label}: {k} abs err {err.max():.3e}"
    # the margin band is a stated tolerance on the flags, not an ambiguity of
    # the computation: only the reach / landing / crossing bands count here.
    # Their expected rate is below AMB_MAX; the bound is one-sided 4 sigma
    # (Poisson) so that small maps do not fail on counting noise.
    comp = (orc["ambig"] & 7) != 0
    lam = AMB_MAX * n
    flips = int(((gm != om) & amb).sum())
    print(f"[parity] {label}: n={n} banded={int(comp.sum())} margin-band="
          f"{int(((orc['ambig'] & 8) != 0).sum())} flag flips inside bands={flips}", flush=True)
    assert comp.sum() <= lam + 4.0 * np.sqrt(lam) + 1.0, (
        f"{label}: {int(comp.sum())} ambiguous of {n} (rate limit {AMB_MAX})")
    return dict(n=n, ambiguous=int(amb.sum()), feasible=int(om.sum()), flips=flips)


def check_best(best, orc: dict, elem_index: int, label: str = ""):
    """The GPU's best pass against the oracle's maps (frame-relative index)."""
    orc_best = orc["best"]
    found = bool(best["found"])
    assert found == (orc_best >= 0), f"{label}: found {found} vs oracle {orc_best}"
    if found:
        bs = orc["score"][orc_best]
        if orc["ambig"][elem_index]:
            # an ambiguous entry: only its score is comparable
            assert float(best["score"]) >= (1 - S_REL) * bs - 1e-6, label
            return
        got = orc["score"][elem_index]
        assert got >= (1 - S_REL) * bs, f"{label}: oracle score at GPU choice {got} < best {bs}"
