"""Comparison of HIP-path outputs with the oracle (test helper).

Tolerances (FP32 GPU vs FP64 oracle):
  * interception times: 1e-4 s absolute on entries outside the oracle's
    ambiguity bands, infinities matching exactly;
  * feasibility flags: identical outside the bands (reach edge, chip landing
    edge, first-crossing flips, and |margin - threshold| < 1e-3 s);
  * scores: 1e-5 relative (to max(|S|, S_FLOOR)) where both sides are
    feasible, outside the reach, landing and crossing bands;
  * best pass: found flags agree, and the oracle's score at the GPU's choice is
    within that tolerance below the oracle's best;
  * banded fraction (reach, landing and crossing bands) at most 1e-3 of the
    entries a test compares, pooled over the test's maps, with no allowance.
"""
from __future__ import annotations

import numpy as np

T_ABS = 1e-4
S_REL = 1e-5
AMB_MAX = 1e-3
# Scores are compared relative to max(|S|, S_FLOOR): S_FLOOR is the smallest
# feasible score under the default weights (0.3 (1 - 12.82 / 15) + 0.2 * 0.1),
# so the default scores keep their plain relative bound while weights that
# let scores pass through zero keep that bound's absolute size there.
S_FLOOR = 0.0637


class BandPool:
    """Entries and reach / landing / crossing-banded entries pooled over
    every map a test compares.  The cap on the banded share is a rate, so it
    is taken over the test's whole sample: ``check()`` fails when the pooled
    share exceeds AMB_MAX (no allowance on top)."""

    def __init__(self, label: str = ""):
        self.label = label
        self.n = 0
        self.banded = 0
        self.flips = 0

    def add(self, n: int, banded: int, flips: int):
        self.n += n
        self.banded += banded
        self.flips += flips

    def check(self):
        rate = self.banded / max(self.n, 1)
        print(f"[parity] {self.label}: pooled banded {self.banded} of {self.n} "
              f"({rate:.2e}), flag flips inside bands {self.flips}", flush=True)
        assert self.banded <= AMB_MAX * self.n, (
            f"{self.label}: {self.banded} banded of {self.n} ({rate:.2e} > {AMB_MAX})")
        return rate


def compare_maps(gpu: dict, orc: dict, label: str = "", check_times: bool = True,
                 pool: BandPool | None = None) -> dict:
    """Entry-by-entry comparison of one set of maps.  The banded share is
    added to ``pool`` (checked by the caller once every map is in); without a
    pool this map alone must stay under the cap."""
    amb = orc["ambig"] != 0
    n = amb.size
    gm = gpu["mask"].astype(bool)
    om = orc["mask"].astype(bool)
    bad = (gm != om) & ~amb
    assert not bad.any(), (f"{label}: {int(bad.sum())} feasibility mismatches outside the bands, "
                           f"first at {np.flatnonzero(bad)[:5]}")
    # scores where both sides are feasible, outside the reach, landing and
    # crossing bands (there the interception times themselves may differ)
    both = gm & om & ((orc["ambig"] & 7) == 0)
    if both.any():
        gs = gpu["score"][both].astype(np.float64)
        os_ = orc["score"][both]
        rel = np.abs(gs - os_) / np.maximum(np.abs(os_), S_FLOOR)
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
    # the computation: only the reach / landing / crossing bands count here
    comp = int(((orc["ambig"] & 7) != 0).sum())
    flips = int(((gm != om) & amb).sum())
    print(f"[parity] {label}: n={n} banded={comp} margin-band="
          f"{int(((orc['ambig'] & 8) != 0).sum())} flag flips inside bands={flips}", flush=True)
    if pool is not None:
        pool.add(n, comp, flips)
    else:
        assert comp <= AMB_MAX * n, f"{label}: {comp} banded of {n} (cap {AMB_MAX})"
    return dict(n=n, ambiguous=int(amb.sum()), banded=comp, feasible=int(om.sum()), flips=flips)


def check_best(best, orc: dict, elem_index: int, label: str = ""):
    """The GPU's best pass against the oracle's maps (frame-relative index)."""
    orc_best = orc["best"]
    found = bool(best["found"])
    assert found == (orc_best >= 0), f"{label}: found {found} vs oracle {orc_best}"
    if found:
        bs = orc["score"][orc_best]
        if orc["ambig"][elem_index]:
            # an ambiguous entry: only its score is comparable
            assert float(best["score"]) >= bs - S_REL * max(abs(bs), S_FLOOR) - 1e-6, label
            return
        got = orc["score"][elem_index]
        assert got >= bs - S_REL * max(abs(bs), S_FLOOR), f"{label}: oracle score at GPU choice {got} < best {bs}"
