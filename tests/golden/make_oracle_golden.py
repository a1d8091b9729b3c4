"""Writes oracle_small_frames.json: a regression record of the oracle on a few
seeded small frames (6v6, 20 cm lattice, one flat 4 m/s pass, 64 samples).

It calls only the oracle (inputs come from the seeded generator).  Re-run it
only when the oracle's arithmetic changes on purpose, and name in the commit
the passage of the paper, or the reading of it, that justifies the change.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import oracle as O  # noqa: E402
from paper_1909_07717_amd.framegen import Params, config_small  # noqa: E402


def main():
    p = Params(n_samples=64).as_f32()
    rec = []
    for seed in range(5):
        f = config_small(seed)
        r = O.search_frame(f, p)
        s = r["score"]
        fin = np.isfinite(s)
        rec.append(dict(seed=seed, n_feasible=int(r["mask"].sum()), best=int(r["best"]),
                        best_score=repr(float(r["best_score"])),
                        score_sum=repr(float(s[fin].sum())),
                        t_team_finite=int(np.isfinite(r["t_team"]).sum()),
                        t_opp_finite=int(np.isfinite(r["t_opp"]).sum())))
    with open(os.path.join(HERE, "oracle_small_frames.json"), "w") as fh:
        json.dump(rec, fh, indent=1)


if __name__ == "__main__":
    main()
