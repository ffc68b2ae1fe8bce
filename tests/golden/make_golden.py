"""Writes tests/golden/rank2_n12.json: a seeded rank-2 column-row update
(Sec. 2.2, Steps 1-2) at n = 12 and the oracle's updated eigenpairs.

Calls only the seeded generators and ``oracle``.  Run from the repository root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1706_00773_amd import workloads as wl  # noqa: E402


def main():
    u = wl.plain_rank2(12, seed=4242, min_gap=1e-3)
    lo, Qo, _ = oracle.update(u.lam, u.Q, u.K, u.sigma)
    out = {
        "source": "oracle.update on workloads.plain_rank2(12, seed=4242, min_gap=1e-3)",
        "lam": u.lam.tolist(),
        "Q": np.asarray(u.Q).ravel(order="F").tolist(),
        "K": np.asarray(u.K).ravel(order="F").tolist(),
        "sigma": [int(s) for s in u.sigma],
        "lam_new": lo.tolist(),
        "Q_new": Qo.ravel(order="F").tolist(),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rank2_n12.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
