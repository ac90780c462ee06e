"""Write the high-precision reference fixtures in this folder.

Calls only ``oracle/`` (the 50-digit mpmath dense GP) on small seeded inputs
with adversarial time grids: duplicate times (gap 0), gaps of 1e-9 and 1e-6
(where the multiplied-out precision blocks of Theorem 1 lose all accuracy in
float64), N = 1 and N = 2.  Run from the repository root:

    python tests/golden/make_golden.py
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.dense import gp_dense_mp  # noqa: E402
from oracle.ssm import model_for  # noqa: E402


def cases():
    rng = np.random.default_rng(20161025)
    out = []
    # Matern-5/2, Exp(1) gaps with a duplicate and two tiny gaps
    gaps = rng.exponential(1.0, 24)
    gaps[5] = 0.0
    gaps[11] = 1e-9
    gaps[17] = 1e-6
    t = np.cumsum(gaps)
    out.append(("matern52_adversarial_gaps", [(2, 0)], [5.0, 2.0, 0.05], t))
    # Matern-3/2 on a sorted uniform grid with repeated times
    t = np.sort(rng.uniform(0.0, 10.0, 24))
    t[7] = t[6]
    t[15] = t[14] + 1e-9
    out.append(("matern32_repeated_times", [(1, 0)], [1.0, 1.0, 0.1], t))
    # Matern-3/2 + 3-harmonic periodic (its transition noise is exactly zero)
    t = np.sort(rng.uniform(0.0, 100.0, 20))
    out.append(("matern32_plus_periodic3", [(1, 0), (3, 3)], [50.0, 1.0, 1.0, 1.0, 24.0, 0.1], t))
    # single points and pairs
    out.append(("matern52_single_point", [(2, 0)], [5.0, 2.0, 0.05], np.array([3.25])))
    out.append(("matern32_two_points", [(1, 0)], [1.0, 1.0, 0.1], np.array([0.5, 1.75])))
    out.append(("matern52_two_equal_times", [(2, 0)], [5.0, 2.0, 0.05], np.array([2.0, 2.0])))
    res = []
    for name, terms, hyper, t in out:
        y = rng.standard_normal(t.shape[0])
        res.append((name, terms, hyper, t, y))
    return res


def main():
    fixtures = []
    for name, terms, hyper, t, y in cases():
        ref = gp_dense_mp(model_for(terms, hyper), t, y, dps=50)
        fixtures.append({
            "name": name, "terms": terms, "hyper": list(hyper),
            "t": [float(v) for v in t], "y": [float(v) for v in y],
            "logml": ref["logml"], "datafit": ref["datafit"], "logdet": ref["logdet"],
            "f_mean": [float(v) for v in ref["f_mean"]], "f_var": [float(v) for v in ref["f_var"]],
        })
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mp_dense_adversarial.json")
    with open(path, "w") as f:
        json.dump({"source": "oracle.dense.gp_dense_mp at 50 digits (eq. ml2, mean2, k3)",
                   "fixtures": fixtures}, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
