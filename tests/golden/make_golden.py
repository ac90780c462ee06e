"""Write the high-precision reference fixtures in this folder.

Calls only ``oracle/`` (the 50-digit mpmath dense GP and state posterior of
``oracle.mpref``) on small seeded inputs.

``mp_dense_adversarial.json``: adversarial time grids (duplicate times, gaps of
1e-9 and 1e-6, where the multiplied-out precision blocks of Theorem 1 lose all
accuracy in float64), N = 1 and N = 2; logML, data fit, log det, latent mean and
variance.

``mp_kinds.json``: every term kind the oracle models (Matern-1/2 .. 7/2,
periodic, quasi-periodic, squared exponential of orders 4, 6, 8 and 10, and sums
of them), with logML, data fit, log det, latent mean and variance and
dlogML/dtheta (central differences of the 50-digit logML at 90 digits); for
state dimensions up to 4 also the posterior state means and the blocks
Cov(z_n, z_n | y) (packed upper, row-major) and Cov(z_{n+1}, z_n | y).  The
squared-exponential trends with lengthscales 0.02, 0.1 and 0.2 are the cases
where float64 work in the model's own state (f, f', ..., f^(5)) loses about
lam^10 eps.  Run from the repository root:

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
from oracle.mpref import gp_dense_mp as gp_dense_mp_terms  # noqa: E402
from oracle.mpref import state_posterior_dense_mp  # noqa: E402
from oracle.ssm import model_for  # noqa: E402

M32, M52, PER, M12, M72, QP, SE = 1, 2, 3, 4, 5, 6, 7
CO2 = [(M32, 0), (QP, 3), (SE, 6)]
CO2_HYPER = [50.0, 1.0, 1.2, 0.8, 6.0, 15.0, 2.0, 0.5, 0.1]


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


def adversarial_times(rng, n, scale):
    """Exp(scale) gaps with one duplicate time and gaps of 1e-9 and 1e-6 (relative to scale)."""
    gaps = rng.exponential(scale, n)
    gaps[n // 4] = 0.0
    gaps[n // 2] = 1e-9 * scale
    gaps[3 * n // 4] = 1e-6 * scale
    return np.cumsum(gaps)


def kind_cases():
    rng = np.random.default_rng(20161026)
    out = []
    # one-term Matern models of every order on adversarial grids (b = 1 .. 4), with blocks
    for name, kind, hyper in (("matern12", M12, [2.0, 1.1, 0.1]), ("matern32", M32, [1.0, 1.0, 0.1]),
                              ("matern52", M52, [5.0, 2.0, 0.05]), ("matern72", M72, [4.0, 1.5, 0.05])):
        out.append((name + "_adversarial", [(kind, 0)], hyper, adversarial_times(rng, 24, 0.5 * hyper[0]), True))
    # the sums of the wide-state path (b = 10, 16) and squared-exponential terms on their own
    t = np.sort(rng.uniform(0.0, 40.0, 16))
    t[9] = t[8]
    out.append(("matern32_periodic3", [(M32, 0), (PER, 3)], [50.0, 1.0, 1.0, 1.0, 24.0, 0.1], t, False))
    out.append(("matern32_quasiperiodic3", [(M32, 0), (QP, 3)], [50.0, 1.0, 1.2, 0.8, 6.0, 15.0, 0.1],
                np.sort(rng.uniform(0.0, 30.0, 16)), False))
    t = np.sort(rng.uniform(0.0, 12.0, 16))
    t[5] = t[4]
    out.append(("co2_three_terms", CO2, CO2_HYPER, t, False))
    out.append(("sqexp6", [(SE, 6)], [1.3, 0.7, 0.1], np.sort(rng.uniform(0.0, 10.0, 20)), False))
    out.append(("matern32_sqexp10", [(M32, 0), (SE, 10)], [3.0, 1.0, 1.5, 0.8, 0.05],
                np.sort(rng.uniform(0.0, 12.0, 16)), False))
    # short squared-exponential trend lengthscales in the three-term sum (points 0.05 apart on
    # average, as in the float64 parity runs of that model)
    for ell_s in (0.02, 0.1, 0.2):
        hyper = list(CO2_HYPER)
        hyper[6] = ell_s
        out.append((f"co2_three_terms_sqexp_lengthscale_{ell_s:g}", CO2, hyper,
                    np.sort(rng.uniform(0.0, 2.4, 48)), False))
    res = []
    for name, terms, hyper, t, blocks in out:
        y = rng.standard_normal(t.shape[0])
        res.append((name, terms, hyper, t, y, blocks))
    # signal-to-noise 1e6: Matern-5/2 with noise variance 1e-6, Exp(1) gaps (its own stream)
    r2 = np.random.default_rng(20161027)
    t = np.cumsum(r2.exponential(1.0, 40))
    res.append(("matern52_noise_1e-6", [(M52, 0)], [2.0, 1.0, 1e-6], t, r2.standard_normal(40), True))
    # further sums of the wide-state path (b = 4 .. 12), one stream of their own
    r3 = np.random.default_rng(20161028)
    more = [("matern52_periodic1", [(M52, 0), (PER, 1)], [3.0, 1.0, 1.0, 0.8, 6.0, 0.1], 20.0),
            ("matern12_matern32_quasiperiodic1", [(M12, 0), (M32, 0), (QP, 1)],
             [1.0, 0.3, 2.0, 1.0, 1.2, 0.8, 6.3, 20.0, 0.1], 20.0),
            ("sqexp4", [(SE, 4)], [2.0, 1.0, 0.1], 15.0),
            ("matern72_sqexp8", [(M72, 0), (SE, 8)], [4.0, 1.0, 3.0, 0.6, 0.05], 15.0),
            ("periodic2", [(PER, 2)], [1.0, 1.0, 5.0, 0.05], 20.0)]
    for name, terms, hyper, span in more:
        t = np.sort(r3.uniform(0.0, span, 16))
        t[6] = t[5]
        res.append((name, terms, hyper, t, r3.standard_normal(16), False))
    return res


def _f(a):
    return [float(v) for v in np.asarray(a).reshape(-1)]


def write_kinds(path):
    fixtures = []
    for name, terms, hyper, t, y, blocks in kind_cases():
        ref = gp_dense_mp_terms(terms, hyper, t, y, dps=50, want_grad=True)
        fx = {"name": name, "terms": terms, "hyper": list(hyper), "t": _f(t), "y": _f(y),
              "logml": ref["logml"], "datafit": ref["datafit"], "logdet": ref["logdet"],
              "f_mean": _f(ref["f_mean"]), "f_var": _f(ref["f_var"]), "grad": _f(ref["grad"])}
        if blocks:
            sp = state_posterior_dense_mp(terms, hyper, t, y, dps=50)
            b = sp["z_mean"].shape[1]
            iu = np.triu_indices(b)
            fx["b"] = b
            fx["z_mean"] = _f(sp["z_mean"])
            fx["S_diag_upper"] = _f(sp["S_diag"][:, iu[0], iu[1]])
            fx["S_sub"] = _f(sp["S_sub"])
        fixtures.append(fx)
        print(name, flush=True)
    with open(path, "w") as f:
        json.dump({"source": "oracle.mpref at 50 digits: dense GP (eq. ml2, mean2, k3), gradient by central "
                             "differences at 90 digits, state posterior blocks (Sec. 3.1 subproblems 2, 4)",
                   "fixtures": fixtures}, f, indent=0)
    print("wrote", path)


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
    write_kinds(os.path.join(os.path.dirname(os.path.abspath(__file__)), "mp_kinds.json"))


if __name__ == "__main__":
    main()
