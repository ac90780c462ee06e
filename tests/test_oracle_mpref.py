"""Pins of the 50-digit references (oracle.mpref) against routes that share none of their code,
and of the float64 oracles against the stored 50-digit fixtures of every term kind.

- The covariance function written out per kind (closed forms; residues of the rational spectral
  density for the squared exponential) against the state-space form (companion or rotation F,
  closed-form or Lyapunov P0, mpmath's expm), Sec. 2.1: h expm(F tau) P0 h^T = k(tau).
- The squared-exponential approximation against the squared exponential itself: the gap shrinks
  as the order grows (the truncated exponential series converges).
- The dense 50-digit GP (logML, mean, variance, gradient) against the float64 dense GP (scipy
  Cholesky, float64 closed forms, the trace formula for the gradient) on comfortable inputs.
- The 50-digit state posterior against the float64 dense state posterior.
- Every term kind raises when the reference does not model it.
- The float64 oracles (C elimination, Python elimination, Kalman filter + RTS smoother) against
  the stored fixtures ``golden/mp_kinds.json`` (written by ``golden/make_golden.py``, which calls
  only ``oracle/``): Matern orders 1/2 .. 7/2 on adversarial gaps with their state blocks, sums
  of terms as the wide-state path runs them, squared exponentials of orders 4, 6, 8 and 10.
"""
import json
import os

import mpmath as mp
import numpy as np
import pytest

from oracle import btd, dense, kalman, mpref, native
from oracle.ssm import MATERN12, MATERN32, MATERN52, MATERN72, PERIODIC, QUASIPERIODIC, SQEXP, model_for

KINDS = os.path.join(os.path.dirname(__file__), "golden", "mp_kinds.json")
FIXTURES = json.load(open(KINDS))["fixtures"]

TERM_CASES = [
    ("m12", [(MATERN12, 0)], [2.0, 1.1, 0.1]),
    ("m32", [(MATERN32, 0)], [1.0, 1.0, 0.1]),
    ("m52", [(MATERN52, 0)], [5.0, 2.0, 0.05]),
    ("m72", [(MATERN72, 0)], [4.0, 1.5, 0.05]),
    ("per3", [(PERIODIC, 3)], [1.2, 0.8, 6.0, 0.1]),
    ("qp3", [(QUASIPERIODIC, 3)], [1.2, 0.8, 6.0, 15.0, 0.1]),
    ("se6", [(SQEXP, 6)], [1.3, 0.7, 0.1]),
    ("se10", [(SQEXP, 10)], [0.9, 1.4, 0.1]),
    ("co2", [(MATERN32, 0), (QUASIPERIODIC, 3), (SQEXP, 6)], [50.0, 1.0, 1.2, 0.8, 6.0, 15.0, 2.0, 0.5, 0.1]),
]


@pytest.mark.parametrize("name,terms,hyper", TERM_CASES, ids=[c[0] for c in TERM_CASES])
def test_kernel_closed_form_equals_state_space_form(name, terms, hyper):
    """Sec. 2.1: the state-space model implies the kernel (for the squared exponential: the
    residue sum of its rational spectral density equals h expm(F tau) P0 h^T with P0 from a
    Lyapunov solve)."""
    k0 = mpref.kernel_mp(terms, hyper, 0.0)
    for tau in (0.0, 1e-9, 0.21, 1.7, 6.3, 19.0):
        a = mpref.kernel_mp(terms, hyper, tau)
        b = mpref.ssm_kernel_mp(terms, hyper, tau)
        assert abs(a - b) <= mp.mpf(10) ** -40 * abs(k0), (tau, a, b)


def test_matern_closed_forms_by_value():
    """Textbook values: Matern-1/2 at lam tau = 1 is var/e; Matern-3/2 at 1 is 2 var/e;
    Matern-5/2 at 1 is (7/3) var/e; Matern-7/2 at 1 is (1 + 1 + 2/5 + 1/15) var/e."""
    for kind, nu2, val in ((MATERN12, 1, 1), (MATERN32, 3, 2), (MATERN52, 5, mp.mpf(7) / 3),
                           (MATERN72, 7, 1 + 1 + mp.mpf(2) / 5 + mp.mpf(1) / 15)):
        ell = 1.3
        tau = float(mp.mpf(ell) / mp.sqrt(nu2))          # lam tau = 1 up to the rounding of tau
        got = mpref.kernel_mp([(kind, 0)], [ell, 0.75, 0.1], tau)
        assert abs(got - mp.mpf(0.75) * val / mp.e) < 1e-15


def test_periodic_weights_sum_to_truncated_series():
    """The Bessel weights are the cosine series of exp(-2 sin^2(w0 tau / 2) / l^2); with many
    harmonics the truncated kernel reaches the untruncated one."""
    ell, var, per = 0.9, 1.3, 5.0
    for tau in (0.0, 0.7, 2.2):
        got = mpref.kernel_mp([(PERIODIC, 40)], [ell, var, per, 0.1], tau)
        with mp.workdps(50):
            s = mp.sin(mp.pi * mp.mpf(tau) / per)
            exact = var * mp.exp(-2 * s * s / mp.mpf(ell) ** 2)
            assert abs(got - exact) < 1e-40


def test_sqexp_approximation_converges_with_order():
    """The order-n approximation approaches var exp(-tau^2 / (2 l^2)) as n grows; order 6 is
    within 3.1e-3 var of it (k(0) = 1.00299 var)."""
    ell, var = 1.1, 0.8
    taus = np.linspace(0.0, 4.0, 21)
    errs = []
    for order in (2, 4, 6, 8, 10):
        e = max(abs(float(mpref.kernel_mp([(SQEXP, order)], [ell, var, 0.1], x)) - var * np.exp(-0.5 * (x / ell) ** 2))
                for x in taus)
        errs.append(e / var)
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1)), errs
    assert errs[2] < 3.1e-3 and errs[4] < 2e-4
    assert abs(float(mpref.kernel_mp([(SQEXP, 6)], [ell, var, 0.1], 0.0)) / var - 1.00299) < 1e-5


def test_unknown_kinds_raise():
    with pytest.raises(ValueError):
        mpref.kernel_mp([(99, 0)], [1.0, 1.0, 0.1], 0.5)
    with pytest.raises(ValueError):
        mpref.gp_dense_mp([(MATERN32, 0)], [1.0, 1.0], [0.0, 1.0], [0.1, 0.2])     # noise missing
    with pytest.raises(ValueError):
        mpref.kernel_mp([(SQEXP, 5)], [1.0, 1.0, 0.1], 0.5)                          # odd order
    m = model_for([(MATERN32, 0)], [1.0, 1.0, 0.1])
    m.terms = [(42, 0)]
    with pytest.raises(ValueError):
        dense.gp_dense_mp(m, [0.0, 1.0], [0.1, 0.2])


@pytest.mark.parametrize("name,terms,hyper", TERM_CASES, ids=[c[0] for c in TERM_CASES])
def test_dense_mp_matches_float64_dense(name, terms, hyper):
    """Comfortable inputs (no tiny gaps): the 50-digit dense GP and the float64 dense GP agree to
    the float64 one's accuracy, gradient included.  The float64 kernel of the squared-exponential
    approximation (float64 roots and Lyapunov solve) is itself off by a measured relative delta
    (about 3e-11 at order 10); the bars grow with it."""
    rng = np.random.default_rng(5)
    n = 14
    t = np.sort(rng.uniform(0.0, 15.0, n))
    y = rng.standard_normal(n)
    m = model_for(terms, hyper)
    r = mpref.gp_dense_mp(terms, hyper, t, y, want_grad=True)
    d = dense.gp_dense(m, t, y, want_grad=True)
    k0 = float(mpref.kernel_mp(terms, hyper, 0.0))
    delta = max(abs(float(m.kernel(np.array(x))) - float(mpref.kernel_mp(terms, hyper, x))) / k0
                for x in np.abs(t[:, None] - t[None, :]).reshape(-1)[::7])
    tol = max(1e-11, 100.0 * delta)
    assert abs(r["logml"] - d["logml"]) <= tol * abs(d["logml"])
    assert np.all(np.abs(r["f_mean"] - d["f_mean"]) <= 10 * tol * (np.abs(d["f_mean"]) + np.sqrt(d["f_var"])))
    assert np.all(np.abs(r["f_var"] - d["f_var"]) <= 10 * tol * d["f_var"])
    assert np.abs(r["grad"] - d["grad"]).max() <= 100 * tol * np.abs(d["grad"]).max()


@pytest.mark.parametrize("name,terms,hyper", [c for c in TERM_CASES if c[0] in ("m52", "m72", "qp3", "se6")],
                         ids=["m52", "m72", "qp3", "se6"])
def test_state_posterior_mp_matches_float64_dense(name, terms, hyper):
    rng = np.random.default_rng(6)
    n = 10
    t = np.sort(rng.uniform(0.0, 12.0, n))
    y = rng.standard_normal(n)
    r = mpref.state_posterior_dense_mp(terms, hyper, t, y)
    d = dense.state_posterior_dense(model_for(terms, hyper), t, y)
    s = np.abs(d["S_diag"]).max()
    assert np.abs(r["S_diag"] - d["S_diag"]).max() <= 1e-10 * s
    assert np.abs(r["S_sub"] - d["S_sub"]).max() <= 1e-10 * s
    assert np.abs(r["z_mean"] - d["z_mean"]).max() <= 1e-10 * max(1.0, np.abs(d["z_mean"]).max())
    g = mpref.gp_dense_mp(terms, hyper, t, y)
    assert abs(r["logml"] - g["logml"]) <= 1e-14 * abs(g["logml"])
    assert np.abs(r["f_var"] - g["f_var"]).max() <= 1e-14 * g["f_var"].max()


# ----------------------------------------------------------------------------- stored fixtures
def _sqexp_lam(fx):
    """Largest 1 / lengthscale over the squared-exponential terms of a fixture (0 if none)."""
    parts, _ = mpref.parse_terms([tuple(x) for x in fx["terms"]], fx["hyper"])
    return max([float(1 / par[0]) for kind, _, par in parts if kind == SQEXP] or [0.0])


def _blocks(fx):
    b, n = fx["b"], len(fx["t"])
    iu = np.triu_indices(b)
    Sd = np.zeros((n, b, b))
    Sd[:, iu[0], iu[1]] = np.array(fx["S_diag_upper"]).reshape(n, -1)
    Sd = Sd + np.triu(Sd, 1).transpose(0, 2, 1)
    return np.array(fx["z_mean"]).reshape(n, b), Sd, np.array(fx["S_sub"]).reshape(max(n - 1, 0), b, b)


def block_errors(z_ref, Sd_ref, Ss_ref, z, Sd, Ss):
    """Largest errors of state means and covariance blocks on the scale sqrt(S_ii S_jj)."""
    d = np.sqrt(np.maximum(np.einsum("nii->ni", Sd_ref), 0.0))
    ez = np.max(np.abs(z - z_ref) / (np.abs(z_ref) + d))
    es = np.max(np.abs(Sd - Sd_ref) / (d[:, :, None] * d[:, None, :]))
    eb = np.max(np.abs(Ss - Ss_ref) / (d[1:, :, None] * d[:-1, None, :])) if len(Ss_ref) else 0.0
    return ez, es, eb


ACCURATE = [f for f in FIXTURES if _sqexp_lam(f) < 1.0]
SHORT_SE = [f for f in FIXTURES if _sqexp_lam(f) >= 1.0]


@pytest.mark.parametrize("fx", ACCURATE, ids=lambda f: f["name"])
def test_float64_oracles_against_50_digit_kinds(fx):
    """logML to 1e-10, mean and variance to the 1e-9 bars, gradient (C tangent-linear) to 1e-9 of
    its largest component; state means and blocks (where stored) to 1e-9 on sqrt(S_ii S_jj)."""
    terms = [tuple(x) for x in fx["terms"]]
    hyper = fx["hyper"]
    t, y = np.array(fx["t"]), np.array(fx["y"])
    m = model_for(terms, hyper)
    mu, v = np.array(fx["f_mean"]), np.array(fx["f_var"])
    outs = [native.btd_factored(terms, hyper, t, y), btd.btd_factored(m, t, y), kalman.kf_rts(m, t, y)]
    for res in outs:
        assert abs(res["logml"] - fx["logml"]) <= 1e-10 * abs(fx["logml"])
        assert np.all(np.abs(res["f_mean"] - mu) <= 1e-9 * (np.abs(mu) + np.sqrt(v)))
        assert np.all(np.abs(res["f_var"] - v) <= 1e-9 * v)
    g = np.array(fx["grad"])
    gc = native.tangent_grad(terms, hyper, t, y)["grad"]
    assert np.abs(gc - g).max() <= 1e-9 * np.abs(g).max()
    if "b" in fx:
        ref = _blocks(fx)
        for res in outs:
            errs = block_errors(*ref, res["z_mean"], res["S_diag"], res["S_sub"])
            assert max(errs) <= 1e-9, errs


@pytest.mark.parametrize("fx", SHORT_SE, ids=lambda f: f["name"])
def test_float64_oracles_lose_lam10_eps_on_short_sqexp_lengthscales(fx):
    """In the model's own state (f, f', ..., f^(5)) P0 spans lam^10: the float64 oracles' mean and
    variance errors against the 50-digit reference stay below 10 lam^10 eps (the reason the
    device parity for these cases is taken against the 50-digit fixtures)."""
    terms = [tuple(x) for x in fx["terms"]]
    hyper = fx["hyper"]
    t, y = np.array(fx["t"]), np.array(fx["y"])
    bound = 10.0 * _sqexp_lam(fx) ** 10 * np.finfo(float).eps
    mu, v = np.array(fx["f_mean"]), np.array(fx["f_var"])
    for res in (native.btd_factored(terms, hyper, t, y, want_blocks=False), kalman.kf_rts(model_for(terms, hyper), t, y)):
        assert np.max(np.abs(res["f_mean"] - mu) / (np.abs(mu) + np.sqrt(v))) <= bound
        assert np.max(np.abs(res["f_var"] - v) / v) <= bound


def test_fixtures_cover_every_kind():
    kinds = {k for f in FIXTURES for k, _ in f["terms"]}
    assert kinds == {MATERN12, MATERN32, MATERN52, MATERN72, PERIODIC, QUASIPERIODIC, SQEXP}
    orders = {h for f in FIXTURES for k, h in f["terms"] if k == SQEXP}
    assert orders == {4, 6, 8, 10}
