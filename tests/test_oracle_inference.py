"""Pins of the oracle's inference routines (Theorem 1, Sec. 2.2-3.1) against independent routes.

Each quantity is checked against something other than the routine itself:
the dense textbook GP (O(N^3) Cholesky of K_y with the closed-form kernel),
50-digit mpmath fixtures, the Kalman filter + RTS smoother, closed forms at
N = 1 and N = 2, finite differences, and invariants of a stationary kernel.
"""
import json
import os

import numpy as np
import pytest

from oracle import btd, dense, kalman, native
from oracle.ssm import MATERN12, MATERN32, MATERN52, MATERN72, PERIODIC, QUASIPERIODIC, SQEXP, model_for
from workloads import make_config

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "mp_dense_adversarial.json")

CASES = [
    ("m32", [(MATERN32, 0)], [1.0, 1.0, 0.1]),
    ("m52", [(MATERN52, 0)], [5.0, 2.0, 0.05]),
    ("m52_short", [(MATERN52, 0)], [0.8, 1.3, 0.2]),
    ("m12", [(MATERN12, 0)], [2.0, 1.1, 0.1]),
    ("m72", [(MATERN72, 0)], [4.0, 1.5, 0.05]),
    ("m32+per3", [(MATERN32, 0), (PERIODIC, 3)], [50.0, 1.0, 1.0, 1.0, 24.0, 0.1]),
    ("m32+qp3", [(MATERN32, 0), (QUASIPERIODIC, 3)], [50.0, 1.0, 1.2, 0.8, 6.0, 15.0, 0.1]),
    ("se6", [(SQEXP, 6)], [1.3, 0.7, 0.1]),
    ("co2", [(MATERN32, 0), (QUASIPERIODIC, 3), (SQEXP, 6)], [50.0, 1.0, 1.2, 0.8, 6.0, 15.0, 2.0, 0.5, 0.1]),
]


def _data(n, seed, span=60.0):
    rng = np.random.default_rng(seed)
    t = np.sort(rng.uniform(0.0, span, n))
    y = rng.standard_normal(n)
    return t, y


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


# ----------------------------------------------------------------------------- Theorem 1
@pytest.mark.parametrize("name,terms,hyper", CASES[:5])
def test_theorem1_AQA_and_btd_inverse(name, terms, hyper):
    """eq. k1: A Q A^T is the stacked prior covariance; its inverse is BTD and equals Kb - I (x) J."""
    m = model_for(terms, hyper)
    # a comfortable grid so that the explicit inverses are accurate
    t = np.cumsum(np.full(7, 0.9 * m.parts[0].ell))
    Abig, Qbig, K = dense.paper_AQA(m, t)
    Kst = dense.stacked_prior_cov(m, t)
    assert np.allclose(K, Kst, rtol=1e-12, atol=1e-12 * np.abs(Kst).max())
    Kinv = np.linalg.inv(Kst)
    b, n = m.b, t.shape[0]
    scale = np.abs(Kinv).max()
    for i in range(n):
        for j in range(n):
            if abs(i - j) > 1:
                assert np.abs(Kinv[i * b:(i + 1) * b, j * b:(j + 1) * b]).max() <= 1e-9 * scale
    # A^-T Q^-1 A^-1 and the literal blocks of the oracle
    hh = np.linalg.inv(Abig).T @ np.linalg.inv(Qbig) @ np.linalg.inv(Abig)
    assert np.allclose(hh, Kinv, rtol=0, atol=1e-9 * scale)
    D, B = btd.precision_blocks(m, t)
    J = np.outer(m.H(), m.H()) / m.noise
    Kb = btd.btd_dense_blocks(D, B) - np.kron(np.eye(n), J)
    assert np.allclose(Kb, Kinv, rtol=0, atol=1e-9 * scale)


@pytest.mark.parametrize("name,terms,hyper", CASES[:5])
def test_determinant_lemma(name, terms, hyper):
    """eq. det_1: log det K_y = log det Kb - log det Kinv + N log s2."""
    m = model_for(terms, hyper)
    t = np.cumsum(np.full(8, 0.8 * m.parts[0].ell))
    n = t.shape[0]
    Kf = m.kernel(t[:, None] - t[None, :])
    lhs = np.linalg.slogdet(Kf + m.noise * np.eye(n))[1]
    D, B = btd.precision_blocks(m, t)
    Kb = btd.btd_dense_blocks(D, B)
    Kst = dense.stacked_prior_cov(m, t)
    rhs = np.linalg.slogdet(Kb)[1] + np.linalg.slogdet(Kst)[1] + n * np.log(m.noise)
    assert rel(rhs, lhs) < 1e-10


# ----------------------------------------------------------------------------- dense vs BTD
@pytest.mark.parametrize("name,terms,hyper", CASES)
@pytest.mark.parametrize("n", [1, 2, 3, 17, 150])
def test_factored_btd_matches_dense_gp(name, terms, hyper, n):
    m = model_for(terms, hyper)
    t, y = _data(n, seed=n)
    d = dense.gp_dense(m, t, y, want_grad=False)
    f = btd.btd_factored(m, t, y)
    assert rel(f["logml"], d["logml"]) < 1e-11
    assert rel(f["logdet"], d["logdet"]) < 1e-10 or abs(f["logdet"] - d["logdet"]) < 1e-10
    scale = np.sqrt(d["f_var"]) + np.abs(d["f_mean"])
    assert np.all(np.abs(f["f_mean"] - d["f_mean"]) <= 1e-10 * scale)
    assert np.all(np.abs(f["f_var"] - d["f_var"]) <= 1e-10 * d["f_var"] + 1e-15)


@pytest.mark.parametrize("name,terms,hyper", CASES)
def test_selected_inverse_matches_dense_state_posterior(name, terms, hyper):
    """Takahashi's blocks S_n, S_{n+1,n} and the state means against the dense stacked posterior."""
    m = model_for(terms, hyper)
    t, y = _data(25, seed=7, span=30.0)
    sp = dense.state_posterior_dense(m, t, y)
    f = btd.btd_factored(m, t, y)
    s = np.abs(sp["S_diag"]).max()
    assert np.abs(f["S_diag"] - sp["S_diag"]).max() <= 1e-9 * s
    assert np.abs(f["S_sub"] - sp["S_sub"]).max() <= 1e-9 * s
    assert np.abs(f["z_mean"] - sp["z_mean"]).max() <= 1e-9 * max(1.0, np.abs(sp["z_mean"]).max())


@pytest.mark.parametrize("name,terms,hyper", CASES[:5])
def test_literal_btd_matches_dense_on_comfortable_grid(name, terms, hyper):
    """The paper's multiplied-out blocks (literal Thomas) are exact when lam*dt is not small."""
    m = model_for(terms, hyper)
    lam = m.parts[0].lam
    rng = np.random.default_rng(3)
    # comfortable means cond(Q_n) moderate: at b = 4 that needs lam*dt >= 1 (cond 2e3 there)
    lo, hi = (0.4, 2.0) if m.b <= 3 else (1.0, 3.0)
    t = np.cumsum(rng.uniform(lo, hi, 40) / lam)
    y = rng.standard_normal(40)
    d = dense.gp_dense(m, t, y, want_grad=False)
    lt = btd.btd_literal(m, t, y)
    assert rel(lt["logml"], d["logml"]) < 1e-9
    assert np.abs(lt["f_var"] - d["f_var"]).max() <= 1e-9 * d["f_var"].max()


def test_literal_btd_loses_accuracy_for_tiny_gaps():
    """The reading behind the factored pivots: with lam*dt ~ 5e-3 the literal blocks fail 1e-8."""
    m = model_for([(MATERN52, 0)], [5.0, 2.0, 0.05])
    rng = np.random.default_rng(11)
    t = np.cumsum(rng.uniform(0.005, 0.02, 60))
    y = rng.standard_normal(60)
    d = dense.gp_dense(m, t, y, want_grad=False)
    f = btd.btd_factored(m, t, y)
    assert rel(f["logml"], d["logml"]) < 1e-11
    with np.errstate(all="ignore"):
        try:
            lt = btd.btd_literal(m, t, y)
            err = rel(lt["logml"], d["logml"])
        except np.linalg.LinAlgError:
            err = np.inf
    assert not err < 1e-8


def _adversarial(n, seed, scale=0.5):
    """Exp(scale) gaps with a duplicate time and gaps of 1e-9 and 1e-6."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(scale, n)
    gaps[n // 4] = 0.0
    gaps[n // 2] = 1e-9
    gaps[3 * n // 4] = 1e-6
    return np.cumsum(gaps), rng.standard_normal(n)


def _block_errors(ref, got):
    """Largest errors of the state means and covariance blocks on the scale sqrt(S_ii S_jj)."""
    d = np.sqrt(np.maximum(np.einsum("nii->ni", ref["S_diag"]), 0.0))
    ez = np.max(np.abs(got["z_mean"] - ref["z_mean"]) / (np.abs(ref["z_mean"]) + d))
    es = np.max(np.abs(got["S_diag"] - ref["S_diag"]) / (d[:, :, None] * d[:, None, :]))
    eb = np.max(np.abs(got["S_sub"] - ref["S_sub"]) / (d[1:, :, None] * d[:-1, None, :])) if len(ref["S_sub"]) else 0.0
    return ez, es, eb


@pytest.mark.parametrize("grid", ["plain", "adversarial"])
@pytest.mark.parametrize("name,terms,hyper", CASES)
def test_c_oracle_state_blocks_match_dense_state_posterior(name, terms, hyper, grid):
    """The C elimination's state means, Cov(z_n, z_n | y) and Cov(z_{n+1}, z_n | y) (the
    selected inverse, Sec. 3.1 subproblems 2 and 4) against the dense stacked-state posterior,
    on plain Exp gaps and on gaps with a duplicate time, 1e-9 and 1e-6 (1e-9 on sqrt(S_ii S_jj))."""
    t, y = _adversarial(40, seed=60 + len(name)) if grid == "adversarial" else _data(40, seed=61, span=20.0)
    sp = dense.state_posterior_dense(model_for(terms, hyper), t, y)
    c = native.btd_factored(terms, hyper, t, y)
    errs = _block_errors(sp, c)
    assert max(errs) <= 1e-9, errs


@pytest.mark.parametrize("name,terms,hyper", [c for c in CASES if c[0] in ("m32+per3", "m32+qp3", "se6", "co2")])
def test_c_oracle_state_blocks_match_50_digit_posterior(name, terms, hyper):
    """The wide-state models' blocks against the 50-digit stacked-state posterior (duplicate time
    included)."""
    from oracle import mpref
    rng = np.random.default_rng(62)
    t = np.sort(rng.uniform(0.0, 30.0, 16))
    t[5] = t[4]
    y = rng.standard_normal(16)
    sp = mpref.state_posterior_dense_mp(terms, hyper, t, y)
    c = native.btd_factored(terms, hyper, t, y)
    errs = _block_errors(sp, c)
    assert max(errs) <= 1e-9, errs
    assert rel(c["logml"], sp["logml"]) < 1e-12


@pytest.mark.parametrize("name,terms,hyper", [c for c in CASES if c[0] in ("m52", "m32+per3", "co2")])
def test_c_oracle_state_blocks_match_kalman_rts_long(name, terms, hyper):
    """N = 2000 with duplicate and near-duplicate times: the C elimination's blocks against the
    Python Kalman filter + RTS smoother (written from the filter equations, lag-one covariance
    S_{n+1} G_n^T)."""
    t, y = _adversarial(2000, seed=63, scale=0.05 if name == "co2" else 0.5)
    k = kalman.kf_rts(model_for(terms, hyper), t, y)
    c = native.btd_factored(terms, hyper, t, y)
    errs = _block_errors(k, c)
    assert max(errs) <= 1e-9, errs
    assert rel(c["logml"], k["logml"]) < 1e-11


def test_kalman_rts_matches_factored_btd():
    for name, terms, hyper in CASES:
        m = model_for(terms, hyper)
        t, y = _data(200, seed=5, span=150.0)
        k = kalman.kf_rts(m, t, y)
        f = btd.btd_factored(m, t, y)
        assert rel(k["logml"], f["logml"]) < 1e-11
        s = np.abs(f["S_diag"]).max()
        assert np.abs(k["S_diag"] - f["S_diag"]).max() <= 1e-9 * s
        assert np.abs(k["S_sub"] - f["S_sub"]).max() <= 1e-9 * s


# ----------------------------------------------------------------------------- closed forms
@pytest.mark.parametrize("name,terms,hyper", CASES)
def test_single_point_closed_form(name, terms, hyper):
    """N = 1: y ~ N(0, k(0) + s2), mean = k(0) y/(k(0)+s2), var = k(0) - k(0)^2/(k(0)+s2)."""
    m = model_for(terms, hyper)
    y = np.array([0.731])
    k0 = float(m.kernel(0.0))
    s = k0 + m.noise
    for res in (btd.btd_factored(m, np.array([2.0]), y), native.btd_factored(terms, hyper, [2.0], y)):
        assert rel(res["logml"], -0.5 * np.log(2 * np.pi * s) - 0.5 * y[0] ** 2 / s) < 1e-14
        assert rel(res["f_mean"][0], k0 * y[0] / s) < 1e-14
        assert rel(res["f_var"][0], k0 - k0 * k0 / s) < 1e-13


def test_two_points_by_hand():
    """N = 2: 2x2 covariance [[k0 + s2, k(d)], [k(d), k0 + s2]] written out."""
    terms, hyper = [(MATERN32, 0)], [1.0, 1.0, 0.1]
    m = model_for(terms, hyper)
    t = np.array([0.5, 1.75])
    y = np.array([0.3, -1.1])
    lam = np.sqrt(3.0)
    kd = (1 + lam * 1.25) * np.exp(-lam * 1.25)
    a, c = 1.0 + 0.1, kd
    det = a * a - c * c
    quad = (a * y[0] ** 2 - 2 * c * y[0] * y[1] + a * y[1] ** 2) / det
    ll = -0.5 * quad - 0.5 * np.log(det) - np.log(2 * np.pi)
    mean0 = (1.0 * (a * y[0] - c * y[1]) + kd * (-c * y[0] + a * y[1])) / det
    for res in (btd.btd_factored(m, t, y), native.btd_factored(terms, hyper, t, y)):
        assert rel(res["logml"], ll) < 1e-14
        assert rel(res["f_mean"][0], mean0) < 1e-13


@pytest.mark.parametrize("fx", json.load(open(GOLDEN))["fixtures"], ids=lambda f: f["name"])
def test_against_50_digit_dense_fixtures(fx):
    """Duplicate times, gaps of 1e-9 / 1e-6, zero process noise: factored elimination to 1e-10."""
    terms = [tuple(x) for x in fx["terms"]]
    t, y = np.array(fx["t"]), np.array(fx["y"])
    m = model_for(terms, fx["hyper"])
    for res in (btd.btd_factored(m, t, y), native.btd_factored(terms, fx["hyper"], t, y),
                kalman.kf_rts(m, t, y)):
        assert rel(res["logml"], fx["logml"]) < 1e-10
        v = np.array(fx["f_var"])
        mu = np.array(fx["f_mean"])
        assert np.all(np.abs(res["f_mean"] - mu) <= 1e-9 * (np.abs(mu) + np.sqrt(v)))
        assert np.all(np.abs(res["f_var"] - v) <= 1e-9 * v + 1e-14)


# ----------------------------------------------------------------------------- invariants
@pytest.mark.parametrize("name,terms,hyper", CASES)
def test_time_reversal_and_translation(name, terms, hyper):
    """Stationary, even kernels: reversing time order and shifting t leave logML unchanged."""
    t, y = _data(120, seed=9)
    a = native.btd_factored(terms, hyper, t, y, want_blocks=False)
    r = native.btd_factored(terms, hyper, (-t[::-1]).copy(), y[::-1].copy(), want_blocks=False)
    s = native.btd_factored(terms, hyper, t + 1234.5, y, want_blocks=False)
    assert rel(r["logml"], a["logml"]) < 1e-11
    assert np.allclose(r["f_var"][::-1], a["f_var"], rtol=1e-9)
    assert rel(s["logml"], a["logml"]) < 1e-9


# ----------------------------------------------------------------------------- gradients
@pytest.mark.parametrize("name,terms,hyper", CASES)
def test_gradients_dense_tangent_fd(name, terms, hyper):
    """Dense trace formula = tangent-linear filter (Python and C) = Richardson differences."""
    m = model_for(terms, hyper)
    t, y = _data(60, seed=21, span=40.0)
    gd = dense.gp_dense(m, t, y)["grad"]
    gk = kalman.kf_tangent_grad(m, t, y)["grad"]
    gc = native.tangent_grad(terms, hyper, t, y)["grad"]
    fd = btd.fd_gradient(lambda h: native.btd_factored(terms, h, t, y, want_blocks=False)["logml"], hyper)
    s = np.abs(gd).max()
    assert np.abs(gk - gd).max() <= 1e-9 * s
    assert np.abs(gc - gd).max() <= 1e-9 * s
    assert np.abs(fd - gd).max() <= 1e-6 * s


@pytest.mark.parametrize("name,terms,hyper", CASES[:5])
def test_trace_gradient_eq_dd1_on_comfortable_grid(name, terms, hyper):
    """The paper's route (eq. dd1 + data-fit derivative, BTD part of Kb^-1 only) on safe gaps."""
    m = model_for(terms, hyper)
    lam = m.parts[0].lam
    rng = np.random.default_rng(4)
    lo, hi = (0.5, 2.0) if m.b <= 3 else (1.0, 3.0)
    t = np.cumsum(rng.uniform(lo, hi, 30) / lam)
    y = rng.standard_normal(30)
    gd = dense.gp_dense(m, t, y)["grad"]
    gt = btd.trace_gradient(m, t, y)
    assert np.abs(gt - gd).max() <= 1e-8 * np.abs(gd).max()


# ----------------------------------------------------------------------------- workloads
def test_config1_oracle_against_dense():
    """Workload 1 (Matern-3/2, N = 1000): factored elimination vs dense GP at 1e-9 relative."""
    w = make_config(1)
    t, y, hyp = w.series(0)
    m = model_for(w.terms, hyp)
    d = dense.gp_dense(m, t, y, want_grad=True)
    c = native.btd_factored(w.terms, hyp, t, y, want_blocks=False)
    g = native.tangent_grad(w.terms, hyp, t, y)
    assert rel(c["logml"], d["logml"]) < 1e-9
    assert np.all(np.abs(c["f_mean"] - d["f_mean"]) <= 1e-9 * (np.abs(d["f_mean"]) + np.sqrt(d["f_var"])))
    assert np.all(np.abs(c["f_var"] - d["f_var"]) <= 1e-9 * d["f_var"])
    assert np.abs(g["grad"] - d["grad"]).max() <= 1e-8 * np.abs(d["grad"]).max()


@pytest.mark.parametrize("k,n", [(2, 3000), (3, 1500), (4, None)])
def test_c_oracle_matches_python_oracle_on_workloads(k, n):
    w = make_config(k, n=n) if k != 4 else make_config(4, n_series=3, max_len=700)
    for i in range(w.n_series):
        t, y, hyp = w.series(i)
        m = model_for(w.terms, hyp)
        p = kalman.kf_rts(m, t, y)
        c = native.btd_factored(w.terms, hyp, t, y)
        assert rel(c["logml"], p["logml"]) < 1e-10
        assert np.abs(c["f_var"] - p["f_var"]).max() <= 1e-8 * p["f_var"].max()
        if n is not None and n <= 1500:
            continue
        pg = kalman.kf_tangent_grad(m, t, y)["grad"]
        cg = native.tangent_grad(w.terms, hyp, t, y)["grad"]
        assert np.abs(cg - pg).max() <= 1e-8 * np.abs(pg).max()
