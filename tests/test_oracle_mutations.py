"""Planted mistakes in the oracle (on the CPU) must trip its pins.

Each test perturbs one ingredient of the oracle the way a plausible bug
would (a transposed transition, a dropped variance, a sign flip in the
rank-one observation term, a wrong edge index) and checks that the
independent route the pins use disagrees by far more than the tolerance.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import btd, dense, kalman
from oracle.ssm import MATERN32, MATERN52, SumModel, model_for


def _data():
    rng = np.random.default_rng(2)
    t = np.sort(rng.uniform(0.0, 20.0, 40))
    return t, rng.standard_normal(40)


def _logml_gap(m, t, y):
    return abs(btd.btd_factored(m, t, y)["logml"] - dense.gp_dense(m, t, y, want_grad=False)["logml"])


def test_transposed_transition_is_caught(monkeypatch):
    # (for Matern-3/2, A^T with the same P0 and h happens to give the same output
    # covariance, k(tau) = A[tau]_00 either way, so only Matern-5/2 can show it)
    m = model_for([(MATERN52, 0)], [1.5, 1.0, 0.1])
    t, y = _data()
    assert _logml_gap(m, t, y) < 1e-10
    monkeypatch.setattr(SumModel, "A", lambda self, dt: scipy.linalg.expm(self._F * dt).T)
    with np.errstate(all="ignore"):
        gap = _logml_gap(m, t, y)
    assert not gap < 1e-6          # NaN (an indefinite Q) counts as caught


def test_missing_signal_variance_in_P0_is_caught(monkeypatch):
    m = model_for([(MATERN52, 0)], [2.0, 1.7, 0.1])
    t, y = _data()
    orig = SumModel.Pinf
    monkeypatch.setattr(SumModel, "Pinf", lambda self: orig(self) / 1.7)
    h = m.H()
    assert abs(h @ m.A(0.0) @ m.Pinf() @ h - m.kernel(0.0)) > 0.1
    assert _logml_gap(m, t, y) > 1e-3


def test_wrong_edge_index_is_caught():
    """Using A[t_n - t_{n-1}] on edge n (the paper's index clash read the other way) breaks parity."""
    m = model_for([(MATERN32, 0)], [1.0, 1.0, 0.1])
    t, y = _data()
    ref = dense.gp_dense(m, t, y, want_grad=False)["logml"]
    # shift the gaps by one edge
    gaps = np.diff(t)
    t_bad = np.concatenate([[t[0]], t[0] + np.cumsum(np.roll(gaps, 1))])
    assert abs(btd.btd_factored(m, t_bad, y)["logml"] - ref) > 1e-4


def test_noise_as_std_instead_of_variance_is_caught():
    """Reading s2 as a standard deviation (the paper's sigma_n vs sigma_n^2) is far off."""
    m = model_for([(MATERN32, 0)], [1.0, 1.0, 0.1])
    m_bad = model_for([(MATERN32, 0)], [1.0, 1.0, 0.1 ** 2])
    t, y = _data()
    assert abs(kalman.kf_rts(m_bad, t, y)["logml"] - dense.gp_dense(m, t, y, want_grad=False)["logml"]) > 1.0


def test_sign_flip_in_gradient_term_is_caught():
    """Dropping the factor 1/2 or flipping the trace term of eq. dd1 disagrees with differences."""
    terms, hyper = [(MATERN32, 0)], [1.0, 1.0, 0.1]
    m = model_for(terms, hyper)
    t, y = _data()
    g = dense.gp_dense(m, t, y)["grad"]
    fd = btd.fd_gradient(lambda h: btd.btd_factored(model_for(terms, h), t, y)["logml"], hyper)
    assert np.abs(g - fd).max() < 1e-5 * np.abs(g).max()
    assert np.abs(2.0 * g - fd).max() > 1e-2 * np.abs(g).max()
