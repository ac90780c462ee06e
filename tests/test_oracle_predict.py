"""CPU pins of the prediction oracles (latent mean and variance at new times).

gp_predict_dense is the textbook formula; kf_rts with NaN observations is the state-space route
(test times merged into the chain as nodes without an observation).  They must agree with each
other, with the training-time posterior where t* = t, and with the prior far from the data.
"""
import numpy as np
import pytest

from oracle import dense, kalman
from oracle.ssm import model_for
from workloads import KIND_MATERN32, KIND_MATERN52, KIND_PERIODIC, make_config


def _merge(t, y, ts):
    """Training first at equal times, test points as NaN observations; returns merged arrays and
    the merged positions of the test points."""
    tm = np.concatenate([t, ts])
    ym = np.concatenate([y, np.full(ts.shape[0], np.nan)])
    is_test = np.concatenate([np.zeros(t.shape[0], bool), np.ones(ts.shape[0], bool)])
    order = np.lexsort((is_test, tm))
    pos = np.empty(tm.shape[0], np.int64)
    pos[order] = np.arange(tm.shape[0])
    return tm[order], ym[order], pos[t.shape[0]:]


CASES = [
    ([(KIND_MATERN32, 0)], [1.0, 1.0, 0.1]),
    ([(KIND_MATERN52, 0)], [2.0, 1.5, 0.05]),
    ([(KIND_MATERN32, 0), (KIND_PERIODIC, 3)], [5.0, 1.0, 1.0, 0.7, 3.0, 0.1]),
]


@pytest.mark.parametrize("terms,hyper", CASES)
def test_dense_prediction_at_training_times_is_the_posterior(terms, hyper):
    rng = np.random.default_rng(1)
    t = np.sort(rng.uniform(0, 20, 200))
    y = np.sin(t) + 0.3 * rng.standard_normal(200)
    m = model_for(terms, np.array(hyper))
    p = dense.gp_predict_dense(m, t, y, t)
    d = dense.gp_dense(m, t, y, want_grad=False)
    assert np.allclose(p["f_mean"], d["f_mean"], rtol=0, atol=1e-10)
    assert np.allclose(p["f_var"], d["f_var"], rtol=1e-8, atol=1e-12)


def test_dense_prediction_far_from_data_is_the_prior():
    rng = np.random.default_rng(2)
    t = np.sort(rng.uniform(0, 10, 100))
    y = rng.standard_normal(100)
    m = model_for([(KIND_MATERN52, 0)], np.array([1.0, 2.5, 0.1]))
    p = dense.gp_predict_dense(m, t, y, np.array([1e4, -1e4]))
    assert np.max(np.abs(p["f_mean"])) < 1e-12
    assert np.allclose(p["f_var"], 2.5, rtol=1e-12)


@pytest.mark.parametrize("terms,hyper", CASES)
def test_state_space_prediction_matches_dense(terms, hyper):
    rng = np.random.default_rng(3)
    t = np.sort(rng.uniform(0, 30, 300))
    y = np.cos(0.5 * t) + 0.2 * rng.standard_normal(300)
    # test times: inside, at training times (ties), before and after the data
    ts = np.sort(np.concatenate([rng.uniform(-2, 32, 45), t[[3, 77, 150]], [t[0], t[-1]]]))
    m = model_for(terms, np.array(hyper))
    tm, ym, pos = _merge(t, y, ts)
    k = kalman.kf_rts(m, tm, ym)
    p = dense.gp_predict_dense(m, t, y, ts)
    scale = np.abs(p["f_mean"]) + np.sqrt(p["f_var"])
    assert np.max(np.abs(k["f_mean"][pos] - p["f_mean"]) / scale) < 1e-9
    assert np.max(np.abs(k["f_var"][pos] - p["f_var"]) / p["f_var"]) < 1e-9
    # nodes without observations add nothing to the likelihood
    k0 = kalman.kf_rts(m, t, y)
    assert abs(k["logml"] - k0["logml"]) < 1e-10 * abs(k0["logml"])


def test_merge_orders_training_before_test_at_equal_times():
    t = np.array([0.0, 1.0, 2.0])
    ts = np.array([1.0, 1.0, 3.0])
    tm, ym, pos = _merge(t, np.zeros(3), ts)
    assert list(tm) == [0.0, 1.0, 1.0, 1.0, 2.0, 3.0]
    assert list(pos) == [2, 3, 5]
    assert np.isnan(ym[pos]).all() and not np.isnan(np.delete(ym, pos)).any()
