"""GPU parity of spingp_predict (latent mean and variance at new times) against the oracle:
the dense predictive formulas on small problems, the Kalman oracle with the prediction times
merged as unobserved nodes on larger ones."""
import numpy as np
import pytest

from gpu_util import TOL_MEAN, TOL_VAR, to_dev
from oracle import dense, kalman, native
from oracle.ssm import model_for
from workloads import KIND_MATERN32, KIND_MATERN52, KIND_PERIODIC, make_config

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1610_08035_amd as spg
    spg.load_library()
    return spg


def _check(fm, fv, ref_m, ref_v, widen=1.0):
    scale = np.abs(ref_m) + np.sqrt(ref_v)
    em = np.max(np.abs(fm - ref_m) / scale)
    ev = np.max(np.abs(fv - ref_v) / ref_v)
    assert em <= TOL_MEAN * widen, f"mean {em:.3e}"
    assert ev <= TOL_VAR * widen, f"variance {ev:.3e}"


CASES = [
    ([(KIND_MATERN32, 0)], [1.0, 1.0, 0.1]),
    ([(KIND_MATERN52, 0)], [2.0, 1.5, 0.05]),
    ([(KIND_MATERN32, 0), (KIND_PERIODIC, 3)], [5.0, 1.0, 1.0, 0.7, 3.0, 0.1]),
]


@pytest.mark.parametrize("terms,hyper", CASES)
def test_predict_small_against_dense(lib, terms, hyper):
    rng = np.random.default_rng(5)
    n = 400
    t = np.sort(rng.uniform(0, 40, n))
    y = np.sin(0.7 * t) + 0.3 * rng.standard_normal(n)
    # inside the data, on training times (ties), before and after it
    ts = np.sort(np.concatenate([rng.uniform(-3, 43, 90), t[[0, 10, 200, n - 1]]]))
    hyp = np.array(hyper)
    h = lib.Handle(terms, n + ts.shape[0])
    h.assemble(to_dev(t), to_dev(y), to_dev(hyp))
    fm, fv = h.predict(to_dev(ts))
    assert h.status()[0] == 0
    ref = dense.gp_predict_dense(model_for(terms, hyp), t, y, ts)
    _check(fm.cpu().numpy(), fv.cpu().numpy(), ref["f_mean"], ref["f_var"])
    h.close()


@pytest.mark.parametrize("kind", [KIND_MATERN32, KIND_MATERN52])
def test_predict_large_against_kalman(lib, kind):
    """2^16 training points, 2^13 prediction times, several tree levels and ragged tails."""
    w = make_config(2 if kind == KIND_MATERN52 else 1, n=1 << 16)
    t, y, hyp = w.series(0)
    rng = np.random.default_rng(6)
    ts = np.sort(rng.uniform(t[0] - 5.0, t[-1] + 5.0, 1 << 13))
    h = lib.Handle(w.terms, t.shape[0] + ts.shape[0])
    h.assemble(to_dev(t), to_dev(y), to_dev(hyp))
    fm, fv = h.predict(to_dev(ts))
    assert h.status()[0] == 0
    # state-space oracle: prediction times merged as unobserved nodes, training first at ties
    tm = np.concatenate([t, ts])
    ym = np.concatenate([y, np.full(ts.shape[0], np.nan)])
    order = np.lexsort((np.concatenate([np.zeros(t.shape[0]), np.ones(ts.shape[0])]), tm))
    pos = np.empty(tm.shape[0], np.int64)
    pos[order] = np.arange(tm.shape[0])
    k = kalman.kf_rts(model_for(w.terms, hyp), tm[order], ym[order])
    _check(fm.cpu().numpy(), fv.cpu().numpy(), k["f_mean"][pos[t.shape[0]:]], k["f_var"][pos[t.shape[0]:]])
    h.close()


def test_predict_at_training_times_is_the_posterior(lib):
    w = make_config(2, n=3000)
    t, y, hyp = w.series(0)
    h = lib.Handle(w.terms, 2 * t.shape[0])
    h.assemble(to_dev(t), to_dev(y), to_dev(hyp))
    fm, fv = h.predict(to_dev(t))
    ref = native.btd_factored(w.terms, hyp, t, y, want_blocks=False)
    _check(fm.cpu().numpy(), fv.cpu().numpy(), ref["f_mean"], ref["f_var"])
    h.close()


def test_handle_works_after_predict(lib):
    """predict overwrites the factorisation; logml_grad refactors, factor + solve work again."""
    w = make_config(2, n=5000)
    t, y, hyp = w.series(0)
    h = lib.Handle(w.terms, 6000)
    h.assemble(to_dev(t), to_dev(y), to_dev(hyp))
    h.predict(to_dev(np.linspace(t[0], t[-1], 700)))
    ll, g = h.logml_grad()
    r = native.tangent_grad(w.terms, hyp, t, y)
    assert abs(ll.item() - r["logml"]) <= 1e-8 * abs(r["logml"])
    h.factor()
    fm = h.solve()
    ref = native.btd_factored(w.terms, hyp, t, y, want_blocks=False)
    assert np.max(np.abs(fm.cpu().numpy() - ref["f_mean"]) / (np.abs(ref["f_mean"]) + np.sqrt(ref["f_var"]))) <= 1e-9
    h.close()


def test_predict_errors(lib):
    w = make_config(2, n=200)
    t, y, hyp = w.series(0)
    h = lib.Handle(w.terms, 300)
    h.assemble(to_dev(t), to_dev(y), to_dev(hyp))
    with pytest.raises(lib.SpinGPError):
        h.predict(to_dev(np.linspace(0, 10, 101)))          # 200 + 101 > max_points
    ts = np.linspace(0, 10, 50)
    ts[20] = ts[19] - 1.0
    h.predict(to_dev(ts))
    assert h.status() == (3, 19)                             # unsorted prediction times
    h.close()
    wb = make_config(4, n_series=3, max_len=50)
    hb = lib.Handle(wb.terms, 1000, max_series=3)
    hb.assemble(to_dev(wb.t), to_dev(wb.y), to_dev(wb.hyper.reshape(-1)), to_dev(wb.offsets, torch.int64))
    with pytest.raises(lib.SpinGPError):
        hb.predict(to_dev(np.linspace(0, 10, 5)))            # several series
    hb.close()
