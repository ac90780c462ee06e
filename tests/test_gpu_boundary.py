"""GPU checks of the boundary's error and masking contract (include/spingp.h):

- the gradient mask of spingp_logml_grad writes 0 for masked components and leaves the others
  bitwise unchanged, also through a HIP graph (captured again when the mask changes);
- device-detected data errors poison the outputs they affect with NaN: every output of a
  one-series handle; with several series only the failing series (all of them for invalid
  offsets), the other series still match the oracle; a prediction time that fails its check
  poisons its own series; a clean assemble clears it all.
"""
import numpy as np
import pytest

from gpu_util import check_grad, check_logml, to_dev
from oracle import native
from workloads import KIND_MATERN32, KIND_PERIODIC, make_config

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1610_08035_amd as spg
    spg.load_library()
    return spg


def _offsets(w):
    return to_dev(w.offsets, torch.int64)


def test_gradient_mask_one_series_and_graph(lib):
    w = make_config(2, n=5000)
    t, y, hyp = w.series(0)
    h = lib.Handle(w.terms, t.shape[0])
    h.assemble(to_dev(t), to_dev(y), to_dev(hyp))
    ll, g = h.logml_grad()
    llm, gm = h.logml_grad(mask=[1, 0, 1])
    g, gm = g.cpu().numpy().reshape(-1), gm.cpu().numpy().reshape(-1)
    assert ll.item() == llm.item()
    assert gm[1] == 0.0 and gm[0] == g[0] and gm[2] == g[2]
    h.close()
    # graph replays: a new mask means a new capture, the same mask replays it
    hg = lib.Handle(w.terms, t.shape[0])
    hg.assemble(to_dev(t), to_dev(y), to_dev(hyp), graph=True)
    lld = torch.empty(1, dtype=torch.float64, device="cuda:0")
    gd = torch.empty(1, 3, dtype=torch.float64, device="cuda:0")
    for mask in ([1, 1, 1], [0, 1, 0], [0, 1, 0], None, [1, 1, 0]):
        lib.spingp_logml_grad(hg._h, lld, gd, mask)
        got = gd.cpu().numpy().reshape(-1)
        want = g * (np.ones(3) if mask is None else np.asarray(mask, dtype=float))
        assert np.array_equal(got, want), (mask, got, want)
        assert lld.item() == ll.item()
    hg.close()


def test_gradient_mask_batched_and_wide(lib):
    w = make_config(4, n_series=6, max_len=400)
    h = lib.Handle(w.terms, max_points=w.n_points, max_series=w.n_series)
    h.assemble(to_dev(w.t), to_dev(w.y), to_dev(w.hyper.reshape(-1)), _offsets(w))
    _, g = h.logml_grad()
    _, gm = h.logml_grad(mask=[0, 1, 1])
    g, gm = g.cpu().numpy(), gm.cpu().numpy()
    assert np.all(gm[:, 0] == 0.0) and np.array_equal(gm[:, 1:], g[:, 1:])
    h.close()
    terms = [(KIND_MATERN32, 0), (KIND_PERIODIC, 3)]
    w3 = make_config(3, n=3000)
    t, y, hyp = w3.series(0)
    h = lib.Handle(terms, t.shape[0])
    h.assemble(to_dev(t), to_dev(y), to_dev(hyp))
    _, g = h.logml_grad()
    mask = [1, 1, 0, 0, 1, 1]
    _, gm = h.logml_grad(mask=mask)
    g, gm = g.cpu().numpy().reshape(-1), gm.cpu().numpy().reshape(-1)
    assert np.array_equal(gm, g * np.asarray(mask, dtype=float))
    h.close()


def test_one_series_errors_poison_every_output(lib):
    w = make_config(2, n=3000)
    t, y, hyp = w.series(0)
    h = lib.Handle(w.terms, t.shape[0] + 100)
    bad = hyp.copy()
    bad[0] = -1.0                                           # negative lengthscale
    h.assemble(to_dev(t), to_dev(y), to_dev(bad))
    h.factor()
    ll, fit, ld = h.logml(parts=True)
    fm, zm = h.solve(states=True)
    fv, sd, ss = h.selinv(blocks=True)
    ll2, g = h.logml_grad()
    assert h.status()[0] == 5
    for a in (ll, fit, ld, fm, zm, fv, sd, ss[:, : t.shape[0] - 1], ll2, g):
        assert torch.isnan(a).all()
    # a decreasing time: the same, and prediction outputs too
    t2 = t.copy()
    t2[100] = t2[99] - 1.0
    h.assemble(to_dev(t2), to_dev(y), to_dev(hyp))
    ll2, g = h.logml_grad()
    pm, pv = h.predict(to_dev(np.linspace(t[0], t[-1], 50)))
    assert h.status() == (3, 99)
    assert torch.isnan(ll2).all() and torch.isnan(g).all() and torch.isnan(pm).all() and torch.isnan(pv).all()
    # a clean assemble clears the status word and the outputs are finite again
    h.assemble(to_dev(t), to_dev(y), to_dev(hyp))
    ll2, g = h.logml_grad()
    assert h.status() == (0, -1)
    r = native.tangent_grad(w.terms, hyp, t, y)
    check_logml(ll2.item(), r["logml"])
    check_grad(g.cpu().numpy(), r["grad"])
    h.close()


def test_wide_errors_poison(lib):
    terms = [(KIND_MATERN32, 0), (KIND_PERIODIC, 3)]
    w3 = make_config(3, n=2000)
    t, y, hyp = w3.series(0)
    y2 = y.copy()
    y2[700] = np.nan
    h = lib.Handle(terms, t.shape[0])
    h.assemble(to_dev(t), to_dev(y2), to_dev(hyp))
    ll, g = h.logml_grad()
    fm = h.solve()
    assert h.status() == (4, 700)
    assert torch.isnan(ll).all() and torch.isnan(g).all() and torch.isnan(fm).all()
    h.close()


def test_batched_errors_poison_only_the_failing_series(lib):
    w = make_config(4, n_series=6, max_len=500)
    S = w.n_series
    hyp = w.hyper.copy()
    hyp[4, 1] = 0.0                                         # series 4: signal variance 0
    t = w.t.copy()
    k = int(w.offsets[1]) + 7
    t[k + 1] = t[k] - 0.25                                  # series 1: decreasing time
    t[int(w.offsets[3]) + 2] = np.nan                       # series 3: a non-finite time
    h = lib.Handle(w.terms, max_points=w.n_points + 60, max_series=S)
    h.assemble(to_dev(t), to_dev(w.y), to_dev(hyp.reshape(-1)), _offsets(w))
    ll, g = h.logml_grad()
    h.factor()
    fm = h.solve().cpu().numpy()
    # the status word keeps the smallest (index << 4) | code: a hyperparameter error (index -1)
    # comes before any point error
    assert h.status() == (5, -1)
    ll, g = ll.cpu().numpy(), g.cpu().numpy()
    for s in range(S):
        a, e = int(w.offsets[s]), int(w.offsets[s + 1])
        if s in (1, 3, 4):
            assert np.isnan(ll[s]) and np.isnan(g[s]).all() and np.isnan(fm[a:e]).all()
        else:
            ts, ys, hs = w.series(s)
            r = native.tangent_grad(w.terms, hs, ts, ys)
            check_logml(ll[s], r["logml"])
            check_grad(g[s], r["grad"])
            assert np.isfinite(fm[a:e]).all()
    # the failing series run on neutral stand-in data, so the others are exact: compare their
    # means too
    for s in (0, 2, 5):
        a, e = int(w.offsets[s]), int(w.offsets[s + 1])
        ts, ys, hs = w.series(s)
        r = native.btd_factored(w.terms, hs, ts, ys, want_blocks=False)
        sc = np.abs(r["f_mean"]) + np.sqrt(r["f_var"])
        assert np.max(np.abs(fm[a:e] - r["f_mean"]) / sc) <= 1e-9
    # prediction: a non-finite prediction time of series 2 poisons series 2 as well
    h.assemble(to_dev(w.t), to_dev(w.y), to_dev(w.hyper.reshape(-1)), _offsets(w))
    m = 10
    ts = np.concatenate([np.sort(np.random.default_rng(s).uniform(w.t[int(w.offsets[s])],
                                                                   w.t[int(w.offsets[s + 1]) - 1], m))
                         for s in range(S)])
    ts[2 * m + 3] = np.nan
    os_ = to_dev(np.arange(S + 1, dtype=np.int64) * m, torch.int64)
    pm, pv = h.predict(to_dev(ts), os_)
    pm, pv = pm.cpu().numpy(), pv.cpu().numpy()
    assert h.status()[0] == 4
    for s in range(S):
        sl = slice(s * m, (s + 1) * m)
        if s == 2:
            assert np.isnan(pm[sl]).all() and np.isnan(pv[sl]).all()
        else:
            assert np.isfinite(pm[sl]).all() and np.isfinite(pv[sl]).all()
    # invalid offsets poison every series
    off = w.offsets.copy()
    off[-1] -= 1
    h.assemble(to_dev(w.t), to_dev(w.y), to_dev(w.hyper.reshape(-1)), to_dev(off, torch.int64))
    ll, g = h.logml_grad()
    assert h.status()[0] == 1
    assert torch.isnan(ll).all() and torch.isnan(g).all()
    # a clean assemble clears every flag
    h.assemble(to_dev(w.t), to_dev(w.y), to_dev(w.hyper.reshape(-1)), _offsets(w))
    ll, g = h.logml_grad()
    assert h.status() == (0, -1) and torch.isfinite(ll).all() and torch.isfinite(g).all()
    h.close()
