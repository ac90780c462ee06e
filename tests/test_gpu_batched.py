"""GPU parity of the batched path: many independent series of uneven length in one launch.

The library concatenates the series into one chain whose step out of each series' last point
has A = 0 and carries the next series' prior, so the chain splits into independent pieces.
Every series is compared with the C oracle run on that series alone; empty series must give
logML 0 and a zero gradient.
"""
import numpy as np
import pytest

from gpu_util import check_grad, check_logml, compare_series, to_dev
from oracle import native
from workloads import KIND_MATERN32, KIND_MATERN52, make_batch, make_config

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


def _run_batch(spg, w, blocks=True, max_points=None, max_series=None):
    h = spg.Handle(w.terms, max_points=max_points or max(w.n_points, 1), max_series=max_series or w.n_series)
    h.assemble(to_dev(w.t), to_dev(w.y), to_dev(w.hyper.reshape(-1)), _offsets(w))
    h.factor()
    ll, fit, ld = h.logml(parts=True)
    fm, zm = h.solve(states=True)
    if blocks:
        fv, sd, ss = h.selinv(blocks=True)
    else:
        fv = h.selinv()
    ll2, g = h.logml_grad()
    rc, bad = h.status()
    torch.cuda.synchronize()
    out = {"logml": ll.cpu().numpy(), "datafit": fit.cpu().numpy(), "logdet": ld.cpu().numpy(),
           "f_mean": fm.cpu().numpy(), "z_mean": zm.cpu().numpy(), "f_var": fv.cpu().numpy(),
           "logml2": ll2.cpu().numpy(), "grad": g.cpu().numpy(), "status": rc, "bad": bad}
    if blocks:
        out["S_diag"] = sd.cpu().numpy()
        out["S_sub"] = ss.cpu().numpy()
    h.close()
    return out


def _series_view(got, s, a, e, blocks):
    v = {"logml": got["logml"][s], "logml2": got["logml2"][s], "datafit": got["datafit"][s],
         "logdet": got["logdet"][s], "grad": got["grad"][s], "status": got["status"],
         "f_mean": got["f_mean"][a:e], "f_var": got["f_var"][a:e], "z_mean": got["z_mean"][:, a:e]}
    if blocks:
        v["S_diag"] = got["S_diag"][:, a:e]
        v["S_sub"] = got["S_sub"][:, a:e]
    return v


def _compare_batch(w, got, blocks=True, series=None):
    assert got["status"] == 0, f"device status {got['status']} at {got['bad']}"
    for s in (range(w.n_series) if series is None else series):
        a, e = int(w.offsets[s]), int(w.offsets[s + 1])
        if e == a:
            assert got["logml"][s] == 0.0 and got["logml2"][s] == 0.0
            assert not np.any(got["grad"][s])
            continue
        t, y, hyp = w.series(s)
        try:
            compare_series(w.terms, t, y, hyp, _series_view(got, s, a, e, blocks), blocks=blocks)
        except AssertionError as err:
            raise AssertionError(f"series {s} (points {a}..{e}): {err}") from None


def test_batched_config4_subset(lib):
    """48 series of the batched workload's length / lengthscale / noise distribution, cut at 700."""
    w = make_config(4, n_series=48, max_len=700)
    _compare_batch(w, _run_batch(lib, w))


@pytest.mark.parametrize("kind", [KIND_MATERN32, KIND_MATERN52])
def test_batched_ragged_and_empty_series(lib, kind):
    """Leading, inner and trailing empty series; lengths 1, 2, R - 1, R, R + 1, work-group and
    multi-work-group sizes; per-series hyperparameters that differ widely."""
    lens = [0, 1, 2, 7, 8, 9, 0, 0, 1, 1023, 1024, 1025, 3, 64, 65, 5000, 1, 0]
    rng = np.random.default_rng(11)
    S = len(lens)
    hyper = np.stack([np.exp(rng.uniform(np.log(0.3), np.log(30.0), S)),
                      np.exp(rng.uniform(np.log(0.5), np.log(3.0), S)),
                      np.exp(rng.uniform(np.log(1e-3), np.log(0.5), S))], axis=1)
    w = make_batch(lens, hyper, [(kind, 0)], seed=12)
    _compare_batch(w, _run_batch(lib, w))


def test_batched_many_short_series(lib):
    """2000 series of 1..40 points: most chunks are partial and many work-groups hold dozens of
    series boundaries."""
    rng = np.random.default_rng(13)
    lens = rng.integers(1, 41, 2000)
    hyper = np.stack([np.exp(rng.uniform(np.log(0.5), np.log(20.0), 2000)), np.ones(2000),
                      rng.uniform(0.01, 0.5, 2000)], axis=1)
    w = make_batch(lens, hyper, [(KIND_MATERN52, 0)], seed=14)
    got = _run_batch(lib, w, blocks=False)
    _compare_batch(w, got, blocks=False, series=range(0, 2000, 7))
    # logML and gradient of every series
    for s in range(2000):
        t, y, hyp = w.series(s)
        r = native.tangent_grad(w.terms, hyp, t, y)
        check_logml(got["logml2"][s], r["logml"])
        check_grad(got["grad"][s], r["grad"])


def test_batched_matches_one_series_handles(lib):
    """The same series through one batched handle and through one single-series handle each."""
    w = make_config(4, n_series=6, max_len=3000)
    got = _run_batch(lib, w, blocks=False)
    for s in range(w.n_series):
        t, y, hyp = w.series(s)
        h = lib.Handle(w.terms, t.shape[0])
        h.assemble(to_dev(t), to_dev(y), to_dev(hyp))
        ll, g = h.logml_grad()
        h.factor()
        fm = h.solve()
        fv = h.selinv()
        a, e = int(w.offsets[s]), int(w.offsets[s + 1])
        check_logml(got["logml2"][s], ll.item(), tol=1e-12)
        check_grad(got["grad"][s], g.cpu().numpy().reshape(-1), tol=1e-10)
        sc = np.abs(fm.cpu().numpy()) + np.sqrt(fv.cpu().numpy())
        assert np.max(np.abs(got["f_mean"][a:e] - fm.cpu().numpy()) / sc) <= 1e-11
        assert np.max(np.abs(got["f_var"][a:e] - fv.cpu().numpy()) / fv.cpu().numpy()) <= 1e-11
        h.close()


def test_batched_handle_reuse_smaller_batch(lib):
    """One handle sized for a large batch, assembled with a smaller one, then the large one."""
    big = make_config(4, n_series=40, max_len=900)
    small = make_config(4, n_series=5, max_len=200)
    h = lib.Handle(big.terms, max_points=big.n_points, max_series=big.n_series)
    for w in (small, big, small):
        h.assemble(to_dev(w.t), to_dev(w.y), to_dev(w.hyper.reshape(-1)), _offsets(w))
        ll, g = h.logml_grad()
        assert h.status()[0] == 0
        ll, g = ll.cpu().numpy(), g.cpu().numpy()
        for s in range(w.n_series):
            t, y, hyp = w.series(s)
            r = native.tangent_grad(w.terms, hyp, t, y)
            check_logml(ll[s], r["logml"])
            check_grad(g[s], r["grad"])
    h.close()


def test_batched_full_config4(lib):
    """The full batched workload (4096 series, lengths log-uniform in [64, 16384], about 1.2e7
    points): logML and gradient of every series; means and variances of every 64th series."""
    w = make_config(4)
    got = _run_batch(lib, w, blocks=False)
    assert got["status"] == 0
    for s in range(w.n_series):
        t, y, hyp = w.series(s)
        r = native.tangent_grad(w.terms, hyp, t, y)
        check_logml(got["logml2"][s], r["logml"])
        check_logml(got["logml"][s], r["logml"])
        check_grad(got["grad"][s], r["grad"])
    _compare_batch(w, got, blocks=False, series=range(0, w.n_series, 64))


def test_batched_status_codes(lib):
    w = make_config(4, n_series=8, max_len=300)
    h = lib.Handle(w.terms, max_points=w.n_points, max_series=w.n_series)
    hyp = to_dev(w.hyper.reshape(-1))
    # times restart at every series boundary: not an error
    h.assemble(to_dev(w.t), to_dev(w.y), hyp, _offsets(w))
    assert h.status() == (0, -1)
    # decreasing time inside series 3
    t = w.t.copy()
    k = int(w.offsets[3]) + 10
    t[k + 1] = t[k] - 0.5
    h.assemble(to_dev(t), to_dev(w.y), hyp, _offsets(w))
    assert h.status() == (3, k)
    # non-finite observation in the last series
    y = w.y.copy()
    k = int(w.offsets[7]) + 4
    y[k] = np.inf
    h.assemble(to_dev(w.t), to_dev(y), hyp, _offsets(w))
    assert h.status() == (4, k)
    # non-positive noise variance of series 5
    hy = w.hyper.copy()
    hy[5, 2] = 0.0
    h.assemble(to_dev(w.t), to_dev(w.y), to_dev(hy.reshape(-1)), _offsets(w))
    assert h.status()[0] == 5
    # offsets that do not end at n_points, and decreasing offsets
    off = w.offsets.copy()
    off[-1] -= 1
    h.assemble(to_dev(w.t), to_dev(w.y), hyp, to_dev(off, torch.int64))
    assert h.status()[0] == 1
    off = w.offsets.copy()
    off[4] = off[2] - 1
    h.assemble(to_dev(w.t), to_dev(w.y), hyp, to_dev(off, torch.int64))
    assert h.status()[0] == 1
    # and back to a valid batch
    h.assemble(to_dev(w.t), to_dev(w.y), hyp, _offsets(w))
    ll, g = h.logml_grad()
    assert h.status() == (0, -1)
    h.close()


def test_batched_host_errors(lib):
    w = make_config(4, n_series=4, max_len=100)
    h = lib.Handle(w.terms, max_points=w.n_points, max_series=3)
    with pytest.raises(lib.SpinGPError):   # more series than the handle was created for
        h.assemble(to_dev(w.t), to_dev(w.y), to_dev(w.hyper.reshape(-1)), _offsets(w))
    h.close()
    h = lib.Handle(w.terms, max_points=w.n_points, max_series=4)
    with pytest.raises(lib.SpinGPError):   # several series need offsets
        lib.spingp_assemble(h._h, to_dev(w.t), to_dev(w.y), to_dev(w.hyper.reshape(-1)), None, 4)
    h.close()


def test_autograd_batched(lib):
    """The autograd function over a batch: per-series logML, gradient of a weighted sum."""
    from paper_1610_08035_amd.autograd import logml
    w = make_config(4, n_series=10, max_len=600)
    hy = to_dev(w.hyper).requires_grad_(True)
    ll = logml(to_dev(w.t), to_dev(w.y), hy, w.terms, to_dev(w.offsets, torch.int64))
    wts = torch.arange(1, 11, dtype=torch.float64, device="cuda:0")
    (wts * ll).sum().backward()
    g = hy.grad.cpu().numpy()
    for s in range(w.n_series):
        t, y, hyp = w.series(s)
        r = native.tangent_grad(w.terms, hyp, t, y)
        check_logml(ll[s].item(), r["logml"])
        check_grad(g[s] / (s + 1), r["grad"])
