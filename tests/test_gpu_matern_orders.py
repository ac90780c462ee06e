"""GPU parity of the Matern-1/2 (b = 1) and Matern-7/2 (b = 4) models against the C oracle:
every output (logML and its parts, the three-component gradient, means, variances, state means
and the selected-inverse blocks) on one series at ragged sizes, batches with empty series,
every tile shape, prediction at new times, and the multiplied-out blocks."""
import numpy as np
import pytest

from gpu_util import check_grad, check_logml, compare_series, to_dev
from oracle import kalman, native
from oracle.ssm import model_for
from workloads import KIND_MATERN12, KIND_MATERN72, make_batch

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KINDS = [KIND_MATERN12, KIND_MATERN72]


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1610_08035_amd as spg
    spg.load_library()
    return spg


def _one(kind, n, hyper, seed):
    w = make_batch([n], np.array([hyper]), [(kind, 0)], seed=seed)
    return w.terms, w.t, w.y, w.hyper[0]


def _run(spg, terms, t, y, hyp, tile=None, blocks=True):
    n = t.shape[0]
    h = spg.Handle(terms, n)
    if tile is not None:
        h.tile = tile
    h.assemble(to_dev(t), to_dev(y), to_dev(hyp))
    h.factor()
    ll, fit, ld = h.logml(parts=True)
    fm, zm = h.solve(states=True)
    if blocks:
        fv, sd, ss = h.selinv(blocks=True)
    else:
        fv = h.selinv()
    ll2, g = h.logml_grad()
    out = {"logml": ll.item(), "datafit": fit.item(), "logdet": ld.item(), "f_mean": fm.cpu().numpy(),
           "z_mean": zm.cpu().numpy(), "f_var": fv.cpu().numpy(), "logml2": ll2.item(),
           "grad": g.cpu().numpy().reshape(-1), "status": h.status()[0]}
    if blocks:
        out["S_diag"] = sd.cpu().numpy()
        out["S_sub"] = ss.cpu().numpy()
    assert h.b == (1 if terms[0][0] == KIND_MATERN12 else 4)
    h.close()
    return out


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", [1, 2, 7, 8, 9, 1023, 1025, 5000])
def test_every_output_ragged_sizes(lib, kind, n):
    terms, t, y, hyp = _one(kind, n, [3.0, 1.4, 0.08], seed=100 + n)
    print(f"\nkind {kind} n={n}", flush=True)
    compare_series(terms, t, y, hyp, _run(lib, terms, t, y, hyp))


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("hyper", [[0.4, 2.0, 0.3], [40.0, 0.6, 0.01]])
def test_other_hyperparameters_and_many_work_groups(lib, kind, hyper):
    """Short and long lengthscales at 2^16 points (64 work-groups of the default tile)."""
    terms, t, y, hyp = _one(kind, 1 << 16, hyper, seed=7)
    compare_series(terms, t, y, hyp, _run(lib, terms, t, y, hyp, blocks=False), blocks=False)


@pytest.mark.parametrize("kind", KINDS)
def test_every_tile(lib, kind):
    terms, t, y, hyp = _one(kind, 3001, [2.0, 1.0, 0.1], seed=8)
    for i in range(lib.spingp_tile_count()):
        try:
            compare_series(terms, t, y, hyp, _run(lib, terms, t, y, hyp, tile=i))
        except AssertionError as e:
            raise AssertionError(f"tile {lib.spingp_tile_shape(i)}: {e}") from None


@pytest.mark.parametrize("kind", KINDS)
def test_batched_with_empty_series(lib, kind):
    lens = [0, 1, 2, 9, 0, 700, 1025, 3, 0]
    rng = np.random.default_rng(9)
    S = len(lens)
    hyper = np.stack([np.exp(rng.uniform(np.log(0.5), np.log(20.0), S)),
                      np.exp(rng.uniform(np.log(0.5), np.log(3.0), S)),
                      np.exp(rng.uniform(np.log(1e-3), np.log(0.5), S))], axis=1)
    w = make_batch(lens, hyper, [(kind, 0)], seed=10)
    h = lib.Handle(w.terms, w.n_points, S)
    h.assemble(to_dev(w.t), to_dev(w.y), to_dev(w.hyper.reshape(-1)), to_dev(w.offsets, torch.int64))
    ll, g = h.logml_grad()
    h.factor()
    fm = h.solve()
    fv = h.selinv()
    assert h.status()[0] == 0
    ll, g, fm, fv = ll.cpu().numpy(), g.cpu().numpy(), fm.cpu().numpy(), fv.cpu().numpy()
    for s in range(S):
        t, y, hyp = w.series(s)
        if t.shape[0] == 0:
            assert ll[s] == 0.0 and not np.any(g[s])
            continue
        r = native.btd_factored(w.terms, hyp, t, y, want_blocks=False)
        gr = native.tangent_grad(w.terms, hyp, t, y)
        a, e = int(w.offsets[s]), int(w.offsets[s + 1])
        check_logml(ll[s], r["logml"])
        check_grad(g[s], gr["grad"])
        sc = np.abs(r["f_mean"]) + np.sqrt(r["f_var"])
        assert np.max(np.abs(fm[a:e] - r["f_mean"]) / sc) <= 1e-9, f"series {s}"
        assert np.max(np.abs(fv[a:e] - r["f_var"]) / r["f_var"]) <= 1e-9, f"series {s}"
    h.close()


@pytest.mark.parametrize("kind", KINDS)
def test_predict_against_kalman(lib, kind):
    terms, t, y, hyp = _one(kind, 4000, [2.5, 1.2, 0.05], seed=11)
    rng = np.random.default_rng(12)
    ts = np.sort(np.concatenate([rng.uniform(t[0] - 3.0, t[-1] + 3.0, 700), t[[0, 100, 3999]]]))
    h = lib.Handle(terms, t.shape[0] + ts.shape[0])
    h.assemble(to_dev(t), to_dev(y), to_dev(hyp))
    fm, fv = h.predict(to_dev(ts))
    assert h.status()[0] == 0
    tm = np.concatenate([t, ts])
    ym = np.concatenate([y, np.full(ts.shape[0], np.nan)])
    order = np.lexsort((np.concatenate([np.zeros(t.shape[0]), np.ones(ts.shape[0])]), tm))
    pos = np.empty(tm.shape[0], np.int64)
    pos[order] = np.arange(tm.shape[0])
    k = kalman.kf_rts(model_for(terms, hyp), tm[order], ym[order])
    rm, rv = k["f_mean"][pos[t.shape[0]:]], k["f_var"][pos[t.shape[0]:]]
    fm, fv = fm.cpu().numpy(), fv.cpu().numpy()
    assert np.max(np.abs(fm - rm) / (np.abs(rm) + np.sqrt(rv))) <= 1e-9
    assert np.max(np.abs(fv - rv) / rv) <= 1e-9
    h.close()


@pytest.mark.parametrize("kind", KINDS)
def test_autograd(lib, kind):
    from paper_1610_08035_amd.autograd import logml
    terms, t, y, hyp = _one(kind, 2000, [1.5, 0.9, 0.2], seed=13)
    hy = to_dev(hyp).requires_grad_(True)
    ll = logml(to_dev(t), to_dev(y), hy, terms)
    ll.sum().backward()
    r = native.tangent_grad(terms, hyp, t, y)
    check_logml(ll.item(), r["logml"])
    check_grad(hy.grad.cpu().numpy(), r["grad"])
