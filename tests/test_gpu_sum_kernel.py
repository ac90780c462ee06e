"""GPU parity of the sum kernel Matern-3/2 + periodic with 3 harmonics (b = 10, six
hyperparameters: l_M, var_M, l_P, var_P, period, s2) against the C oracle.

The library runs this model on its wide-state path (one wavefront per element operation,
level-by-level reduction over all nodes); the oracle is the same sequential block-tridiagonal
elimination and tangent-linear gradient used for the Matern models.
"""
import numpy as np
import pytest

from gpu_util import check_grad, compare_series, to_dev
from oracle import native
from workloads import make_config

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1610_08035_amd as spg
    spg.load_library()
    return spg


def _run(spg, terms, t, y, hyper, blocks=True, graph=False):
    n = t.shape[0]
    h = spg.Handle(terms, max_points=max(n, 1))
    assert h.b == 10 and h.n_hyper == 6
    td, yd, hd = to_dev(t), to_dev(y), to_dev(hyper)
    h.assemble(td, yd, hd, graph=graph)
    h.factor()
    ll, fit, ld = h.logml(parts=True)
    fm, zm = h.solve(states=True)
    if blocks:
        fv, sd, ss = h.selinv(blocks=True)
    else:
        fv = h.selinv()
    ll2, g = h.logml_grad()
    rc, bad = h.status()
    out = {"logml": ll.item(), "datafit": fit.item(), "logdet": ld.item(), "f_mean": fm.cpu().numpy(),
           "z_mean": zm.cpu().numpy(), "f_var": fv.cpu().numpy(), "logml2": ll2.item(),
           "grad": g.cpu().numpy().reshape(-1), "status": rc}
    if blocks:
        out["S_diag"] = sd.cpu().numpy()
        out["S_sub"] = ss.cpu().numpy()
    h.close()
    return out


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 65, 1000, 4097])
def test_sum_kernel_small(lib, n):
    """Every output, state blocks included, at sizes with ragged levels."""
    w = make_config(3, n=n)
    t, y, hyp = w.series(0)
    print(f"\nsum kernel n={n}", flush=True)
    compare_series(w.terms, t, y, hyp, _run(lib, w.terms, t, y, hyp))


@pytest.mark.parametrize("hyper", [[5.0, 0.5, 0.7, 2.0, 7.0, 0.05], [200.0, 2.0, 3.0, 0.5, 50.0, 0.3]])
def test_sum_kernel_other_hyperparameters(lib, hyper):
    w = make_config(3, n=3000)
    w.hyper = np.array([hyper], dtype=np.float64)
    t, y, hyp = w.series(0)
    print(f"\nsum kernel hyper={hyper}", flush=True)
    compare_series(w.terms, t, y, hyp, _run(lib, w.terms, t, y, hyp))


def test_sum_kernel_duplicate_times(lib):
    w = make_config(3, n=2000)
    t = w.t.copy()
    t[500:505] = t[499]
    w.t = t
    t, y, hyp = w.series(0)
    compare_series(w.terms, t, y, hyp, _run(lib, w.terms, t, y, hyp))


def test_sum_kernel_full_config3(lib):
    """N = 2^18, t uniform on [0, 1e4], period 24: logML, the six-component gradient, means and
    variances at every point."""
    w = make_config(3)
    t, y, hyp = w.series(0)
    print(f"\nsum kernel full n={t.shape[0]}", flush=True)
    compare_series(w.terms, t, y, hyp, _run(lib, w.terms, t, y, hyp, blocks=False), blocks=False)


def test_sum_kernel_graph_replay(lib):
    """Graph replays equal eager calls, also after a hyperparameter update in device memory."""
    w = make_config(3, n=20000)
    t, y = to_dev(w.t), to_dev(w.y)
    hyp = to_dev(w.hyper.reshape(-1))
    eager = lib.Handle(w.terms, w.n_points)
    eager.assemble(t, y, hyp)
    gh = lib.Handle(w.terms, w.n_points)
    gh.assemble(t, y, hyp, graph=True)
    ll = torch.empty(1, dtype=torch.float64, device="cuda:0")
    g = torch.empty(1, 6, dtype=torch.float64, device="cuda:0")
    for rep in range(3):
        if rep == 1:
            hyp.mul_(1.05)
        lib.spingp_logml_grad(gh._h, ll, g)
        e_ll, e_g = eager.logml_grad()
        torch.cuda.synchronize()
        assert torch.equal(ll, e_ll) and torch.equal(g, e_g), f"replay {rep}"
    hy = hyp.cpu().numpy()
    r = native.tangent_grad(w.terms, hy, w.t, w.y)
    assert abs(ll.item() - r["logml"]) <= 1e-8 * abs(r["logml"])
    check_grad(g.cpu().numpy(), r["grad"])
    eager.close()
    gh.close()


def test_sum_kernel_host_errors(lib):
    with pytest.raises(lib.SpinGPError):
        lib.Handle([(1, 0), (3, 3)], 100, max_series=2)       # one series only
    with pytest.raises(lib.SpinGPError):
        lib.Handle([(1, 0), (3, 7)], 100)                     # b = 18 > 16
    with pytest.raises(lib.SpinGPError):
        lib.Handle([(1, 0), (9, 1)], 100)                     # unknown kind
    with pytest.raises(lib.SpinGPError):
        lib.Handle([(4, 0)] * 9, 100)                         # more than 8 terms
    h = lib.Handle([(1, 0), (3, 3)], 100)
    assert lib.spingp_tile_count() >= 1
    with pytest.raises(lib.SpinGPError):
        h.tile = 1                                            # a single schedule
    w = make_config(3, n=50)
    hy = w.hyper.reshape(-1).copy()
    hy[4] = -1.0                                              # period must be positive
    h.assemble(to_dev(w.t), to_dev(w.y), to_dev(hy))
    assert h.status()[0] == 5
    h.close()


def test_sum_kernel_autograd(lib):
    from paper_1610_08035_amd.autograd import logml
    w = make_config(3, n=5000)
    t, y, hyp = w.series(0)
    hy = to_dev(hyp).requires_grad_(True)
    ll = logml(to_dev(t), to_dev(y), hy, w.terms)
    ll.sum().backward()
    r = native.tangent_grad(w.terms, hyp, t, y)
    assert abs(ll.item() - r["logml"]) <= 1e-8 * abs(r["logml"])
    check_grad(hy.grad.cpu().numpy(), r["grad"])
