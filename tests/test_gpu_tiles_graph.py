"""GPU checks of the tile shapes, the autotuner and HIP-graph replay of spingp_logml_grad.

Every tile shape must reproduce the oracle on one series and on a batch; the tuner must pick
a compiled shape and leave results unchanged; graph replays must match eager calls replay
after replay, also after the hyperparameters change in device memory.
"""
import numpy as np
import pytest

from gpu_util import check_grad, check_logml, compare_series, to_dev
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


def _tiles(spg):
    return list(range(spg.spingp_tile_count()))


@pytest.mark.parametrize("n", [1, 3, 1000, 70001])
def test_every_tile_one_series(lib, n):
    w = make_config(2, n=n)
    t, y, hyp = w.series(0)
    for i in _tiles(lib):
        h = lib.Handle(w.terms, n)
        h.tile = i
        h.assemble(to_dev(t), to_dev(y), to_dev(hyp))
        assert h.tile == i
        h.factor()
        ll, fit, ld = h.logml(parts=True)
        fm, zm = h.solve(states=True)
        fv, sd, ss = h.selinv(blocks=True)
        ll2, g = h.logml_grad()
        got = {"logml": ll.item(), "datafit": fit.item(), "logdet": ld.item(), "logml2": ll2.item(),
               "grad": g.cpu().numpy().reshape(-1), "status": h.status()[0], "f_mean": fm.cpu().numpy(),
               "z_mean": zm.cpu().numpy(), "f_var": fv.cpu().numpy(), "S_diag": sd.cpu().numpy(),
               "S_sub": ss.cpu().numpy()}
        try:
            compare_series(w.terms, t, y, hyp, got)
        except AssertionError as e:
            raise AssertionError(f"tile {lib.spingp_tile_shape(i)}: {e}") from None
        h.close()


def test_every_tile_batched(lib):
    w = make_config(4, n_series=30, max_len=1500)
    off = to_dev(w.offsets, torch.int64)
    h = lib.Handle(w.terms, w.n_points, w.n_series)
    for i in _tiles(lib):
        h.tile = i
        h.assemble(to_dev(w.t), to_dev(w.y), to_dev(w.hyper.reshape(-1)), off)
        ll, g = h.logml_grad()
        fm = h.solve()
        fv = h.selinv()
        assert h.status()[0] == 0
        ll, g, fm, fv = ll.cpu().numpy(), g.cpu().numpy(), fm.cpu().numpy(), fv.cpu().numpy()
        for s in range(w.n_series):
            t, y, hyp = w.series(s)
            r = native.btd_factored(w.terms, hyp, t, y)
            gr = native.tangent_grad(w.terms, hyp, t, y)
            a, e = int(w.offsets[s]), int(w.offsets[s + 1])
            check_logml(ll[s], r["logml"])
            check_grad(g[s], gr["grad"])
            sc = np.abs(r["f_mean"]) + np.sqrt(r["f_var"])
            assert np.max(np.abs(fm[a:e] - r["f_mean"]) / sc) <= 1e-9
            assert np.max(np.abs(fv[a:e] - r["f_var"]) / r["f_var"]) <= 1e-9
    h.close()


def test_set_tile_after_assemble_rebinds(lib):
    """Switching the shape of an assembled handle re-maps the bound batch; results agree."""
    w = make_config(4, n_series=12, max_len=800)
    h = lib.Handle(w.terms, w.n_points, w.n_series)
    h.assemble(to_dev(w.t), to_dev(w.y), to_dev(w.hyper.reshape(-1)), to_dev(w.offsets, torch.int64))
    ref_ll, ref_g = [x.cpu().numpy() for x in h.logml_grad()]
    for i in reversed(_tiles(lib)):
        h.tile = i
        ll, g = [x.cpu().numpy() for x in h.logml_grad()]
        assert h.status()[0] == 0
        for s in range(w.n_series):
            check_logml(ll[s], ref_ll[s], tol=1e-12)
            check_grad(g[s], ref_g[s], tol=1e-10)
    h.close()


def test_tune_and_autotune_cache(lib):
    w = make_config(4, n_series=64, max_len=2000)
    args = (to_dev(w.t), to_dev(w.y), to_dev(w.hyper.reshape(-1)), to_dev(w.offsets, torch.int64))
    h = lib.Handle(w.terms, w.n_points, w.n_series)
    h.assemble(*args)
    best = h.tune(reps=2)
    assert 0 <= best < lib.spingp_tile_count()
    ll, g = [x.cpu().numpy() for x in h.logml_grad()]
    # a second handle of the same problem class takes the cached shape without timing
    h2 = lib.Handle(w.terms, w.n_points, w.n_series)
    h2.assemble(*args, autotune=True)
    assert h2.tile == best
    ll2, g2 = [x.cpu().numpy() for x in h2.logml_grad()]
    assert h2.status()[0] == 0
    for s in range(w.n_series):
        t, y, hyp = w.series(s)
        r = native.tangent_grad(w.terms, hyp, t, y)
        check_logml(ll[s], r["logml"])
        check_logml(ll2[s], r["logml"])
        check_grad(g[s], r["grad"])
        check_grad(g2[s], r["grad"])
    h.close()
    h2.close()


def test_autotune_miss_with_bad_input_reports_status(lib):
    """A cache miss on invalid data does not tune; the error is left for spingp_status."""
    w = make_config(2, n=3333)
    t = w.t.copy()
    t[100] = t[99] - 1.0
    h = lib.Handle(w.terms, w.n_points)
    h.assemble(to_dev(t), to_dev(w.y), to_dev(w.hyper.reshape(-1)), autotune=True)
    assert h.status() == (3, 99)
    h.close()


@pytest.mark.parametrize("batched", [False, True])
def test_graph_replays_match_eager(lib, batched):
    """Replays of the captured graph, with eager library and torch work and synchronisations
    between them, each equal the eager result; a hyperparameter update in device memory is
    picked up by the next replay without a new capture."""
    if batched:
        w = make_config(4, n_series=20, max_len=1200)
        off = to_dev(w.offsets, torch.int64)
    else:
        w = make_config(2, n=50000)
        off = None
    t, y = to_dev(w.t), to_dev(w.y)
    hyp = to_dev(w.hyper.reshape(-1))
    S = w.n_series
    eager = lib.Handle(w.terms, w.n_points, S)
    eager.assemble(t, y, hyp, off)
    gh = lib.Handle(w.terms, w.n_points, S)
    gh.assemble(t, y, hyp, off, graph=True)
    ll = torch.empty(S, dtype=torch.float64, device="cuda:0")
    g = torch.empty(S, 3, dtype=torch.float64, device="cuda:0")
    for rep in range(4):
        if rep == 2:
            hyp.mul_(1.1)          # new hyperparameters, same device buffer
        ll.fill_(np.nan)
        g.fill_(np.nan)
        lib.spingp_logml_grad(gh._h, ll, g)
        scratch = torch.randn(1 << 16, dtype=torch.float64, device="cuda:0").sum()   # eager work
        e_ll, e_g = eager.logml_grad()
        torch.cuda.synchronize()
        assert np.isfinite(scratch.item())
        assert torch.equal(ll, e_ll), f"replay {rep}: logML differs from the eager call"
        assert torch.equal(g, e_g), f"replay {rep}: gradient differs from the eager call"
    assert gh.status()[0] == 0
    # the replayed result after the update against the oracle
    hy = hyp.cpu().numpy().reshape(S, 3)
    for s in range(S):
        a, e = int(w.offsets[s]), int(w.offsets[s + 1])
        r = native.tangent_grad(w.terms, hy[s], w.t[a:e], w.y[a:e])
        check_logml(ll[s].item(), r["logml"])
        check_grad(g[s].cpu().numpy(), r["grad"])
    # other output pointers: a new capture
    ll2 = torch.empty_like(ll)
    g2 = torch.empty_like(g)
    lib.spingp_logml_grad(gh._h, ll2, g2)
    torch.cuda.synchronize()
    assert torch.equal(ll2, ll) and torch.equal(g2, g)
    eager.close()
    gh.close()


def test_small_lane_tiles_only_on_small_handles(lib):
    """Shapes with R < 8 need twice the lane workspace: a handle above 2^20 points refuses them
    and its tuner never picks them; a small handle accepts every shape."""
    small = [i for i in _tiles(lib) if lib.spingp_tile_shape(i)[0] < 8]
    assert small, "the library compiles R = 4 shapes"
    w = make_config(2, n=5000)
    t, y, hyp = (to_dev(a) for a in w.series(0))
    big = lib.Handle(w.terms, (1 << 20) + 1)
    for i in small:
        with pytest.raises(lib.SpinGPError):
            big.tile = i
    big.assemble(t, y, hyp)
    assert lib.spingp_tile_shape(big.tune(reps=1))[0] >= 8
    ll_big, g_big = [x.cpu().numpy() for x in big.logml_grad()]
    h = lib.Handle(w.terms, 1 << 20)
    h.assemble(t, y, hyp)
    for i in small:
        h.tile = i
        ll, g = [x.cpu().numpy() for x in h.logml_grad()]
        check_logml(ll.item(), ll_big.item(), tol=1e-12)
        check_grad(g.reshape(-1), g_big.reshape(-1), tol=1e-10)
    big.close()
    h.close()
