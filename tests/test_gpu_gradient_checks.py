"""The device gradient of logML against two routes that do not go through the oracle's
tangent-linear filter: Richardson-extrapolated central differences of the device's own logML
(per-lane path b = 3, wide path b = 10 and b = 16), and the paper's trace formula (Sec. 2.4,
eq. dd1 with the data-fit derivative, from the oracle's selected inverse) on a grid with
comfortable gaps, where that formula's Q^-1 is well conditioned."""
import numpy as np
import pytest

from gpu_util import to_dev
from oracle import btd
from oracle.ssm import model_for
from workloads import KIND_MATERN32, KIND_MATERN52, KIND_PERIODIC, KIND_QUASIPERIODIC, KIND_SQEXP
from workloads.generate import make_series

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [
    ("matern52", [(KIND_MATERN52, 0)], [5.0, 2.0, 0.05], 2000, 1500.0),
    ("matern32+periodic3", [(KIND_MATERN32, 0), (KIND_PERIODIC, 3)], [50.0, 1.0, 1.2, 0.8, 24.0, 0.1], 2000, 400.0),
    ("co2_three_terms", [(KIND_MATERN32, 0), (KIND_QUASIPERIODIC, 3), (KIND_SQEXP, 6)],
     [0.8, 0.3, 1.0, 4.0, 1.0, 60.0, 8.0, 20.0, 0.05], 1500, 30.0),
]


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1610_08035_amd as spg
    spg.load_library()
    return spg


@pytest.mark.parametrize("name,terms,hyper,n,span", CASES, ids=[c[0] for c in CASES])
def test_gradient_against_central_differences_of_device_logml(lib, name, terms, hyper, n, span):
    rng = np.random.default_rng(31)
    t = np.sort(rng.uniform(0.0, span, n))
    hyp = np.asarray(hyper, dtype=np.float64)
    y = make_series(t, terms, hyp, rng)
    h = lib.Handle(terms, n)
    hd = to_dev(hyp)
    h.assemble(to_dev(t), to_dev(y), hd)
    ll, g = h.logml_grad()
    g = g.cpu().numpy().reshape(-1)
    assert h.status()[0] == 0

    def logml_at(row):
        hd.copy_(torch.from_numpy(np.asarray(row, dtype=np.float64)))
        v, _ = h.logml_grad()
        return float(v.item())

    fd = btd.fd_gradient(logml_at, hyp)
    h.close()
    scale = np.abs(g).max()
    err = np.abs(fd - g).max() / scale
    print(f"\n{name}: max |FD - grad| / max|grad| = {err:.2e}", flush=True)
    assert err <= 1e-6, (fd, g)


def test_gradient_against_trace_formula_on_comfortable_grid(lib):
    terms = [(KIND_MATERN52, 0)]
    hyp = np.array([5.0, 2.0, 0.05])
    m = model_for(terms, hyp)
    rng = np.random.default_rng(4)
    t = np.cumsum(rng.uniform(0.5, 2.0, 40) / m.parts[0].lam)
    y = rng.standard_normal(40)
    gt = btd.trace_gradient(m, t, y)
    h = lib.Handle(terms, t.shape[0])
    h.assemble(to_dev(t), to_dev(y), to_dev(hyp))
    _, g = h.logml_grad()
    g = g.cpu().numpy().reshape(-1)
    h.close()
    assert np.abs(g - gt).max() <= 1e-8 * np.abs(gt).max(), (g, gt)
