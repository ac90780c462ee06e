"""GPU parity of the materialised blocks (spingp_blocks): the edge blocks A_n, Q_n and the
multiplied-out posterior-precision blocks D_n, B_n of Theorem 1, against the oracle (closed-form
edges of the C oracle, literal blocks of oracle/btd.py).  Comfortable grids only: D and B need
Q^-1."""
import numpy as np
import pytest

from gpu_util import to_dev
from oracle import btd, native
from oracle.ssm import model_for
from workloads import KIND_MATERN32, KIND_MATERN52

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1610_08035_amd as spg
    spg.load_library()
    return spg


def _grid(n, seed):
    rng = np.random.default_rng(seed)
    return np.cumsum(0.1 + 0.05 * rng.uniform(size=n))


def _unpack(Qp, b):
    n = Qp.shape[1]
    out = np.zeros((n, b, b))
    k = 0
    for i in range(b):
        for j in range(i, b):
            out[:, i, j] = Qp[k]
            out[:, j, i] = Qp[k]
            k += 1
    return out


def _check_series(terms, hyp, t, A, Q, D, Bs, a, e):
    """Blocks of the series occupying [a, e) of the device arrays against the oracle."""
    b = 2 if terms[0][0] == KIND_MATERN32 else 3
    n = e - a
    Ao, Qo, P, h = native.edges(terms, hyp, t)
    Dr, Br = btd.precision_blocks(model_for(terms, hyp), t)
    Ag = A[:, a:e].T.reshape(n, b, b)
    Bg = Bs[:, a:e].T.reshape(n, b, b)
    Qg = _unpack(Q[:, a:e], b)
    Dg = _unpack(D[:, a:e], b)
    sc_p = np.abs(P).max()
    assert np.abs(Ag[: n - 1] - Ao).max() <= 1e-13
    assert np.abs(Qg[: n - 1] - Qo).max() <= 1e-13 * sc_p
    # the series' last node: no edge
    assert not np.any(Ag[n - 1]) and not np.any(Qg[n - 1]) and not np.any(Bg[n - 1])
    # D and B contain Q^-1, whose forward error in any FP64 inverse is about cond(Q) eps: the
    # bar is 1e-9 of the block, or 64 cond(Q) eps where that is larger (Matern-5/2 Q_n at
    # lam dt ~ 0.1 has cond ~ 1e7)
    cq = np.array([np.linalg.cond(Qo[k]) for k in range(n - 1)])
    eps = np.finfo(np.float64).eps
    for k in range(n):
        c = max(cq[k - 1] if k > 0 else 1.0, cq[k] if k < n - 1 else 1.0)
        tol = max(1e-9, 64.0 * c * eps)
        s = np.abs(Dr[k]).max()
        assert np.abs(Dg[k] - Dr[k]).max() <= tol * s, f"D_{k}: tol {tol:.2e}"
    for k in range(n - 1):
        tol = max(1e-9, 64.0 * cq[k] * eps)
        s = np.abs(Br[k]).max()
        assert np.abs(Bg[k] - Br[k]).max() <= tol * s, f"B_{k}: tol {tol:.2e}"


@pytest.mark.parametrize("kind,hyper", [(KIND_MATERN32, [1.0, 1.0, 0.1]), (KIND_MATERN52, [2.0, 1.5, 0.2])])
def test_blocks_one_series(lib, kind, hyper):
    n = 700
    t = _grid(n, 3)
    y = np.sin(t)
    terms = [(kind, 0)]
    hyp = np.array(hyper)
    h = lib.Handle(terms, n)
    h.assemble(to_dev(t), to_dev(y), to_dev(hyp))
    A, Q, D, Bs = (x.cpu().numpy() for x in h.blocks())
    assert h.status()[0] == 0
    _check_series(terms, hyp, t, A, Q, D, Bs, 0, n)
    h.close()


def test_blocks_several_series(lib):
    """Three series with their own hyperparameters; blocks never couple two series."""
    lens = [130, 9, 401]
    ts = [_grid(m, 10 + i) for i, m in enumerate(lens)]
    hyps = np.array([[1.5, 1.0, 0.1], [0.8, 2.0, 0.3], [3.0, 0.5, 0.05]])
    terms = [(KIND_MATERN52, 0)]
    offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    t = np.concatenate(ts)
    y = np.cos(t)
    h = lib.Handle(terms, t.shape[0], max_series=3)
    h.assemble(to_dev(t), to_dev(y), to_dev(hyps.reshape(-1)), to_dev(offsets, torch.int64))
    A, Q, D, Bs = (x.cpu().numpy() for x in h.blocks())
    assert h.status()[0] == 0
    for s in range(3):
        _check_series(terms, hyps[s], ts[s], A, Q, D, Bs, int(offsets[s]), int(offsets[s + 1]))
    h.close()


def test_blocks_order_and_model_errors(lib):
    h = lib.Handle([(KIND_MATERN52, 0)], 10)
    with pytest.raises(lib.SpinGPError):
        h._keep = (torch.zeros(1, dtype=torch.float64, device="cuda:0"),)
        h.n = 10
        h.blocks()                                 # before assemble
    h.close()
    hw = lib.Handle([(1, 0), (3, 3)], 10)
    t = to_dev(np.arange(10.0))
    hw.assemble(t, t, to_dev(np.array([1.0, 1.0, 1.0, 1.0, 5.0, 0.1])))
    with pytest.raises(lib.SpinGPError):
        hw.blocks()                                # the sum kernel has no materialised blocks
    hw.close()
