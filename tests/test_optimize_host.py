"""Host logic of the hyperparameter optimiser: the scaled conjugate gradient method on
functions with known minimisers (no GPU)."""
import numpy as np
import pytest

from paper_1610_08035_amd.optimize import scg


def _quadratic(A, b):
    def fun(x):
        return 0.5 * x @ A @ x - b @ x, A @ x - b
    return fun


def test_scg_quadratic_reaches_the_solution():
    rng = np.random.default_rng(0)
    M = rng.standard_normal((6, 6))
    A = M @ M.T + 0.5 * np.eye(6)
    b = rng.standard_normal(6)
    x, f, g, info = scg(_quadratic(A, b), np.zeros(6), gtol=1e-12, max_iter=200)
    assert info.converged and info.reason == "gradient"
    assert np.allclose(x, np.linalg.solve(A, b), rtol=0, atol=1e-10)
    # every accepted step lowers the objective (up to its rounding, where steps are judged by
    # the gradient)
    assert all(b_ <= a + 1e-14 * (1 + abs(a)) for a, b_ in zip(info.history, info.history[1:]))


def test_scg_rosenbrock():
    def rosen(x):
        f = 100.0 * (x[1] - x[0] ** 2) ** 2 + (1.0 - x[0]) ** 2
        g = np.array([-400.0 * x[0] * (x[1] - x[0] ** 2) - 2.0 * (1.0 - x[0]), 200.0 * (x[1] - x[0] ** 2)])
        return f, g
    x, f, g, info = scg(rosen, np.array([-1.2, 1.0]), gtol=1e-9, max_iter=5000)
    assert info.converged
    assert np.allclose(x, [1.0, 1.0], atol=1e-6)


def test_scg_negative_curvature_at_the_start():
    """Starting on a concave part (f = x^4 - x^2 near 0) exercises the branch that makes the
    scaled curvature positive; the iteration still descends to a minimiser at +-1/sqrt(2)."""
    def fun(x):
        return float(x[0] ** 4 - x[0] ** 2), np.array([4 * x[0] ** 3 - 2 * x[0]])
    x, f, g, info = scg(fun, np.array([0.05]), gtol=1e-12, max_iter=500)
    assert info.converged
    assert abs(abs(x[0]) - 1 / np.sqrt(2)) < 1e-8
    assert f < fun(np.array([0.05]))[0]


def test_scg_rejects_non_finite_trial_points():
    """A trial point where the objective is not finite is rejected like an uphill step."""
    calls = {"bad": 0}

    def fun(x):
        if x[0] > 3.0:
            calls["bad"] += 1
            return np.inf, np.array([np.nan])
        return float((x[0] - 2.9) ** 2), np.array([2.0 * (x[0] - 2.9)])
    x, f, g, info = scg(fun, np.array([-50.0]), gtol=1e-10, max_iter=1000)
    assert info.converged
    assert abs(x[0] - 2.9) < 1e-8


def test_scg_ftol_and_max_iter():
    A = np.diag([1.0, 1e4])
    x, f, g, info = scg(_quadratic(A, np.array([1.0, 1.0])), np.zeros(2), max_iter=1)
    assert not info.converged and info.reason == "max_iter" and info.n_iter == 1
    x, f, g, info = scg(_quadratic(A, np.array([1.0, 1.0])), np.zeros(2), gtol=0.0, ftol=1e-3,
                        max_iter=100)
    assert info.converged and info.reason == "objective change"


@pytest.mark.parametrize("n", [1, 3, 10])
def test_scg_separable_sum(n):
    """A sum of independent one-dimensional problems (the shape of a batch of series)."""
    c = np.linspace(-2, 2, n)
    w = np.linspace(1, 50, n)

    def fun(x):
        return float(np.sum(w * (np.exp(x) - x * np.exp(c)))), w * (np.exp(x) - np.exp(c))
    x, f, g, info = scg(fun, np.zeros(n), gtol=1e-10, max_iter=2000)
    assert info.converged
    assert np.allclose(x, c, atol=1e-8)


class _OracleHandle:
    """Stands in for a device handle on the CPU: logml_grad reads the bound hyperparameter
    buffer at call time (as the library does) and evaluates the C oracle per series."""

    def __init__(self, terms, n_hyper):
        self.terms, self.n_hyper, self.calls = terms, n_hyper, 0

    def assemble(self, t, y, hyper, offsets=None):
        import numpy as _np
        self.t, self.y, self.hyper = t.numpy(), y.numpy(), hyper
        self.off = _np.array([0, self.t.shape[0]]) if offsets is None else offsets.numpy()

    def status(self):
        return 0, -1

    def logml_grad(self):
        import torch
        from oracle import native
        S = self.off.shape[0] - 1
        hy = self.hyper.numpy().reshape(S, self.n_hyper)
        ll, g = np.zeros(S), np.zeros((S, self.n_hyper))
        for s in range(S):
            a, e = self.off[s], self.off[s + 1]
            if e > a:
                r = native.tangent_grad(self.terms, hy[s], self.t[a:e], self.y[a:e])
                ll[s], g[s] = r["logml"], r["grad"]
        self.calls += 1
        return torch.from_numpy(ll), torch.from_numpy(g)


def test_fit_host_logic_with_the_oracle_in_place_of_the_device():
    """fit() on the CPU through a stand-in handle: log-space search, chain rule, fixed
    components and a batch with an empty series; the result is the oracle's own optimum."""
    torch = pytest.importorskip("torch")
    from scipy.optimize import minimize
    from oracle import native
    from paper_1610_08035_amd.optimize import fit
    from workloads import KIND_MATERN32, make_batch
    lens = [400, 0, 700]
    true = np.array([[2.0, 1.0, 0.1], [1.0, 1.0, 0.1], [5.0, 1.0, 0.2]])
    w = make_batch(lens, true, [(KIND_MATERN32, 0)], seed=41)
    hyper0 = np.tile([1.0, 2.0, 0.5], (3, 1))
    hd = _OracleHandle(w.terms, 3)
    res = fit(torch.from_numpy(w.t), torch.from_numpy(w.y), w.terms, hyper0,
              offsets=torch.from_numpy(w.offsets), fixed=[1], handle=hd)
    assert res.converged, res.reason
    assert np.all(res.hyper[:, 1] == 2.0)
    assert res.logml[1] == 0.0 and np.all(res.hyper[1] == hyper0[1])
    for s in (0, 2):
        t, y, _ = w.series(s)

        def fun(xv):
            th = np.array([np.exp(xv[0]), 2.0, np.exp(xv[1])])
            r = native.tangent_grad(w.terms, th, t, y)
            return -r["logml"], -np.array([r["grad"][0] * th[0], r["grad"][2] * th[2]])
        ref = minimize(fun, np.log([1.0, 0.5]), jac=True, method="L-BFGS-B",
                       options={"gtol": 1e-9 * t.shape[0], "ftol": 1e-15})
        assert np.allclose(np.log(res.hyper[s, [0, 2]]), ref.x, atol=1e-4)
        assert abs(res.logml[s] + ref.fun) <= 1e-9 * abs(ref.fun)
