"""Pins of the oracle's state-space models against closed forms (Sec. 2.1)."""
import numpy as np
import pytest
import scipy.linalg

from oracle import native
from oracle.ssm import (MATERN12, MATERN32, MATERN52, MATERN72, PERIODIC, QUASIPERIODIC, SQEXP, Matern, Periodic,
                        SquaredExponential, model_for)

MODELS = [
    ([(MATERN32, 0)], [1.0, 1.0, 0.1]),
    ([(MATERN32, 0)], [0.3, 2.5, 0.1]),
    ([(MATERN52, 0)], [5.0, 2.0, 0.05]),
    ([(MATERN52, 0)], [0.7, 0.4, 0.2]),
    ([(PERIODIC, 3)], [1.0, 1.0, 24.0, 0.1]),
    ([(PERIODIC, 2)], [0.6, 1.7, 3.0, 0.1]),
    ([(MATERN32, 0), (PERIODIC, 3)], [50.0, 1.0, 1.0, 1.0, 24.0, 0.1]),
    ([(MATERN52, 0), (MATERN32, 0)], [3.0, 1.2, 0.8, 0.5, 0.3]),
    ([(MATERN12, 0)], [1.5, 0.8, 0.1]),
    ([(MATERN72, 0)], [4.0, 1.5, 0.05]),
    ([(MATERN72, 0)], [0.6, 0.9, 0.2]),
    ([(QUASIPERIODIC, 3)], [1.0, 1.0, 24.0, 50.0, 0.1]),
    ([(MATERN32, 0), (QUASIPERIODIC, 3)], [50.0, 1.0, 1.2, 0.8, 6.0, 15.0, 0.1]),
    ([(SQEXP, 6)], [1.3, 0.7, 0.1]),
    ([(MATERN32, 0), (QUASIPERIODIC, 3), (SQEXP, 6)], [50.0, 1.0, 1.2, 0.8, 6.0, 15.0, 2.0, 0.5, 0.1]),
]
TAUS = np.array([0.0, 1e-9, 1e-4, 0.01, 0.3, 1.0, 2.7, 10.0, 55.0])


@pytest.mark.parametrize("terms,hyper", MODELS)
def test_state_space_reproduces_kernel(terms, hyper):
    """h^T expm(F tau) P0 h equals the closed-form covariance k(tau) (stationary SSM)."""
    m = model_for(terms, hyper)
    h, P = m.H(), m.Pinf()
    for tau in TAUS:
        k_ssm = h @ m.A(tau) @ P @ h
        assert abs(k_ssm - m.kernel(tau)) <= 1e-13 * max(1.0, abs(m.kernel(0.0)))


def test_matern_kernel_values_closed_form():
    """Textbook Matern values (l=1, var=1): nu=3/2 at tau=1 is 2 e^-sqrt3; nu=5/2 is (1+sqrt5+5/3) e^-sqrt5."""
    assert Matern(MATERN32, 1.0, 1.0).kernel(1.0) == pytest.approx((1 + np.sqrt(3)) * np.exp(-np.sqrt(3)), rel=1e-15)
    assert Matern(MATERN52, 1.0, 1.0).kernel(1.0) == pytest.approx(
        (1 + np.sqrt(5) + 5.0 / 3.0) * np.exp(-np.sqrt(5)), rel=1e-15)
    # nu = 1/2: the exponential kernel; nu = 7/2: (1 + r + 2 r^2/5 + r^3/15) e^-r, r = sqrt7 tau / l
    assert Matern(MATERN12, 1.0, 1.0).kernel(1.0) == pytest.approx(np.exp(-1.0), rel=1e-15)
    r7 = np.sqrt(7.0)
    assert Matern(MATERN72, 1.0, 1.0).kernel(1.0) == pytest.approx(
        (1 + r7 + 2.0 * 7.0 / 5.0 + 7.0 * r7 / 15.0) * np.exp(-r7), rel=1e-15)
    # paper eq. ss_matern: P0 = diag(1, 3/l^2) for unit variance
    assert np.allclose(Matern(MATERN32, 2.0, 1.0).Pinf(), np.diag([1.0, 3.0 / 4.0]), rtol=0, atol=1e-15)


@pytest.mark.parametrize("kind,ell,var", [(MATERN32, 1.0, 1.0), (MATERN32, 0.4, 3.0), (MATERN52, 5.0, 2.0),
                                          (MATERN52, 0.5, 0.7), (MATERN12, 0.8, 1.3), (MATERN72, 3.0, 1.1),
                                          (MATERN72, 0.45, 0.6)])
def test_matern_lyapunov(kind, ell, var):
    """Stationary covariance solves F P0 + P0 F^T + L q L^T = 0 with L = e_b: only the last entry is nonzero."""
    m = Matern(kind, ell, var)
    R = m.F() @ m.Pinf() + m.Pinf() @ m.F().T
    b = m.b
    mask = np.ones((b, b), bool)
    mask[b - 1, b - 1] = False
    if mask.any():
        assert np.abs(R[mask]).max() <= 1e-13 * np.abs(R).max()
    assert R[b - 1, b - 1] < 0
    # q matches the Matern spectral density at 0: var * 2 sqrt(pi) Gamma(nu+1/2)/Gamma(nu) (2 nu)^nu / l^(2 nu)
    nu = m.b - 0.5
    from scipy.special import gamma
    q = var * 2.0 * np.sqrt(np.pi) * gamma(nu + 0.5) / gamma(nu) * (2 * nu) ** nu / ell ** (2 * nu)
    assert -R[b - 1, b - 1] == pytest.approx(q, rel=1e-12)


@pytest.mark.parametrize("terms,hyper", MODELS)
def test_group_property_and_Q(terms, hyper):
    """A[a] A[b] = A[a + b] (Sec. 2.1); Q[0] = 0; Q[dt] is PSD; Q -> P0 for long gaps."""
    m = model_for(terms, hyper)
    for a, b in [(0.1, 0.2), (1.0, 3.5), (0.0, 2.0), (7.0, 11.0)]:
        assert np.allclose(m.A(a) @ m.A(b), m.A(a + b), rtol=1e-12, atol=1e-13)
    assert np.abs(m.Q(0.0)).max() == 0.0
    for dt in [1e-6, 0.01, 0.5, 3.0]:
        w = np.linalg.eigvalsh(m.Q(dt))
        assert w.min() >= -1e-13 * np.abs(m.Pinf()).max()
    if all(k != PERIODIC for k, _ in terms):
        assert np.allclose(m.Q(1e4), m.Pinf(), rtol=0, atol=1e-12 * np.abs(m.Pinf()).max())


def test_periodic_noise_is_zero_and_weights_sum_to_one():
    p = Periodic(3, 1.0, 1.0, 24.0)
    for dt in [0.3, 5.0, 100.0]:
        A = scipy.linalg.expm(p.F() * dt)
        assert np.abs(p.Pinf() - A @ p.Pinf() @ A.T).max() <= 1e-14
    # sum over all harmonics of q_j^2 is e^-z (I_0 + 2 sum I_j) = 1
    assert Periodic(60, 1.0, 1.0, 24.0).q2().sum() == pytest.approx(1.0, rel=1e-14)
    # the values quoted for l = 1: q^2 = (0.46576, 0.41582, 0.09988, 0.01631)
    assert np.allclose(p.q2(), [0.46576, 0.41582, 0.09988, 0.01631], atol=5e-6)


@pytest.mark.parametrize("ell,J", [(1.0, 3), (0.7, 5), (2.0, 2)])
def test_periodic_truncation_bound(ell, J):
    """|exact periodic kernel - J-harmonic kernel| <= var * sum_{j > J} q_j^2."""
    p = Periodic(J, ell, 1.3, 24.0)
    tail = 1.3 * (1.0 - p.q2().sum())
    tau = np.linspace(-50, 50, 401)
    err = np.abs(p.kernel_untruncated(tau) - p.kernel(tau)).max()
    assert err <= tail * (1 + 1e-12) + 1e-15


@pytest.mark.parametrize("terms,hyper", MODELS)
def test_parameter_derivatives_against_differences(terms, hyper):
    """dA (expm Frechet), dP0 and dk (closed form) against central differences."""
    m = model_for(terms, hyper)
    hyper = np.asarray(hyper, float)
    dt = 0.83
    dA, dP, dk = m.dA(dt), m.dPinf(), m.dkernel(np.array([0.0, 0.6, 2.2]))
    for i in range(m.n_kernel_params):
        e = 1e-6 * hyper[i]
        hp, hm = hyper.copy(), hyper.copy()
        hp[i] += e
        hm[i] -= e
        mp_, mm_ = model_for(terms, hp), model_for(terms, hm)
        fdA = (mp_.A(dt) - mm_.A(dt)) / (2 * e)
        fdP = (mp_.Pinf() - mm_.Pinf()) / (2 * e)
        fdk = (mp_.kernel(np.array([0.0, 0.6, 2.2])) - mm_.kernel(np.array([0.0, 0.6, 2.2]))) / (2 * e)
        scale = max(1.0, np.abs(fdA).max())
        assert np.abs(dA[i] - fdA).max() <= 1e-6 * scale
        assert np.abs(dP[i] - fdP).max() <= 1e-6 * max(1.0, np.abs(fdP).max())
        assert np.abs(dk[i] - fdk).max() <= 1e-6 * max(1.0, np.abs(fdk).max())


@pytest.mark.parametrize("terms,hyper", MODELS)
def test_c_closed_forms_match_expm(terms, hyper):
    """The C oracle's closed-form A, Q, P0 (and its Bessel series) against scipy's expm route."""
    m = model_for(terms, hyper)
    t = np.cumsum(np.array([0.0, 0.0, 1e-9, 1e-5, 0.01, 0.4, 1.0, 3.3, 12.0, 60.0, 0.2]))
    A, Q, P, h = native.edges(terms, hyper, t)
    # closed forms agree to rounding; a Lyapunov-solved P0 (squared exponential) to its solve
    lyap = any(k == SQEXP for k, _ in terms)
    assert np.allclose(P, m.Pinf(), rtol=1e-12 if lyap else 1e-14,
                       atol=(1e-15 * np.abs(P).max()) if lyap else 1e-16)
    assert np.array_equal(h, m.H())
    for i in range(t.shape[0] - 1):
        dt = t[i + 1] - t[i]
        # scipy's scaling-and-squaring expm carries an error of about eps * |F dt|
        scale = max(1.0, np.abs(m.F() * dt).max())
        assert np.abs(A[i] - m.A(dt)).max() <= 1e-13 * scale
        assert np.abs(Q[i] - m.Q(dt)).max() <= 1e-13 * scale * np.abs(P).max()


def test_quasi_periodic_limits():
    """The quasi-periodic term is the periodic term times exp(-|tau| / decay): the product
    form holds at every lag, and a very long decay gives back the periodic logML."""
    qp = model_for([(QUASIPERIODIC, 3)], [0.9, 1.3, 5.0, 7.0, 0.1])
    per = model_for([(PERIODIC, 3)], [0.9, 1.3, 5.0, 0.1])
    for tau in TAUS:
        assert qp.kernel(tau) == pytest.approx(per.kernel(tau) * np.exp(-tau / 7.0), rel=1e-14, abs=1e-300)
    rng = np.random.default_rng(3)
    t = np.sort(rng.uniform(0, 30, 200))
    y = np.cos(t) + 0.3 * rng.standard_normal(200)
    far = native.btd_factored([(QUASIPERIODIC, 3)], [0.9, 1.3, 5.0, 1e9, 0.1], t, y, want_blocks=False)
    ref = native.btd_factored([(PERIODIC, 3)], [0.9, 1.3, 5.0, 0.1], t, y, want_blocks=False)
    assert abs(far["logml"] - ref["logml"]) <= 1e-6 * abs(ref["logml"])


@pytest.mark.parametrize("order,err", [(2, 0.15), (4, 0.018), (6, 3.1e-3), (8, 6.5e-4)])
def test_squared_exponential_approximation_converges(order, err):
    """The SDE of the truncated spectral density approaches var exp(-tau^2 / 2 l^2): the
    largest error over the lags shrinks with the order (about 5x per two orders)."""
    m = SquaredExponential(order, 1.3, 0.7)
    tau = np.linspace(0.0, 6.0, 61)
    e = np.abs(m.kernel(tau) - m.kernel_untruncated(tau)).max() / m.var
    assert e <= err


def test_squared_exponential_scaling_in_lengthscale():
    """P0 entry (i, j) scales as lam^(i+j) (the state holds f and its derivatives), the
    stable roots as lam: the Lyapunov solutions at two lengthscales agree after rescaling."""
    a, b = SquaredExponential(6, 1.0, 1.0), SquaredExponential(6, 0.37, 1.0)
    i = np.arange(6)
    scale = b.lam ** (i[:, None] + i[None, :])
    assert np.allclose(b.Pinf() / scale, a.Pinf(), rtol=1e-8, atol=1e-10 * np.abs(a.Pinf()).max())
    assert np.allclose(np.sort_complex(np.linalg.eigvals(b.F())), np.sort_complex(np.linalg.eigvals(a.F())) * b.lam,
                       rtol=1e-9)
    R = a.F() @ a.Pinf() + a.Pinf() @ a.F().T
    mask = np.ones((6, 6), bool)
    mask[5, 5] = False
    assert np.abs(R[mask]).max() <= 1e-10 * np.abs(R).max()
