"""Seeded synthetic workloads for temporal-GP inference.

Every array is drawn from ``numpy.random.default_rng`` (PCG64) with the
configuration number as the seed, so a workload is reproduced bit for bit
from its name and sizes alone.  Draw order per series: (i) times, (ii) for the
batched workload the lengths, lengthscales and noise variances first, then one
child stream per series, (iii) the initial latent state, (iv) the transition
noise, (v) periodic amplitudes, (vi) the observation noise.

The latent signal is a sample of the GP prior.  Matern terms are simulated as
white noise through a cascade of first-order low-pass stages (the Jordan form
of the Matern-(p+1/2) SDE, whose transfer function is (s + lam)^-(p+1)); this
is a different state basis from the companion form the inference code uses,
and its stationary covariance comes from scipy's Lyapunov solver.  Periodic
terms are sums of random-phase harmonics with the Bessel weights of the
truncated periodic kernel.  Nothing here computes a likelihood, a mean or a
variance: the module only draws data.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg
import scipy.special

KIND_MATERN32 = 1
KIND_MATERN52 = 2
KIND_PERIODIC = 3
KIND_MATERN12 = 4
KIND_MATERN72 = 5
KIND_QUASIPERIODIC = 6
KIND_SQEXP = 7

_MATERN_ORDER = {KIND_MATERN12: 1, KIND_MATERN32: 2, KIND_MATERN52: 3, KIND_MATERN72: 4}
_MATERN_NU = {KIND_MATERN12: 0.5, KIND_MATERN32: 1.5, KIND_MATERN52: 2.5, KIND_MATERN72: 3.5}


def state_dim(terms) -> int:
    """State dimension b of a sum of terms ``[(kind, harmonics), ...]``."""
    b = 0
    for kind, harm in terms:
        if kind in _MATERN_ORDER:
            b += _MATERN_ORDER[kind]
        elif kind in (KIND_PERIODIC, KIND_QUASIPERIODIC):
            b += 2 * (harm + 1)
        elif kind == KIND_SQEXP:
            b += harm
        else:
            raise ValueError(f"unknown term kind {kind}")
    return b


def n_hyper(terms) -> int:
    """Hyperparameters per series: (l, var) per Matern and squared exponential, (l, var,
    period) per periodic, (l, var, period, decay) per quasi-periodic, then noise."""
    n = 0
    for kind, _ in terms:
        n += {KIND_PERIODIC: 3, KIND_QUASIPERIODIC: 4}.get(kind, 2)
    return n + 1


@dataclass
class Workload:
    name: str
    terms: list
    t: np.ndarray          # [n_points] float64, series concatenated, non-decreasing per series
    y: np.ndarray          # [n_points] float64
    offsets: np.ndarray    # [n_series + 1] int64
    hyper: np.ndarray      # [n_series, n_hyper] float64
    notes: dict = field(default_factory=dict)

    @property
    def n_series(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_points(self) -> int:
        return int(self.t.shape[0])

    @property
    def b(self) -> int:
        return state_dim(self.terms)

    def series(self, i):
        a, e = int(self.offsets[i]), int(self.offsets[i + 1])
        return self.t[a:e], self.y[a:e], self.hyper[i]


# --------------------------------------------------------------------------
# prior simulation (data generation only)
# --------------------------------------------------------------------------

def _cascade_stationary_cov(order: int, lam: float) -> np.ndarray:
    """Stationary covariance of white noise (unit intensity) through `order` stages (s+lam)^-1."""
    F = -lam * np.eye(order) + np.diag(np.ones(order - 1), -1)
    W = np.zeros((order, order))
    W[0, 0] = 1.0
    P = scipy.linalg.solve_continuous_lyapunov(F, -W)
    return 0.5 * (P + P.T)


def _cascade_transition(order: int, lam: float, dt: np.ndarray) -> np.ndarray:
    """exp(F dt) for F = -lam I + S (S the sub-diagonal shift): e^{-lam dt} sum_k (S dt)^k / k!."""
    dt = np.asarray(dt, dtype=np.float64)
    out = np.zeros(dt.shape + (order, order))
    e = np.exp(-lam * dt)
    for i in range(order):
        for j in range(i + 1):
            k = i - j
            out[..., i, j] = e * dt ** k / float(np.prod(np.arange(1, k + 1)))
    return out


def _matern_prior_path(t: np.ndarray, kind: int, ell: float, var: float,
                       rng: np.random.Generator) -> np.ndarray:
    """One sample path of a Matern GP at sorted times t (exact in distribution)."""
    order = _MATERN_ORDER[kind]
    n = t.shape[0]
    # (iii) initial state, (iv) transition noise, drawn in one piece
    z0 = rng.standard_normal(order)
    xi = rng.standard_normal((max(n - 1, 0), order))
    return _matern_batch([t], kind, np.array([[ell, var, 0.0]]), [(z0, xi)])


def _periodic_prior_path(t, harmonics, ell, var, period, rng):
    """Random-phase harmonic sum with Bessel weights q_j^2 (truncated periodic kernel)."""
    z = 1.0 / (ell * ell)
    j = np.arange(harmonics + 1)
    q2 = scipy.special.ive(j, z) * np.where(j == 0, 1.0, 2.0)
    amp = rng.standard_normal((harmonics + 1, 2))
    w0 = 2.0 * np.pi / period
    f = np.zeros_like(t)
    for jj in range(harmonics + 1):
        s = np.sqrt(var * q2[jj])
        f += s * (amp[jj, 0] * np.cos(jj * w0 * t) + amp[jj, 1] * np.sin(jj * w0 * t))
    return f


def _quasi_periodic_prior_path(t, harmonics, ell, var, period, decay, rng):
    """Quasi-periodic sample path: every harmonic is a 2-state rotation by j w0 dt that decays
    by e^{-dt/decay}, with stationary covariance var q_j^2 I (exact in distribution)."""
    n = t.shape[0]
    z = 1.0 / (ell * ell)
    j = np.arange(harmonics + 1)
    q2 = scipy.special.ive(j, z) * np.where(j == 0, 1.0, 2.0)
    w0 = 2.0 * np.pi / period
    dt = np.diff(t)
    e = np.exp(-dt / decay)
    f = np.zeros(n)
    for jj in range(harmonics + 1):
        s2 = var * q2[jj]
        x0 = np.sqrt(s2) * rng.standard_normal(2)
        xi = rng.standard_normal((max(n - 1, 0), 2))
        if n == 0:
            continue
        # state ordered (sin part, cos part): the helper returns the last component
        c, s = np.cos(jj * w0 * dt), np.sin(jj * w0 * dt)
        A = np.zeros((n - 1, 2, 2))
        A[:, 1, 1], A[:, 1, 0] = e * c, -e * s
        A[:, 0, 1], A[:, 0, 0] = e * s, e * c
        w = np.sqrt(s2 * np.maximum(1.0 - e * e, 0.0))[:, None] * xi
        f += _recurrence_last_component(A, w, x0[::-1].copy())
    return f


def _sqexp_prior_path(t, ell, var, rng, n_features=256):
    """Smooth path with (approximately) the squared-exponential covariance var exp(-tau^2 / (2 l^2)),
    by random Fourier features: frequencies drawn from the kernel's spectral density N(0, 1/l^2),
    uniform phases, sqrt(2 var / D) sum_d cos(w_d t + phi_d)."""
    w = rng.standard_normal(n_features) / ell
    phi = rng.uniform(0.0, 2.0 * np.pi, n_features)
    f = np.empty(t.shape[0])
    for s in range(0, t.shape[0], 1 << 15):          # bounded temporaries for long series
        f[s:s + (1 << 15)] = np.cos(np.outer(t[s:s + (1 << 15)], w) + phi).sum(axis=1)
    return np.sqrt(2.0 * var / n_features) * f


def make_series(t, terms, hyper_row, rng):
    """Draw y = f + eps at times t for one series with hyperparameter row `hyper_row`."""
    t = np.asarray(t, dtype=np.float64)
    f = np.zeros_like(t)
    p = 0
    for kind, harm in terms:
        if kind in _MATERN_ORDER:
            f += _matern_prior_path(t, kind, hyper_row[p], hyper_row[p + 1], rng)
            p += 2
        elif kind == KIND_QUASIPERIODIC:
            f += _quasi_periodic_prior_path(t, harm, hyper_row[p], hyper_row[p + 1], hyper_row[p + 2],
                                            hyper_row[p + 3], rng)
            p += 4
        elif kind == KIND_SQEXP:
            f += _sqexp_prior_path(t, hyper_row[p], hyper_row[p + 1], rng)
            p += 2
        else:
            f += _periodic_prior_path(t, harm, hyper_row[p], hyper_row[p + 1], hyper_row[p + 2], rng)
            p += 3
    noise = hyper_row[p]
    # (vi) observation noise
    return f + np.sqrt(noise) * rng.standard_normal(t.shape[0])


def _single(name, terms, t, hyper_row, rng, notes):
    y = make_series(t, terms, hyper_row, rng)
    return Workload(name=name, terms=list(terms), t=t, y=y,
                    offsets=np.array([0, t.shape[0]], dtype=np.int64),
                    hyper=np.asarray(hyper_row, dtype=np.float64)[None, :].copy(), notes=notes)


def make_config(k: int, n: int | None = None, n_series: int | None = None,
                max_len: int | None = None) -> Workload:
    """Workload k in 1..5; `n`, `n_series`, `max_len` shrink it for small test cases."""
    if k == 1:
        n = 1000 if n is None else n
        rng = np.random.default_rng(1)
        t = np.sort(rng.uniform(0.0, 100.0, n))
        return _single("matern32_n%d_uniform100" % n, [(KIND_MATERN32, 0)], t,
                       [1.0, 1.0, 0.1], rng, {"grid": "sorted U[0,100]"})
    if k in (2, 5):
        n = (1 << 20 if k == 2 else 1 << 24) if n is None else n
        rng = np.random.default_rng(k)
        t = np.cumsum(rng.exponential(1.0, n))
        return _single("matern52_n%d_exp1gaps" % n, [(KIND_MATERN52, 0)], t,
                       [5.0, 2.0, 0.05], rng, {"grid": "cumsum Exp(1)"})
    if k == 3:
        n = (1 << 18) if n is None else n
        rng = np.random.default_rng(3)
        t = np.sort(rng.uniform(0.0, 1.0e4, n))
        terms = [(KIND_MATERN32, 0), (KIND_PERIODIC, 3)]
        return _single("matern32+periodic3_n%d_uniform1e4" % n, terms, t,
                       [50.0, 1.0, 1.0, 1.0, 24.0, 0.1], rng, {"grid": "sorted U[0,1e4]"})
    if k == 4:
        S = 4096 if n_series is None else n_series
        rng = np.random.default_rng(4)
        lens = np.round(np.exp(rng.uniform(np.log(64.0), np.log(16384.0), S))).astype(np.int64)
        if max_len is not None:
            lens = np.minimum(lens, max_len)
        ells = np.exp(rng.uniform(np.log(0.5), np.log(20.0), S))
        noises = rng.uniform(0.01, 0.5, S)
        hyper = np.stack([ells, np.ones(S), noises], axis=1)
        w = make_batch(lens, hyper, [(KIND_MATERN52, 0)], seed=4)
        w.name = "batched_matern52_%dseries" % S
        w.notes["lengths"] = "log-U[64,16384]"
        return w
    raise ValueError("config must be 1..5")


def _recurrence_last_component(A, w, x0):
    """x_0 = x0, x_{k+1} = A_k x_k + w_k (A: [n-1, d, d], w: [n-1, d]); returns x_k[d-1] for all
    k, with about sqrt(n) blocks of sqrt(n) steps, vectorised over the blocks."""
    n = A.shape[0] + 1
    d = x0.shape[0]
    block = max(16, int(np.sqrt(n)) + 1)
    nb = (n + block - 1) // block
    Ap = np.broadcast_to(np.eye(d), (nb * block, d, d)).copy()
    Ap[: n - 1] = A
    wp = np.zeros((nb * block, d))
    wp[: n - 1] = w
    Ap = Ap.reshape(nb, block, d, d)
    wp = wp.reshape(nb, block, d)
    state = np.zeros((nb, d))
    phi = np.broadcast_to(np.eye(d), (nb, d, d)).copy()
    local_last = np.zeros((nb, block))
    for j in range(block):
        local_last[:, j] = state[:, d - 1]
        state = np.einsum("bij,bj->bi", Ap[:, j], state) + wp[:, j]
        phi = Ap[:, j] @ phi
    X = np.zeros((nb, d))
    X[0] = x0
    for b in range(nb - 1):
        X[b + 1] = phi[b] @ X[b] + state[b]
    out = np.zeros((nb, block))
    yv = X
    for j in range(block):
        out[:, j] = yv[:, d - 1] + local_last[:, j]
        yv = np.einsum("bij,bj->bi", Ap[:, j], yv)
    return out.reshape(-1)[:n]


def _psd_factor_apply(Q, xi):
    """W xi for W W^T = Q (batched, PSD up to rounding): an LDL^T factorisation with pivots below
    1e-14 of the diagonal scale treated as zero (their column is dropped), so near-singular Q
    from tiny gaps is handled; W = L sqrt(D)."""
    n, d, _ = Q.shape
    Lm = np.zeros((n, d, d))
    D = np.zeros((n, d))
    scale = np.max(np.abs(np.einsum("kii->ki", Q)), axis=1)
    for j in range(d):
        Dj = Q[:, j, j] - np.einsum("kc,kc->k", Lm[:, j, :j] ** 2, D[:, :j])
        ok = Dj > 1e-14 * scale
        D[:, j] = np.where(ok, Dj, 0.0)
        Lm[:, j, j] = 1.0
        safe = np.where(ok, Dj, 1.0)
        for r in range(j + 1, d):
            num = Q[:, r, j] - np.einsum("kc,kc,kc->k", Lm[:, r, :j], Lm[:, j, :j], D[:, :j])
            Lm[:, r, j] = np.where(ok, num / safe, 0.0)
    return np.einsum("kij,kj->ki", Lm, np.sqrt(D) * xi)


def _matern_batch(ts, kind, hyper, draws):
    """Prior sample paths of independent Matern series, concatenated, in one recurrence: the
    step out of a series' last point has A = 0 and carries the next series' initial state.
    `draws[i]` = (standard normal of the initial state, standard normals of the transition noise)."""
    order = _MATERN_ORDER[kind]
    lens = np.array([t.shape[0] for t in ts], dtype=np.int64)
    nz = np.nonzero(lens)[0]
    n = int(lens.sum())
    A = np.zeros((max(n - 1, 0), order, order))
    w = np.zeros((max(n - 1, 0), order))
    x0_first = None
    pos = 0
    for k, i in enumerate(nz):
        L = int(lens[i])
        lam = np.sqrt(2.0 * _MATERN_NU[kind]) / hyper[i, 0]
        P = _cascade_stationary_cov(order, lam)
        P *= hyper[i, 1] / P[order - 1, order - 1]
        x0 = np.linalg.cholesky(P) @ draws[i][0]
        if k == 0:
            x0_first = x0
        else:
            w[pos - 1] = x0          # boundary step: A = 0, noise = next initial state
        dt = np.diff(ts[i])
        for a in range(0, L - 1, 1 << 20):          # slices bound the temporary memory
            e = min(L - 1, a + (1 << 20))
            Ai = _cascade_transition(order, lam, dt[a:e])
            # Q_n = P - A P A^T (PSD up to rounding; the factor drops non-positive pivots)
            Q = P[None] - Ai @ P[None] @ np.swapaxes(Ai, -1, -2)
            A[pos + a: pos + e] = Ai
            w[pos + a: pos + e] = _psd_factor_apply(Q, draws[i][1][a:e])
        pos += L
    if n == 0:
        return np.zeros(0)
    return _recurrence_last_component(A, w, x0_first)


def make_batch(lens, hyper, terms, seed) -> Workload:
    """Independent series of the given lengths (zero allowed) and hyperparameter rows, one child
    stream per series: times are cumulative Exp(1) gaps, y a prior sample plus noise."""
    lens = np.asarray(lens, dtype=np.int64)
    hyper = np.asarray(hyper, dtype=np.float64).reshape(lens.shape[0], -1)
    S = lens.shape[0]
    children = np.random.SeedSequence(seed).spawn(S)
    ts, ys = [], []
    if len(terms) == 1 and terms[0][0] in _MATERN_ORDER:
        # one Matern term: the same draws per series as make_series, one vectorised recurrence
        order = _MATERN_ORDER[terms[0][0]]
        draws, eps = [], []
        for i in range(S):
            r = np.random.default_rng(children[i])
            n = int(lens[i])
            ts.append(np.cumsum(r.exponential(1.0, n)))
            if n > 0:
                draws.append((r.standard_normal(order), r.standard_normal((n - 1, order))))
                eps.append(r.standard_normal(n))
            else:
                draws.append(None)
                eps.append(np.zeros(0))
        f = _matern_batch(ts, terms[0][0], hyper, draws)
        pos = 0
        for i in range(S):
            n = int(lens[i])
            ys.append(f[pos: pos + n] + np.sqrt(hyper[i, 2]) * eps[i])
            pos += n
    else:
        for i in range(S):
            r = np.random.default_rng(children[i])
            t = np.cumsum(r.exponential(1.0, int(lens[i])))
            ts.append(t)
            ys.append(make_series(t, terms, hyper[i], r) if lens[i] > 0 else np.zeros(0))
    offsets = np.zeros(S + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(lens)
    return Workload(name="batch_%dseries_seed%d" % (S, seed), terms=list(terms),
                    t=np.concatenate(ts), y=np.concatenate(ys), offsets=offsets, hyper=hyper.copy(),
                    notes={"grid": "cumsum Exp(1) per series"})
