"""High-precision references for small inputs (test infrastructure only; see the package header).

Everything here runs in mpmath arithmetic from the float64 inputs, so the only rounding left
is mpmath's own at the working precision (50 digits by default).  Two routes are kept apart
so that each pins the other:

  kernel_mp   the covariance function of every term, written out per kind:
                Matern-1/2 .. 7/2 closed forms, k = var * poly(lam |tau|) * exp(-lam |tau|),
                  lam = sqrt(2 nu) / l (Sec. 2.1; the variance and |tau| restored);
                periodic with J harmonics: var * sum_j q_j^2 cos(j w0 tau), q_0^2 = I_0(z)e^-z,
                  q_j^2 = 2 I_j(z) e^-z, z = l^-2, w0 = 2 pi / period (the Bessel
                  expansion of exp(z cos x) truncated after J harmonics);
                quasi-periodic: the periodic kernel times exp(-|tau| / l_decay);
                squared exponential of order n: the kernel of the rational spectral density
                  q / |P(i w)|^2, P(s) = prod_k (s - lam r_k) over the stable roots (the
                  exponential series of 1/S(w) truncated after n + 1 terms, Sec. 2.2 "a
                  state-space form may be approximate"), evaluated by residues at the roots:
                  k(tau) = sum_k q exp(p_k |tau|) / (P'(p_k) P(-p_k)).
  ssm_blocks  the same terms as linear SDEs (Sec. 2.1, eq. ss1): per block F, the stationary
                covariance P0 and the observation row h; Matern and the harmonics with their
                closed-form P0, the squared exponential with P0 from a Lyapunov solve;
                transitions A(dt) = expm(F dt) by mpmath's expm.

  gp_dense_mp               logML, data fit, log det K_y, latent mean and variance by a dense
                            factorisation of K_y = K_f + s2 I (eq. ml2, mean2, k3), K_f from
                            kernel_mp; optionally dlogML/dtheta by central differences of that
                            logML at raised precision.
  state_posterior_dense_mp  posterior means of the states and the blocks Cov(z_n, z_n | y),
                            Cov(z_{n+1}, z_n | y) (the block-tridiagonal part of the inverse
                            precision, Sec. 3.1 subproblems 2 and 4), by conditioning the
                            stacked prior Cov(z_i, z_j) = A(t_i - t_j) P0 (t_i >= t_j) on y.

A term kind that is not listed raises ValueError; nothing is modelled as something else.
"""
from __future__ import annotations

import functools

import mpmath as mp
import numpy as np

MATERN32, MATERN52, PERIODIC, MATERN12, MATERN72, QUASIPERIODIC, SQEXP = 1, 2, 3, 4, 5, 6, 7
_MATERN_B = {MATERN12: 1, MATERN32: 2, MATERN52: 3, MATERN72: 4}
_N_PARAMS = {MATERN12: 2, MATERN32: 2, MATERN52: 2, MATERN72: 2, PERIODIC: 3, QUASIPERIODIC: 4, SQEXP: 2}


def _mpf(v):
    """An mpmath number from a float64 input (exactly) or from an mpmath number (kept)."""
    return v if isinstance(v, mp.mpf) else mp.mpf(float(v))


def parse_terms(terms, hyper):
    """Split a hyperparameter row into per-term tuples (kind, harmonics or order, params) and the
    noise variance, in the row layout of the library: each term's parameters in order, the
    noise variance last.  Unknown kinds raise."""
    parts, p = [], 0
    for kind, harm in terms:
        kind = int(kind)
        if kind not in _N_PARAMS:
            raise ValueError(f"term kind {kind} has no high-precision model")
        k = _N_PARAMS[kind]
        parts.append((kind, int(harm), [_mpf(v) for v in hyper[p:p + k]]))
        p += k
    if len(hyper) != p + 1:
        raise ValueError(f"expected {p + 1} hyperparameters, got {len(hyper)}")
    return parts, _mpf(hyper[p])


# ------------------------------------------------------------------------------ kernels
def _matern_kernel(kind, ell, var, tau):
    b = _MATERN_B[kind]
    lam = mp.sqrt(2 * b - 1) / ell                       # sqrt(2 nu), nu = b - 1/2
    r = lam * abs(tau)
    if b == 1:
        poly = mp.mpf(1)
    elif b == 2:
        poly = 1 + r
    elif b == 3:
        poly = 1 + r + r * r / 3
    else:
        poly = 1 + r + 2 * r * r / 5 + r ** 3 / 15
    return var * poly * mp.exp(-r)


def _bessel_weights(J, ell):
    z = 1 / (ell * ell)
    return [mp.besseli(j, z) * mp.exp(-z) * (1 if j == 0 else 2) for j in range(J + 1)]


def _periodic_kernel(J, ell, var, period, tau):
    w0 = 2 * mp.pi / period
    return var * mp.fsum(q * mp.cos(j * w0 * tau) for j, q in enumerate(_bessel_weights(J, ell)))


@functools.lru_cache(maxsize=None)
def _se_unit_roots(order, prec):
    """Stable roots r_k (Re r_k < 0) of the unit-lengthscale spectral factor: u_k are the roots
    of sum_{j=0}^{order} u^j / j!, and u = -r^2 / 2."""
    if order < 2 or order % 2:
        raise ValueError("the squared-exponential approximation needs an even order >= 2")
    with mp.workprec(prec):
        us = mp.polyroots([1 / mp.factorial(j) for j in range(order, -1, -1)], maxsteps=400,
                          extraprec=4 * prec)
        out = []
        for u in us:
            r = mp.sqrt(-2 * u)
            if mp.re(r) > 0:
                r = -r
            out.append(r)
        return tuple(out)


def _se_noise_density(order, lam, var):
    """White-noise density q of the order-n factor: var sqrt(2 pi) n! 2^n lam^(2n - 1)."""
    return var * mp.sqrt(2 * mp.pi) * mp.factorial(order) * mp.mpf(2) ** order * lam ** (2 * order - 1)


def _se_kernel(order, ell, var, tau):
    lam = 1 / ell
    p = [lam * r for r in _se_unit_roots(order, mp.mp.prec)]
    q = _se_noise_density(order, lam, var)
    x = abs(tau)
    total = mp.mpc(0)
    for j, pj in enumerate(p):
        dP = mp.fprod(pj - pk for k, pk in enumerate(p) if k != j)     # P'(p_j)
        Pm = mp.fprod(-pj - pk for pk in p)                             # P(-p_j)
        total += mp.exp(pj * x) / (dP * Pm)
    return q * mp.re(total)


def term_kernel(kind, harm, par, tau):
    if kind in _MATERN_B:
        return _matern_kernel(kind, par[0], par[1], tau)
    if kind == PERIODIC:
        return _periodic_kernel(harm, par[0], par[1], par[2], tau)
    if kind == QUASIPERIODIC:
        return _periodic_kernel(harm, par[0], par[1], par[2], tau) * mp.exp(-abs(tau) / par[3])
    if kind == SQEXP:
        return _se_kernel(harm, par[0], par[1], tau)
    raise ValueError(f"term kind {kind} has no high-precision model")


def kernel_mp(terms, hyper, tau, dps: int = 50):
    """k(tau) of the sum of terms (closed forms and residues), at `dps` digits."""
    with mp.workdps(dps):
        parts, _ = parse_terms(terms, hyper)
        tau = mp.mpf(float(tau)) if not isinstance(tau, mp.mpf) else tau
        return mp.fsum(term_kernel(k, h, par, tau) for k, h, par in parts)


# ------------------------------------------------------------------------------ state space
def _lyapunov(F, W):
    """P with F P + P F^T + W = 0 (vectorised: (I kron F + F kron I) vec P = -vec W)."""
    n = F.rows
    M = mp.matrix(n * n, n * n)
    rhs = mp.matrix(n * n, 1)
    for i in range(n):
        for j in range(n):
            r = i * n + j
            rhs[r] = -W[i, j]
            for k in range(n):
                M[r, k * n + j] += F[i, k]          # (F P)_ij
                M[r, i * n + k] += F[j, k]          # (P F^T)_ij
    v = mp.lu_solve(M, rhs)
    P = mp.matrix(n, n)
    for i in range(n):
        for j in range(n):
            P[i, j] = (v[i * n + j] + v[j * n + i]) / 2
    return P


def _companion(coeffs):
    """Companion matrix of s^n + c_{n-1} s^{n-1} + ... + c_0 (coeffs = [c_0, ..., c_{n-1}])."""
    n = len(coeffs)
    F = mp.matrix(n, n)
    for i in range(n - 1):
        F[i, i + 1] = 1
    for k in range(n):
        F[n - 1, k] = -coeffs[k]
    return F


def _matern_block(kind, ell, var):
    b = _MATERN_B[kind]
    lam = mp.sqrt(2 * b - 1) / ell
    F = _companion([mp.binomial(b, k) * lam ** (b - k) for k in range(b)])
    # P0_ij = (-1)^j k^(i+j)(0) for the Matern-nu kernel: the even derivatives at 0 are
    # 3/2: -lam^2;  5/2: -lam^2/3, lam^4;  7/2: -lam^2/5, lam^4/5, -lam^6 (times var)
    d = {1: [1], 2: [1, -lam ** 2], 3: [1, -lam ** 2 / 3, lam ** 4],
         4: [1, -lam ** 2 / 5, lam ** 4 / 5, -lam ** 6]}[b]
    P = mp.matrix(b, b)
    for i in range(b):
        for j in range(b):
            if (i + j) % 2 == 0:
                P[i, j] = var * (-1) ** j * d[(i + j) // 2]
    h = [mp.mpf(1)] + [mp.mpf(0)] * (b - 1)
    return [(F, P, h)]


def _harmonic_blocks(J, ell, var, period, decay=None):
    w0 = 2 * mp.pi / period
    lam = 0 if decay is None else 1 / decay
    out = []
    for j, q in enumerate(_bessel_weights(J, ell)):
        F = mp.matrix([[-lam, -j * w0], [j * w0, -lam]])
        P = mp.matrix([[var * q, 0], [0, var * q]])
        out.append((F, P, [mp.mpf(1), mp.mpf(0)]))
    return out


def _se_block(order, ell, var):
    lam = 1 / ell
    p = [lam * r for r in _se_unit_roots(order, mp.mp.prec)]
    # coefficients of prod (s - p_k), c[i] multiplying s^i (c[order] = 1); real up to the
    # rounding of the conjugate pairs
    c = [mp.mpc(1)]
    for pk in p:
        c = [(c[i - 1] if i > 0 else 0) - pk * (c[i] if i < len(c) else 0) for i in range(len(c) + 1)]
    coeffs = [mp.re(c[k]) for k in range(order)]
    F = _companion(coeffs)
    W = mp.matrix(order, order)
    W[order - 1, order - 1] = _se_noise_density(order, lam, var)
    P = _lyapunov(F, W)
    h = [mp.mpf(1)] + [mp.mpf(0)] * (order - 1)
    return [(F, P, h)]


def ssm_blocks(terms, hyper):
    """(blocks, noise): the block-diagonal state-space model, one (F, P0, h) per block, in the
    state order of the library (terms in order; a periodic term as one 2 x 2 block per
    harmonic, cosine state first)."""
    parts, noise = parse_terms(terms, hyper)
    blocks = []
    for kind, harm, par in parts:
        if kind in _MATERN_B:
            blocks += _matern_block(kind, par[0], par[1])
        elif kind == PERIODIC:
            blocks += _harmonic_blocks(harm, par[0], par[1], par[2])
        elif kind == QUASIPERIODIC:
            blocks += _harmonic_blocks(harm, par[0], par[1], par[2], decay=par[3])
        elif kind == SQEXP:
            blocks += _se_block(harm, par[0], par[1])
        else:
            raise ValueError(f"term kind {kind} has no high-precision model")
    return blocks, noise


def _blockdiag(mats):
    n = sum(M.rows for M in mats)
    out = mp.matrix(n, n)
    o = 0
    for M in mats:
        for i in range(M.rows):
            for j in range(M.cols):
                out[o + i, o + j] = M[i, j]
        o += M.rows
    return out


def ssm_kernel_mp(terms, hyper, tau, dps: int = 50):
    """h expm(F |tau|) P0 h^T of the state-space form (the kernel it implies)."""
    with mp.workdps(dps):
        blocks, _ = ssm_blocks(terms, hyper)
        x = abs(mp.mpf(float(tau)))
        total = mp.mpf(0)
        for F, P, h in blocks:
            M = mp.expm(F * x) * P
            total += mp.fsum(h[i] * M[i, j] * h[j] for i in range(F.rows) for j in range(F.rows))
        return total


# ------------------------------------------------------------------------------ dense GP
def _logml_terms(terms, hyper, t, y, want_mean_var):
    parts, noise = parse_terms(terms, hyper)
    n = len(t)
    Kf = mp.matrix(n, n)
    for i in range(n):
        for j in range(i + 1):
            v = mp.fsum(term_kernel(k, h, par, t[i] - t[j]) for k, h, par in parts)
            Kf[i, j] = Kf[j, i] = v
    Ky = Kf + noise * mp.eye(n)
    L = mp.cholesky(Ky)
    logdet = 2 * mp.fsum(mp.log(L[i, i]) for i in range(n))
    alpha = mp.cholesky_solve(Ky, mp.matrix(y)) if n else mp.matrix(0, 1)
    datafit = mp.fsum(y[i] * alpha[i] for i in range(n))
    logml = -datafit / 2 - logdet / 2 - n * mp.log(2 * mp.pi) / 2
    out = {"logml": logml, "datafit": datafit, "logdet": logdet}
    if want_mean_var:
        mean = Kf * alpha
        X = mp.inverse(Ky) * Kf
        out["f_mean"] = [mean[i] for i in range(n)]
        out["f_var"] = [Kf[i, i] - mp.fsum(Kf[i, j] * X[j, i] for j in range(n)) for i in range(n)]
    return out


def gp_dense_mp(terms, hyper, t, y, dps: int = 50, want_grad: bool = False) -> dict:
    """Dense GP at `dps` digits: logML, data fit y^T K_y^-1 y, log det K_y, latent mean and
    variance; with want_grad, dlogML/dtheta for every entry of the hyperparameter row by central
    differences of the logML at dps + 40 digits with steps of 10^-(dps/2 + 5) (truncation and
    rounding both far below 10^-dps)."""
    with mp.workdps(dps):
        tt = [mp.mpf(float(v)) for v in t]
        yy = [mp.mpf(float(v)) for v in y]
        r = _logml_terms(terms, hyper, tt, yy, True)
        out = {"logml": float(r["logml"]), "datafit": float(r["datafit"]), "logdet": float(r["logdet"]),
               "f_mean": np.array([float(v) for v in r["f_mean"]]),
               "f_var": np.array([float(v) for v in r["f_var"]])}
    if want_grad:
        out["grad"] = grad_mp(terms, hyper, t, y, dps)
    return out


def grad_mp(terms, hyper, t, y, dps: int = 50) -> np.ndarray:
    g = []
    with mp.workdps(dps + 40):
        tt = [mp.mpf(float(v)) for v in t]
        yy = [mp.mpf(float(v)) for v in y]
        base = [mp.mpf(float(v)) for v in hyper]
        for i in range(len(base)):
            h = mp.mpf(10) ** (-(dps // 2 + 5)) * max(mp.mpf(1), abs(base[i]))
            up = list(base)
            dn = list(base)
            up[i] += h
            dn[i] -= h
            lu = _logml_terms(terms, up, tt, yy, False)["logml"]
            ld = _logml_terms(terms, dn, tt, yy, False)["logml"]
            g.append(float((lu - ld) / (2 * h)))
    return np.array(g)


def state_posterior_dense_mp(terms, hyper, t, y, dps: int = 50) -> dict:
    """Posterior of the stacked states at `dps` digits: z_mean [n, b], S_diag [n, b, b] =
    Cov(z_n, z_n | y), S_sub [n-1, b, b] = Cov(z_{n+1}, z_n | y), plus logML, f_mean, f_var
    from the same K_y.  t must be sorted (non-decreasing)."""
    with mp.workdps(dps):
        blocks, noise = ssm_blocks(terms, hyper)
        tt = [mp.mpf(float(v)) for v in t]
        yy = [mp.mpf(float(v)) for v in y]
        n = len(tt)
        if any(tt[i + 1] < tt[i] for i in range(n - 1)):
            raise ValueError("times must be sorted")
        P0 = _blockdiag([P for _, P, _ in blocks])
        h = mp.matrix([v for _, _, hb in blocks for v in hb])
        b = P0.rows
        P0h = P0 * h

        def A(x):
            return _blockdiag([mp.expm(F * x) for F, _, _ in blocks])

        # C[i][j] = Cov(z_i, y_j) (a b-vector); K_f[i, j] = h^T C[i][j]
        C = [[None] * n for _ in range(n)]
        Asub = [None] * max(n - 1, 0)
        for i in range(n):
            C[i][i] = P0h
            for j in range(i):
                M = A(tt[i] - tt[j])
                if j == i - 1:
                    Asub[j] = M
                C[i][j] = M * P0h                    # Cov(z_i, z_j) h, t_i >= t_j
                C[j][i] = P0 * (M.T * h)             # Cov(z_j, z_i) h = P0 A^T h
        Kf = mp.matrix(n, n)
        for i in range(n):
            for j in range(n):
                Kf[i, j] = mp.fsum(h[k] * C[i][j][k] for k in range(b))
        Ky = Kf + noise * mp.eye(n)
        Kinv = mp.inverse(Ky)
        alpha = Kinv * mp.matrix(yy)
        L = mp.cholesky(Ky)
        logdet = 2 * mp.fsum(mp.log(L[i, i]) for i in range(n))
        datafit = mp.fsum(yy[i] * alpha[i] for i in range(n))
        logml = -datafit / 2 - logdet / 2 - n * mp.log(2 * mp.pi) / 2
        Cm = []                                      # C_i as a b x n matrix
        for i in range(n):
            M = mp.matrix(b, n)
            for j in range(n):
                for k in range(b):
                    M[k, j] = C[i][j][k]
            Cm.append(M)
        X = [Kinv * Cm[i].T for i in range(n)]       # K_y^-1 C_i^T, n x b
        z_mean = np.zeros((n, b))
        S_diag = np.zeros((n, b, b))
        S_sub = np.zeros((max(n - 1, 0), b, b))
        f_mean = np.zeros(n)
        f_var = np.zeros(n)
        for i in range(n):
            mu = Cm[i] * alpha
            S = P0 - Cm[i] * X[i]
            f_mean[i] = float(mp.fsum(h[k] * mu[k] for k in range(b)))
            f_var[i] = float(mp.fsum(h[r] * S[r, c] * h[c] for r in range(b) for c in range(b)))
            for r in range(b):
                z_mean[i, r] = float(mu[r])
                for c in range(b):
                    S_diag[i, r, c] = float((S[r, c] + S[c, r]) / 2)
        for i in range(n - 1):
            S = Asub[i] * P0 - Cm[i + 1] * X[i]
            for r in range(b):
                for c in range(b):
                    S_sub[i, r, c] = float(S[r, c])
        return {"logml": float(logml), "datafit": float(datafit), "logdet": float(logdet),
                "z_mean": z_mean, "S_diag": S_diag, "S_sub": S_sub, "f_mean": f_mean, "f_var": f_var}
