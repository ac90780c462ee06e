"""O(N^3) textbook GP (test infrastructure only; see the package header).

This is the plain definition every faster route must reproduce:
  K_f[i, j] = k(t_i - t_j),   K_y = K_f + s2 I        (eq. k2 with G K G^T = K_f)
  logML = -1/2 y^T K_y^-1 y - 1/2 log det K_y - N/2 log 2 pi     (eq. ml2, n read as N)
  mean  = K_f K_y^-1 y                                 (eq. mean2 at t* = t)
  var_i = (K_f - K_f K_y^-1 K_f)_ii                    (diagonal of eq. k3: latent f, no s2)
  dlogML/dtheta = 1/2 tr((a a^T - K_y^-1) dK_y/dtheta),  a = K_y^-1 y
The state-level posterior (mean of z_n and the blocks Cov(z_n, z_n | y),
Cov(z_{n+1}, z_n | y)) uses the stacked prior covariance of Sec. 2.1:
Cov(z_i, z_j) = A[t_i - t_j] P0 for t_i >= t_j, conditioned on y by the same
dense formulas.  `stacked_prior_cov` also builds the paper's  A Q A^T  product
(eq. k1) so tests can check Theorem 1 directly.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .ssm import SumModel


def gp_dense(model: SumModel, t, y, want_grad: bool = True) -> dict:
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = t.shape[0]
    tau = t[:, None] - t[None, :]
    Kf = model.kernel(tau)
    Ky = Kf + model.noise * np.eye(n)
    L = scipy.linalg.cholesky(Ky, lower=True)
    alpha = scipy.linalg.cho_solve((L, True), y)
    logdet = 2.0 * np.sum(np.log(np.diag(L)))
    datafit = float(y @ alpha)
    out = {
        "logml": -0.5 * datafit - 0.5 * logdet - 0.5 * n * np.log(2.0 * np.pi),
        "datafit": datafit,
        "logdet": logdet,
        "f_mean": Kf @ alpha,
    }
    V = scipy.linalg.solve_triangular(L, Kf, lower=True)
    out["f_var"] = np.diag(Kf) - np.sum(V * V, axis=0)
    if want_grad:
        Kinv = scipy.linalg.cho_solve((L, True), np.eye(n))
        W = np.outer(alpha, alpha) - Kinv
        g = [0.5 * np.sum(W * dK) for dK in model.dkernel(tau)]
        g.append(0.5 * np.trace(W))          # dK_y / d s2 = I
        out["grad"] = np.array(g)
    return out


def gp_predict_dense(model: SumModel, t, y, t_star) -> dict:
    """Latent predictive mean and variance at new times t* (eq. mean4-mean6, eq. k3 at t*):
    m* = K(t*, t) K_y^-1 y,   v* = k(0) - diag(K(t*, t) K_y^-1 K(t, t*))."""
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    ts = np.asarray(t_star, dtype=np.float64)
    n = t.shape[0]
    Ky = model.kernel(t[:, None] - t[None, :]) + model.noise * np.eye(n)
    Ks = model.kernel(ts[:, None] - t[None, :])
    L = scipy.linalg.cholesky(Ky, lower=True)
    alpha = scipy.linalg.cho_solve((L, True), y)
    V = scipy.linalg.solve_triangular(L, Ks.T, lower=True)
    return {"f_mean": Ks @ alpha, "f_var": model.kernel(np.zeros(1))[0] - np.sum(V * V, axis=0)}


def stacked_prior_cov(model: SumModel, t) -> np.ndarray:
    """Prior covariance of the stacked states [z_0; ...; z_{N-1}] (N b x N b)."""
    t = np.asarray(t, dtype=np.float64)
    n, b = t.shape[0], model.b
    P = model.Pinf()
    K = np.zeros((n * b, n * b))
    for i in range(n):
        for j in range(i + 1):
            blk = model.A(t[i] - t[j]) @ P
            K[i * b:(i + 1) * b, j * b:(j + 1) * b] = blk
            K[j * b:(j + 1) * b, i * b:(i + 1) * b] = blk.T
    return K


def paper_AQA(model: SumModel, t):
    """The factors of eq. k1: the block lower-triangular A, block-diagonal Q and A Q A^T."""
    t = np.asarray(t, dtype=np.float64)
    n, b = t.shape[0], model.b
    Abig = np.zeros((n * b, n * b))
    Qbig = np.zeros((n * b, n * b))
    for i in range(n):
        Abig[i * b:(i + 1) * b, i * b:(i + 1) * b] = np.eye(b)
        for j in range(i):
            Abig[i * b:(i + 1) * b, j * b:(j + 1) * b] = model.A(t[i] - t[j])
        Qbig[i * b:(i + 1) * b, i * b:(i + 1) * b] = model.Pinf() if i == 0 else model.Q(t[i] - t[i - 1])
    return Abig, Qbig, Abig @ Qbig @ Abig.T


def state_posterior_dense(model: SumModel, t, y) -> dict:
    """Dense posterior of the stacked states: means and the tridiagonal blocks of the covariance."""
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n, b = t.shape[0], model.b
    K = stacked_prior_cov(model, t)
    G = np.kron(np.eye(n), model.H()[None, :])
    Ky = G @ K @ G.T + model.noise * np.eye(n)
    KG = K @ G.T
    sol = np.linalg.solve(Ky, np.column_stack([y, KG.T]))
    mu = KG @ sol[:, 0]
    S = K - KG @ sol[:, 1:]
    S = 0.5 * (S + S.T)
    z_mean = mu.reshape(n, b)
    S_diag = np.stack([S[i * b:(i + 1) * b, i * b:(i + 1) * b] for i in range(n)])
    S_sub = np.stack([S[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] for i in range(n - 1)]) \
        if n > 1 else np.zeros((0, b, b))
    return {"z_mean": z_mean, "S_diag": S_diag, "S_sub": S_sub, "S_full": S}


def gp_dense_mp(model: SumModel, t, y, dps: int = 50) -> dict:
    """High-precision dense GP (mpmath) for small N: logML, mean and variance.

    The kernel of every term is written out per kind in `oracle.mpref` and evaluated in
    mpmath arithmetic from the float64 inputs; a kind it does not model raises."""
    from .mpref import gp_dense_mp as _gp_dense_mp
    return _gp_dense_mp(model.terms, model.hyper_row, t, y, dps=dps)
