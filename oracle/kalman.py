"""Covariance-form Kalman filter and RTS smoother (test infrastructure only).

This is the state-space GP of the paper's comparison method (Sec. 1 and
Sec. 4.2, "KF model"), written from the textbook filter equations for the
model of eq. ss1 with z_0 ~ N(0, P0):
  predict   m_{n|n-1} = A_{n-1} m_{n-1|n-1},  P_{n|n-1} = A P_{n-1|n-1} A^T + Q_{n-1}
  update    s_n = h^T P h + s2,  v_n = y_n - h^T m,  K = P h / s_n,
            m_{n|n} = m + K v_n,  P_{n|n} = P - K s_n K^T
  logML     = sum_n -1/2 log(2 pi s_n) - 1/2 v_n^2 / s_n
  RTS       G_n = P_{n|n} A_n^T P_{n+1|n}^-1,
            mu_n = m_{n|n} + G_n (mu_{n+1} - m_{n+1|n}),
            S_n  = P_{n|n} + G_n (S_{n+1} - P_{n+1|n}) G_n^T,
            S_{n+1,n} = S_{n+1} G_n^T   (lag-one smoothed covariance)
The gradient is forward-mode (tangent-linear): every filter quantity carries
its derivative with respect to each hyperparameter, so it needs no inverse of
Q_n and holds at any gap, including dt = 0.
"""
from __future__ import annotations

import numpy as np

from .ssm import SumModel


def kf_rts(model: SumModel, t, y) -> dict:
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n, b = t.shape[0], model.b
    h = model.H()
    s2 = model.noise
    mp_ = np.zeros((n, b))
    Pp = np.zeros((n, b, b))
    mf = np.zeros((n, b))
    Pf = np.zeros((n, b, b))
    A = np.zeros((max(n - 1, 0), b, b))
    m = np.zeros(b)
    P = model.Pinf().copy()
    logdet = 0.0
    datafit = 0.0
    for i in range(n):
        if i > 0:
            A[i - 1] = model.A(t[i] - t[i - 1])
            m = A[i - 1] @ m
            P = A[i - 1] @ P @ A[i - 1].T + model.Q(t[i] - t[i - 1])
            P = 0.5 * (P + P.T)
        mp_[i], Pp[i] = m, P
        if np.isnan(y[i]):
            # no observation at this time (a prediction point): the filtered state is the
            # predicted one and the point adds nothing to the likelihood
            mf[i], Pf[i] = m, P
            continue
        u = P @ h
        s = float(h @ u) + s2
        v = y[i] - float(h @ m)
        K = u / s
        m = m + K * v
        P = P - np.outer(K, u)
        P = 0.5 * (P + P.T)
        mf[i], Pf[i] = m, P
        logdet += np.log(s)
        datafit += v * v / s
    # RTS smoother
    mu = np.zeros((n, b))
    S = np.zeros((n, b, b))
    Ssub = np.zeros((max(n - 1, 0), b, b))
    mu[-1], S[-1] = mf[-1], Pf[-1]
    for i in range(n - 2, -1, -1):
        G = np.linalg.solve(Pp[i + 1], A[i] @ Pf[i]).T      # P_{i|i} A^T P_{i+1|i}^-1
        mu[i] = mf[i] + G @ (mu[i + 1] - mp_[i + 1])
        Si = Pf[i] + G @ (S[i + 1] - Pp[i + 1]) @ G.T
        S[i] = 0.5 * (Si + Si.T)
        Ssub[i] = S[i + 1] @ G.T
    n_obs = int(np.count_nonzero(~np.isnan(y)))
    return {
        "logml": -0.5 * datafit - 0.5 * logdet - 0.5 * n_obs * np.log(2.0 * np.pi),
        "datafit": datafit, "logdet": logdet,
        "m_pred": mp_, "P_pred": Pp, "m_filt": mf, "P_filt": Pf,
        "z_mean": mu, "S_diag": S, "S_sub": Ssub,
        "f_mean": mu @ h, "f_var": np.einsum("i,nij,j->n", h, S, h),
    }


def kf_tangent_grad(model: SumModel, t, y) -> dict:
    """logML and d logML / d theta (kernel parameters in order, then the noise variance)."""
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n, b = t.shape[0], model.b
    h = model.H()
    s2 = model.noise
    npar = model.n_params
    m = np.zeros(b)
    P = model.Pinf().copy()
    dm = np.zeros((npar, b))
    dP = np.zeros((npar, b, b))
    for i, d in enumerate(model.dPinf()):
        dP[i] = d
    ll = 0.0
    g = np.zeros(npar)
    ds2 = np.zeros(npar)
    ds2[-1] = 1.0
    for i in range(n):
        if i > 0:
            dt = t[i] - t[i - 1]
            A = model.A(dt)
            Q = model.Q(dt)
            dA = model.dA(dt) + [np.zeros((b, b))]
            dQ = model.dQ(dt) + [np.zeros((b, b))]
            for k in range(npar):
                dm[k] = dA[k] @ m + A @ dm[k]
                dP[k] = dA[k] @ P @ A.T + A @ dP[k] @ A.T + A @ P @ dA[k].T + dQ[k]
            m = A @ m
            P = A @ P @ A.T + Q
            P = 0.5 * (P + P.T)
        u = P @ h
        s = float(h @ u) + s2
        v = y[i] - float(h @ m)
        ll += -0.5 * np.log(2.0 * np.pi * s) - 0.5 * v * v / s
        for k in range(npar):
            du = dP[k] @ h
            dsk = float(h @ du) + ds2[k]
            dv = -float(h @ dm[k])
            g[k] += -0.5 * dsk / s - v * dv / s + 0.5 * v * v * dsk / (s * s)
            dK = (du - u * dsk / s) / s
            dm[k] = dm[k] + dK * v + (u / s) * dv
            dP[k] = dP[k] - (np.outer(du, u) + np.outer(u, du)) / s + np.outer(u, u) * dsk / (s * s)
        K = u / s
        m = m + K * v
        P = P - np.outer(K, u)
        P = 0.5 * (P + P.T)
    return {"logml": ll, "grad": g}
