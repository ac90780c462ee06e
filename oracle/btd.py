"""Sequential block-tridiagonal elimination of the posterior precision (test infrastructure only).

Paper Sec. 2.2-3.1.  With G = I_N (x) h^T and Sigma = s2 I, the posterior
precision of the stacked states is the symmetric block-tridiagonal (BTD) matrix
    Kb = Kinv + G^T Sigma^-1 G,
where Kinv = A^-T Q^-1 A^-1 (Theorem 1, eq. hh1) has, for node n and edge n
(edge n joins nodes n and n+1 with A_n = A[t_{n+1} - t_n], Q_n = Q[...]):
    D_n = [n = 0: P0^-1] + [n > 0: Q_{n-1}^-1] + [n < N-1: A_n^T Q_n^-1 A_n]
    B_n = Kinv[n+1, n] = -Q_n^-1 A_n
and G^T Sigma^-1 G = I_N (x) J with J = h h^T / s2 (the paper's sigma_n typo
read as s2^-1).  The four computational subproblems of Sec. 3.1 are:
  1  solve Kb x = r with r = G^T Sigma^-1 y                (posterior mean, eq. mean3)
  2  the diagonal blocks of Kb^-1                          (variance, eq. k3)
  3  log det Kb, giving log det K_y by the determinant lemma (eq. det_1):
        log det K_y = log det Kb - log det Kinv + N log s2,
        log det Kinv = -log det P0 - sum_n log det Q_n
  4  tr(Kb^-1 dKb/dtheta) from the BTD part of Kb^-1 only  (eq. dd1)
All four come from one block LDL^T in natural order (the Thomas algorithm of
Sec. 3.1): pivots Dh_0 = D_0, Dh_{n+1} = D_{n+1} - B_n Dh_n^-1 B_n^T,
forward and back substitution, and Takahashi's recursion for the selected
inverse S_n = Dh_n^-1 + L_n^T S_{n+1} L_n, S_{n+1,n} = -S_{n+1} L_n with
L_n = B_n Dh_n^-1.

Two pivot representations:
  literal   D_n, B_n multiplied out exactly as above (faithful to the paper;
            needs Q_n^-1, so it is only accurate when no gap is tiny).
  factored  the same elimination with each pivot written through the Woodbury
            identity, Dh_n = C_n^-1 + A_n^T Q_n^-1 A_n where
              C_0 = (P0^-1 + J)^-1 = (I + P0 J)^-1 P0,
              V_n = Q_n + A_n C_n A_n^T,  C_{n+1} = (V_n^-1 + J)^-1 = (I + V_n J)^-1 V_n,
            so no Q^-1 is ever formed; log det Dh_n telescopes to
            log det K_y = sum_n log det(I + V_{n-1} J) + N log s2  (V_{-1} = P0).
            Forward substitution carries x^f_n = C_n rhat_n, back substitution
            x_n = x^f_n + G_n (x_{n+1} - A_n x^f_n) with G_n = C_n A_n^T V_n^-1 = Dh_n^-1 A_n^T Q_n^-1,
            and Takahashi becomes S_n = C_n + G_n (S_{n+1} - V_n) G_n^T, S_{n+1,n} = S_{n+1} G_n^T.
The trace gradient (subproblem 4, eq. dd1 with the data-fit derivative) is
written with the literal blocks and is therefore a comfortable-input check only.
"""
from __future__ import annotations

import numpy as np

from .ssm import SumModel


def _logdet_spd(M):
    L = np.linalg.cholesky(0.5 * (M + M.T))
    return 2.0 * np.sum(np.log(np.diag(L)))


def precision_blocks(model: SumModel, t):
    """Literal BTD blocks (D_n, B_n) of Kb = Kinv + I (x) J (Theorem 1)."""
    t = np.asarray(t, dtype=np.float64)
    n, b = t.shape[0], model.b
    h = model.H()
    J = np.outer(h, h) / model.noise
    D = np.zeros((n, b, b))
    B = np.zeros((max(n - 1, 0), b, b))
    D[0] += np.linalg.inv(model.Pinf())
    for i in range(n - 1):
        A = model.A(t[i + 1] - t[i])
        Qi = np.linalg.inv(model.Q(t[i + 1] - t[i]))
        D[i] += A.T @ Qi @ A
        D[i + 1] += Qi
        B[i] = -Qi @ A
    D += J[None]
    return D, B


def btd_literal(model: SumModel, t, y) -> dict:
    """Subproblems 1-3 (+2 as the selected inverse) with the multiplied-out blocks."""
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n, b = t.shape[0], model.b
    h = model.H()
    s2 = model.noise
    D, B = precision_blocks(model, t)
    r = h[None, :] * (y / s2)[:, None]
    # block LDL^T (Thomas)
    Dh = np.zeros_like(D)
    rh = np.zeros_like(r)
    Dh[0], rh[0] = D[0], r[0]
    for i in range(n - 1):
        L = B[i] @ np.linalg.inv(Dh[i])
        Dh[i + 1] = D[i + 1] - L @ B[i].T
        rh[i + 1] = r[i + 1] - L @ rh[i]
    logdetKb = sum(_logdet_spd(Dh[i]) for i in range(n))
    x = np.zeros_like(r)
    x[-1] = np.linalg.solve(Dh[-1], rh[-1])
    for i in range(n - 2, -1, -1):
        x[i] = np.linalg.solve(Dh[i], rh[i] - B[i].T @ x[i + 1])
    # Takahashi selected inverse
    S = np.zeros_like(D)
    Ssub = np.zeros_like(B)
    S[-1] = np.linalg.inv(Dh[-1])
    for i in range(n - 2, -1, -1):
        L = B[i] @ np.linalg.inv(Dh[i])
        Ssub[i] = -S[i + 1] @ L
        S[i] = np.linalg.inv(Dh[i]) - L.T @ Ssub[i]
        S[i] = 0.5 * (S[i] + S[i].T)
    logdetKinv = -_logdet_spd(model.Pinf()) - sum(
        _logdet_spd(model.Q(t[i + 1] - t[i])) for i in range(n - 1))
    logdet = logdetKb - logdetKinv + n * np.log(s2)
    datafit = float(y @ y) / s2 - float(np.sum(r * x))      # y^T Sigma^-1 y - r^T Kb^-1 r
    return {
        "logml": -0.5 * datafit - 0.5 * logdet - 0.5 * n * np.log(2.0 * np.pi),
        "datafit": datafit, "logdet": logdet, "z_mean": x, "S_diag": S, "S_sub": Ssub,
        "f_mean": x @ h, "f_var": np.einsum("i,nij,j->n", h, S, h), "D": D, "B": B,
    }


def btd_factored(model: SumModel, t, y) -> dict:
    """The same elimination with Woodbury pivots (valid for tiny gaps, dt = 0 and Q = 0)."""
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n, b = t.shape[0], model.b
    h = model.H()
    s2 = model.noise
    J = np.outer(h, h) / s2
    I = np.eye(b)
    C = np.zeros((n, b, b))          # C_n = (Dh_n - A_n^T Q_n^-1 A_n)^-1
    V = np.zeros((max(n - 1, 0), b, b))
    A = np.zeros((max(n - 1, 0), b, b))
    xf = np.zeros((n, b))            # C_n rhat_n
    logdet_terms = 0.0
    Vprev = model.Pinf()
    xprev_pred = np.zeros(b)         # A_{n-1} x^f_{n-1}
    for i in range(n):
        eta = h * (y[i] / s2)
        M = I + Vprev @ J
        logdet_terms += np.log(np.linalg.det(M))
        C[i] = np.linalg.solve(M, Vprev)
        C[i] = 0.5 * (C[i] + C[i].T)
        # rhat_i = eta_i + V_{i-1}^-1 A_{i-1} x^f_{i-1}  =>  C_i rhat_i = M^-1 (V eta + A x^f)
        xf[i] = np.linalg.solve(M, Vprev @ eta + xprev_pred)
        if i < n - 1:
            A[i] = model.A(t[i + 1] - t[i])
            V[i] = model.Q(t[i + 1] - t[i]) + A[i] @ C[i] @ A[i].T
            V[i] = 0.5 * (V[i] + V[i].T)
            Vprev = V[i]
            xprev_pred = A[i] @ xf[i]
    x = np.zeros((n, b))
    S = np.zeros((n, b, b))
    Ssub = np.zeros((max(n - 1, 0), b, b))
    x[-1], S[-1] = xf[-1], C[-1]
    for i in range(n - 2, -1, -1):
        G = np.linalg.solve(V[i], A[i] @ C[i]).T          # C_i A_i^T V_i^-1
        x[i] = xf[i] + G @ (x[i + 1] - A[i] @ xf[i])
        Si = C[i] + G @ (S[i + 1] - V[i]) @ G.T
        S[i] = 0.5 * (Si + Si.T)
        Ssub[i] = S[i + 1] @ G.T
    r = h[None, :] * (y / s2)[:, None]
    logdet = logdet_terms + n * np.log(s2)
    datafit = float(y @ y) / s2 - float(np.sum(r * x))
    return {
        "logml": -0.5 * datafit - 0.5 * logdet - 0.5 * n * np.log(2.0 * np.pi),
        "datafit": datafit, "logdet": logdet, "z_mean": x, "S_diag": S, "S_sub": Ssub,
        "f_mean": x @ h, "f_var": np.einsum("i,nij,j->n", h, S, h),
    }


def btd_dense_blocks(D, B) -> np.ndarray:
    """Assemble the full BTD matrix from its blocks (tiny N, for checks)."""
    n, b = D.shape[0], D.shape[1]
    K = np.zeros((n * b, n * b))
    for i in range(n):
        K[i * b:(i + 1) * b, i * b:(i + 1) * b] = D[i]
    for i in range(n - 1):
        K[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] = B[i]
        K[i * b:(i + 1) * b, (i + 1) * b:(i + 2) * b] = B[i].T
    return K


def trace_gradient(model: SumModel, t, y) -> np.ndarray:
    """d logML / d theta through eq. dd1 and the data-fit derivative (comfortable inputs only).

    For a kernel parameter theta (Sec. 2.4), with x = Kb^-1 r and S the BTD part of Kb^-1:
      d logML = -1/2 x^T dKinv x - 1/2 tr(S dKinv) + 1/2 d log det Kinv,
      d log det Kinv = -tr(P0^-1 dP0) - sum_n tr(Q_n^-1 dQ_n),
    where dKinv has the BTD pattern of Theorem 1 (only blocks on it enter the trace).
    For the noise variance s2 ("computed similarly"):
      d logML / d s2 = 1/2 sum_n [(y_n - h^T x_n)^2 + h^T S_n h] / s2^2 - N / (2 s2).
    """
    t = np.asarray(t, dtype=np.float64)
    n, b = t.shape[0], model.b
    h = model.H()
    sol = btd_literal(model, t, y)
    x, S, Ssub = sol["z_mean"], sol["S_diag"], sol["S_sub"]
    P = model.Pinf()
    Pi = np.linalg.inv(P)
    grads = []
    for k, dP in enumerate(model.dPinf()):
        dD = np.zeros((n, b, b))
        dB = np.zeros((max(n - 1, 0), b, b))
        dD[0] += -Pi @ dP @ Pi
        dlogdet = -np.trace(Pi @ dP)
        for i in range(n - 1):
            dt = t[i + 1] - t[i]
            A = model.A(dt)
            Qi = np.linalg.inv(model.Q(dt))
            dA = model.dA(dt)[k]
            dQ = model.dQ(dt)[k]
            dQi = -Qi @ dQ @ Qi
            dD[i] += dA.T @ Qi @ A + A.T @ dQi @ A + A.T @ Qi @ dA
            dD[i + 1] += dQi
            dB[i] = -(dQi @ A + Qi @ dA)
            dlogdet -= np.trace(Qi @ dQ)
        quad = sum(x[i] @ dD[i] @ x[i] for i in range(n)) + 2.0 * sum(
            x[i + 1] @ dB[i] @ x[i] for i in range(n - 1))
        tr = sum(np.sum(S[i] * dD[i]) for i in range(n)) + 2.0 * sum(
            np.sum(Ssub[i] * dB[i]) for i in range(n - 1))
        grads.append(-0.5 * quad - 0.5 * tr + 0.5 * dlogdet)
    s2 = model.noise
    resid = np.asarray(y) - x @ h
    fvar = np.einsum("i,nij,j->n", h, S, h)
    grads.append(0.5 * np.sum(resid * resid + fvar) / (s2 * s2) - 0.5 * n / s2)
    return np.array(grads)


def fd_gradient(logml_fn, hyper_row, rel_step: float = 1e-3) -> np.ndarray:
    """Richardson-extrapolated central differences of logml_fn(hyper_row) in each parameter."""
    hyper_row = np.asarray(hyper_row, dtype=np.float64)
    g = np.zeros_like(hyper_row)
    for i in range(hyper_row.shape[0]):
        hstep = rel_step * abs(hyper_row[i])

        def cd(step):
            hp, hm = hyper_row.copy(), hyper_row.copy()
            hp[i] += step
            hm[i] -= step
            return (logml_fn(hp) - logml_fn(hm)) / (2.0 * step)

        g[i] = (4.0 * cd(hstep / 2.0) - cd(hstep)) / 3.0
    return g
