"""Oracle state-space models (test infrastructure only; see the package header).

Paper Sec. 2.1: a temporal GP is the output H z(t) of a linear SDE
dz = F z dt + L dW.  Between two time points the state moves by the
transition A[dt] = expm(F dt) (the paper writes this for Matern-3/2 in
eq. ss_matern) and picks up Gaussian noise with covariance
Q[dt] = P0 - A[dt] P0 A[dt]^T, where P0 is the stationary covariance.

Readings adopted where the paper is silent or garbled:
  * P0 carries the signal variance: P0 = var * diag(1, lam^2) for Matern-3/2
    (eq. ss_matern drops the variance), and the kernel uses |tau|.
  * Matern-5/2 (b = 3) and the periodic kernel (b = 2(J+1)) are not written
    out in the paper; both follow the same construction.  P0 of Matern-5/2
    holds the derivatives of k at 0: E[f f]=k(0), E[f' f']=-k''(0),
    E[f f'']=k''(0), E[f'' f'']=k''''(0).
  * The periodic term is the J-harmonic truncation of
    var * exp(-2 sin^2(pi tau / p) / l^2): harmonic j is a rotation at
    angular rate j*2*pi/p with stationary covariance var * q_j^2 * I2, where
    q_0^2 = I_0(z) e^-z, q_j^2 = 2 I_j(z) e^-z, z = l^-2 (the Bessel
    generating function of e^{z cos x}).  Its Q is zero: a rotation keeps q_j^2 I2.
  * A sum of kernels stacks the states: F, P0, A, Q block-diagonal, H side by side.

Transitions come from scipy.linalg.expm and their parameter derivatives from
scipy.linalg.expm_frechet, so this module never uses a hand-derived closed
form for A[dt]; the closed forms it does hold (P0, the kernel functions) are
pinned by tests against the Lyapunov equation and H expm(F tau) P0 H^T.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.special

MATERN32, MATERN52, PERIODIC, MATERN12, MATERN72, QUASIPERIODIC, SQEXP = 1, 2, 3, 4, 5, 6, 7
_MATERN_B = {MATERN12: 1, MATERN32: 2, MATERN52: 3, MATERN72: 4}


class Matern:
    """Matern-nu, nu in {1/2, 3/2, 5/2, 7/2} (b = nu + 1/2); hyperparameters (lengthscale,
    variance).  F is the companion matrix of (s + lam)^b, lam = sqrt(2 nu) / lengthscale."""

    n_params = 2

    def __init__(self, kind: int, lengthscale: float, variance: float):
        if kind not in _MATERN_B:
            raise ValueError("Matern kind must be 4 (nu=1/2), 1 (3/2), 2 (5/2) or 5 (7/2)")
        self.kind = kind
        self.ell = float(lengthscale)
        self.var = float(variance)
        self.b = _MATERN_B[kind]
        nu = self.b - 0.5
        self.lam = np.sqrt(2.0 * nu) / self.ell

    # --- SDE ---------------------------------------------------------------
    def F(self):
        # companion matrix: last row -binom(b, k) lam^(b-k), k = 0..b-1
        b, l = self.b, self.lam
        F = np.diag(np.ones(b - 1), 1)
        F[b - 1, :] = [-scipy.special.comb(b, k, exact=True) * l ** (b - k) for k in range(b)]
        return F

    def dF_dlam(self):
        b, l = self.b, self.lam
        F = np.zeros((b, b))
        F[b - 1, :] = [-scipy.special.comb(b, k, exact=True) * (b - k) * l ** (b - k - 1) for k in range(b)]
        return F

    def H(self):
        h = np.zeros(self.b)
        h[0] = 1.0
        return h

    def Pinf(self):
        l, v = self.lam, self.var
        if self.kind == MATERN12:
            return np.array([[v]])
        if self.kind == MATERN32:
            return v * np.diag([1.0, l * l])
        if self.kind == MATERN52:
            return v * np.array([[1.0, 0.0, -l * l / 3.0],
                                 [0.0, l * l / 3.0, 0.0],
                                 [-l * l / 3.0, 0.0, l ** 4]])
        return v * np.array([[1.0, 0.0, -l ** 2 / 5.0, 0.0],
                             [0.0, l ** 2 / 5.0, 0.0, -l ** 4 / 5.0],
                             [-l ** 2 / 5.0, 0.0, l ** 4 / 5.0, 0.0],
                             [0.0, -l ** 4 / 5.0, 0.0, l ** 6]])

    def dPinf_dlam(self):
        l, v = self.lam, self.var
        if self.kind == MATERN12:
            return np.zeros((1, 1))
        if self.kind == MATERN32:
            return v * np.diag([0.0, 2.0 * l])
        if self.kind == MATERN52:
            return v * np.array([[0.0, 0.0, -2.0 * l / 3.0],
                                 [0.0, 2.0 * l / 3.0, 0.0],
                                 [-2.0 * l / 3.0, 0.0, 4.0 * l ** 3]])
        return v * np.array([[0.0, 0.0, -2.0 * l / 5.0, 0.0],
                             [0.0, 2.0 * l / 5.0, 0.0, -4.0 * l ** 3 / 5.0],
                             [-2.0 * l / 5.0, 0.0, 4.0 * l ** 3 / 5.0, 0.0],
                             [0.0, -4.0 * l ** 3 / 5.0, 0.0, 6.0 * l ** 5]])

    # derivatives with respect to the raw hyperparameters (lengthscale, variance)
    def dF(self):
        dlam_dell = -self.lam / self.ell
        return [self.dF_dlam() * dlam_dell, np.zeros((self.b, self.b))]

    def dPinf(self):
        dlam_dell = -self.lam / self.ell
        return [self.dPinf_dlam() * dlam_dell, self.Pinf() / self.var]

    # --- covariance function --------------------------------------------------
    def kernel(self, tau):
        r = np.abs(tau) * self.lam
        if self.kind == MATERN12:
            return self.var * np.exp(-r)
        if self.kind == MATERN32:
            return self.var * (1.0 + r) * np.exp(-r)
        if self.kind == MATERN52:
            return self.var * (1.0 + r + r * r / 3.0) * np.exp(-r)
        return self.var * (1.0 + r + 2.0 * r * r / 5.0 + r ** 3 / 15.0) * np.exp(-r)

    def dkernel(self, tau):
        """[dk/dlengthscale, dk/dvariance] of the closed-form kernel."""
        tau = np.abs(tau)
        l = self.lam
        e = np.exp(-l * tau)
        r = l * tau
        if self.kind == MATERN12:
            dk_dlam = -self.var * tau * e
        elif self.kind == MATERN32:
            dk_dlam = -self.var * l * tau * tau * e
        elif self.kind == MATERN52:
            dk_dlam = -self.var * (l * tau * tau / 3.0) * (1.0 + l * tau) * e
        else:
            dk_dlam = -self.var * tau * (r / 15.0) * (3.0 + 3.0 * r + r * r) * e
        return [dk_dlam * (-l / self.ell), self.kernel(tau) / self.var]


class Periodic:
    """J-harmonic periodic term; hyperparameters (lengthscale, variance, period)."""

    n_params = 3

    def __init__(self, harmonics: int, lengthscale: float, variance: float, period: float):
        self.J = int(harmonics)
        self.ell = float(lengthscale)
        self.var = float(variance)
        self.period = float(period)
        self.b = 2 * (self.J + 1)
        self.w0 = 2.0 * np.pi / self.period
        self.z = 1.0 / (self.ell * self.ell)

    def q2(self):
        j = np.arange(self.J + 1)
        return scipy.special.ive(j, self.z) * np.where(j == 0, 1.0, 2.0)

    def dq2_dz(self):
        j = np.arange(self.J + 1)
        dive = 0.5 * (scipy.special.ive(j - 1, self.z) + scipy.special.ive(j + 1, self.z)) \
            - scipy.special.ive(j, self.z)
        return dive * np.where(j == 0, 1.0, 2.0)

    def F(self):
        F = np.zeros((self.b, self.b))
        for j in range(self.J + 1):
            F[2 * j, 2 * j + 1] = -j * self.w0
            F[2 * j + 1, 2 * j] = j * self.w0
        return F

    def H(self):
        h = np.zeros(self.b)
        h[0::2] = 1.0
        return h

    def Pinf(self):
        return np.diag(np.repeat(self.var * self.q2(), 2))

    def dF(self):
        z = np.zeros((self.b, self.b))
        return [z, z.copy(), -self.F() / self.period]

    def dPinf(self):
        dz_dell = -2.0 / self.ell ** 3
        return [np.diag(np.repeat(self.var * self.dq2_dz() * dz_dell, 2)),
                self.Pinf() / self.var,
                np.zeros((self.b, self.b))]

    def kernel(self, tau):
        tau = np.asarray(tau, dtype=np.float64)
        out = np.zeros_like(tau)
        for j, q in enumerate(self.q2()):
            out = out + q * np.cos(j * self.w0 * tau)
        return self.var * out

    def kernel_untruncated(self, tau):
        s = np.sin(np.pi * np.asarray(tau) / self.period)
        return self.var * np.exp(-2.0 * s * s / (self.ell * self.ell))

    def dkernel(self, tau):
        tau = np.asarray(tau, dtype=np.float64)
        q2, dq = self.q2(), self.dq2_dz()
        dz_dell = -2.0 / self.ell ** 3
        d_ell = np.zeros_like(tau)
        d_per = np.zeros_like(tau)
        for j in range(self.J + 1):
            d_ell = d_ell + dq[j] * dz_dell * np.cos(j * self.w0 * tau)
            # d cos(j w0 tau)/dp = sin(j w0 tau) * j * tau * w0 / p
            d_per = d_per + q2[j] * np.sin(j * self.w0 * tau) * j * tau * self.w0 / self.period
        return [self.var * d_ell, self.kernel(tau) / self.var, self.var * d_per]


class QuasiPeriodic(Periodic):
    """Quasi-periodic term: the J-harmonic periodic term times an exponential (Matern-1/2)
    decay, k(tau) = k_periodic(tau) exp(-|tau| / l_decay); hyperparameters (lengthscale,
    variance, period, decay lengthscale).  State space: every harmonic block rotates and decays,
    F_j = [[-lam, -j w0], [j w0, -lam]] with lam = 1 / l_decay; P0 as for the periodic term."""

    n_params = 4

    def __init__(self, harmonics, lengthscale, variance, period, decay):
        super().__init__(harmonics, lengthscale, variance, period)
        self.decay = float(decay)
        self.lam = 1.0 / self.decay

    def F(self):
        return super().F() - self.lam * np.eye(self.b)

    def dF(self):
        z = np.zeros((self.b, self.b))
        return [z, z.copy(), -super().F() / self.period, np.eye(self.b) / self.decay ** 2]

    def dPinf(self):
        return super().dPinf() + [np.zeros((self.b, self.b))]

    def kernel(self, tau):
        return super().kernel(tau) * np.exp(-np.abs(tau) / self.decay)

    def kernel_untruncated(self, tau):
        return super().kernel_untruncated(tau) * np.exp(-np.abs(tau) / self.decay)

    def dkernel(self, tau):
        tau = np.asarray(tau, dtype=np.float64)
        e = np.exp(-np.abs(tau) / self.decay)
        kp = Periodic.kernel(self, tau)
        d_ell, _, d_per = Periodic.dkernel(self, tau)
        return [d_ell * e, kp / self.var * e, d_per * e, kp * e * np.abs(tau) / self.decay ** 2]


class SquaredExponential:
    """Squared-exponential term var * exp(-tau^2 / (2 l^2)) through a rational approximation of
    its spectral density S(w) = var sqrt(2 pi) l exp(-l^2 w^2 / 2): the exponential in 1 / S is
    truncated after `order` + 1 terms (order even, so the polynomial has no real root), and the
    stable spectral factor gives an SDE of that order in the state (f, f', ...).  With
    lam = 1 / l the stable roots are lam r_k for fixed r_k, F is the companion matrix of
    prod (s - lam r_k), the white-noise density is q = var sqrt(2 pi) order! 2^order
    lam^(2 order - 1), and P0 solves the Lyapunov equation.  The model is the kernel this SDE
    implies (it equals the squared exponential only as order grows).  Hyperparameters
    (lengthscale, variance)."""

    n_params = 2

    def __init__(self, order, lengthscale, variance):
        n = int(order)
        if n < 2 or n % 2:
            raise ValueError("the squared-exponential approximation needs an even order >= 2")
        self.b = n
        self.ell = float(lengthscale)
        self.var = float(variance)
        self.lam = 1.0 / self.ell
        # roots in u = -r^2 / 2 of the truncated exponential, then the stable square roots
        u = np.roots([1.0 / float(scipy.special.factorial(k)) for k in range(n, -1, -1)])
        r = np.sqrt(-2.0 * u.astype(complex))
        r = np.where(r.real < 0, r, -r)
        self.unit_coeffs = np.real(np.poly(r))[1:]            # monic, s^(n-1) ... s^0
        self.kappa = np.sqrt(2.0 * np.pi) * float(scipy.special.factorial(n)) * 2.0 ** n

    def F(self):
        n, l = self.b, self.lam
        F = np.diag(np.ones(n - 1), 1)
        F[n - 1, :] = [-self.unit_coeffs[n - 1 - j] * l ** (n - j) for j in range(n)]
        return F

    def dF_dlam(self):
        n, l = self.b, self.lam
        F = np.zeros((n, n))
        F[n - 1, :] = [-self.unit_coeffs[n - 1 - j] * (n - j) * l ** (n - j - 1) for j in range(n)]
        return F

    def H(self):
        h = np.zeros(self.b)
        h[0] = 1.0
        return h

    def Pinf(self):
        n = self.b
        q = self.var * self.kappa * self.lam ** (2 * n - 1)
        W = np.zeros((n, n))
        W[n - 1, n - 1] = q
        P = scipy.linalg.solve_continuous_lyapunov(self.F(), -W)
        return 0.5 * (P + P.T)

    def dF(self):
        return [self.dF_dlam() * (-self.lam / self.ell), np.zeros((self.b, self.b))]

    def dPinf(self):
        # P_ij scales as lam^(i+j): dP/dlam = (i + j) P / lam
        i = np.arange(self.b)
        P = self.Pinf()
        dlam = (i[:, None] + i[None, :]) * P / self.lam
        return [dlam * (-self.lam / self.ell), P / self.var]

    def kernel(self, tau):
        tau = np.abs(np.asarray(tau, dtype=np.float64))
        F, P = self.F(), self.Pinf()
        out = np.array([(scipy.linalg.expm(F * x) @ P)[0, 0] for x in tau.reshape(-1)])
        return out.reshape(tau.shape)

    def kernel_untruncated(self, tau):
        return self.var * np.exp(-0.5 * (np.asarray(tau) / self.ell) ** 2)

    def dkernel(self, tau):
        tau = np.abs(np.asarray(tau, dtype=np.float64))
        F, P = self.F(), self.Pinf()
        dF, dP = self.dF(), self.dPinf()
        d_ell = []
        for x in tau.reshape(-1):
            E = scipy.linalg.expm(F * x)
            dE = scipy.linalg.expm_frechet(F * x, dF[0] * x, compute_expm=False)
            d_ell.append((dE @ P + E @ dP[0])[0, 0])
        d_ell = np.array(d_ell).reshape(tau.shape)
        return [d_ell, self.kernel(tau) / self.var]


class SumModel:
    """Sum of terms: block-diagonal state space.  Parameters are the terms' in order."""

    def __init__(self, terms, hyper_row):
        """terms: [(kind, harmonics)], hyper_row: term parameters then the noise variance."""
        self.terms = [(int(k), int(h)) for k, h in terms]
        self.hyper_row = np.array(hyper_row, dtype=np.float64)
        self.parts = []
        p = 0
        for kind, harm in terms:
            if kind in _MATERN_B:
                self.parts.append(Matern(kind, hyper_row[p], hyper_row[p + 1]))
                p += 2
            elif kind == PERIODIC:
                self.parts.append(Periodic(harm, hyper_row[p], hyper_row[p + 1], hyper_row[p + 2]))
                p += 3
            elif kind == SQEXP:
                self.parts.append(SquaredExponential(harm, hyper_row[p], hyper_row[p + 1]))
                p += 2
            elif kind == QUASIPERIODIC:
                self.parts.append(QuasiPeriodic(harm, hyper_row[p], hyper_row[p + 1], hyper_row[p + 2],
                                                hyper_row[p + 3]))
                p += 4
            else:
                raise ValueError(f"unknown kind {kind}")
        self.noise = float(hyper_row[p])
        self.n_kernel_params = p
        self.n_params = p + 1
        self.b = sum(m.b for m in self.parts)
        self._F = scipy.linalg.block_diag(*[m.F() for m in self.parts])
        self._P = scipy.linalg.block_diag(*[m.Pinf() for m in self.parts])
        self._h = np.concatenate([m.H() for m in self.parts])
        self._dF, self._dP = [], []
        for i, m in enumerate(self.parts):
            for dF, dP in zip(m.dF(), m.dPinf()):
                blocksF = [np.zeros((q.b, q.b)) for q in self.parts]
                blocksP = [np.zeros((q.b, q.b)) for q in self.parts]
                blocksF[i] = dF
                blocksP[i] = dP
                self._dF.append(scipy.linalg.block_diag(*blocksF))
                self._dP.append(scipy.linalg.block_diag(*blocksP))

    # --- model matrices -------------------------------------------------------
    def F(self):
        return self._F

    def H(self):
        return self._h

    def Pinf(self):
        return self._P

    def dPinf(self):
        """d Pinf / d theta_i for every kernel parameter (noise excluded)."""
        return self._dP

    def A(self, dt):
        """Transition over a gap dt: expm(F dt)."""
        return scipy.linalg.expm(self._F * dt)

    def Q(self, dt):
        """Process noise over a gap dt: P0 - A P0 A^T (eq. ss_matern)."""
        A = self.A(dt)
        Q = self._P - A @ self._P @ A.T
        return 0.5 * (Q + Q.T)

    def dA(self, dt):
        """[d expm(F dt)/d theta_i] via the Frechet derivative of expm."""
        out = []
        for dF in self._dF:
            if not dF.any():
                out.append(np.zeros_like(self._F))
            else:
                out.append(scipy.linalg.expm_frechet(self._F * dt, dF * dt, compute_expm=False))
        return out

    def dQ(self, dt):
        A = self.A(dt)
        out = []
        for dA, dP in zip(self.dA(dt), self._dP):
            d = dP - dA @ self._P @ A.T - A @ dP @ A.T - A @ self._P @ dA.T
            out.append(0.5 * (d + d.T))
        return out

    # --- covariance function --------------------------------------------------
    def kernel(self, tau):
        return sum(m.kernel(tau) for m in self.parts)

    def dkernel(self, tau):
        out = []
        for m in self.parts:
            out.extend(m.dkernel(tau))
        return out


def model_for(terms, hyper_row) -> SumModel:
    return SumModel(terms, hyper_row)
