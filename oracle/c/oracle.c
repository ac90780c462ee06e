/*
 * Sequential CPU oracle for temporal-GP inference in sparse-precision form.
 *
 * TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the benchmark's
 * cpu_baseline leg load this library.  It shares no code with the device path.
 *
 * What it computes (paper Sec. 2.2-3.1, Theorem 1): the block LDL^T of the
 * block-tridiagonal posterior precision Kb = Kinv + I (x) J in natural order
 * (the Thomas algorithm of Sec. 3.1), with each pivot kept in the Woodbury
 * form Dh_n = C_n^-1 + A_n^T Q_n^-1 A_n so no Q^-1 is formed:
 *     C_0 = (I + P0 J)^-1 P0,  V_n = Q_n + A_n C_n A_n^T,  C_{n+1} = (I + V_n J)^-1 V_n,
 *     log det K_y = sum_n log det(I + V_{n-1} J) + N log s2      (V_{-1} = P0, eq. det_1),
 * forward substitution x^f_n = C_n rhat_n, back substitution
 *     x_n = x^f_n + G_n (x_{n+1} - A_n x^f_n),   G_n = C_n A_n^T V_n^-1,
 * and Takahashi's selected inverse S_n = C_n + G_n (S_{n+1} - V_n) G_n^T,
 * S_{n+1,n} = S_{n+1} G_n^T (subproblems 1-3 and the BTD part of Kb^-1).
 * The gradient is the tangent-linear (forward-mode) derivative of the same
 * sequential elimination, written in its filter form.
 *
 * The state-space blocks are closed forms: A[dt] = e^{-lam dt} sum_k (N dt)^k/k!
 * with N = F + lam I nilpotent for Matern, rotations for periodic harmonics,
 * Q[dt] = P0 - A P0 A^T (eq. ss_matern).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MAXB 24
#define MAXP 16

typedef struct {
  int n_parts;
  int kind[8], harm[8], off[8], dim[8], pidx[8];
  double ell[8], var[8], period[8], lam[8], decay[8];
  double se_coef[8][MAXB];   /* squared exponential: monic unit-lengthscale coefficients */
  double q2[8][MAXB], dq2[8][MAXB];
  int b, n_kernel_params;
  double noise;
  double P[MAXB * MAXB];
  double dP[MAXP][MAXB * MAXB];
  double h[MAXB];
} model_t;

/* ---------------- small dense linear algebra (row-major b x b) ---------------- */
static void mm(int b, const double* X, const double* Y, double* Z) { /* Z = X Y */
  for (int i = 0; i < b; ++i)
    for (int j = 0; j < b; ++j) {
      double s = 0.0;
      for (int k = 0; k < b; ++k) s += X[i * b + k] * Y[k * b + j];
      Z[i * b + j] = s;
    }
}
static void mmt(int b, const double* X, const double* Y, double* Z) { /* Z = X Y^T */
  for (int i = 0; i < b; ++i)
    for (int j = 0; j < b; ++j) {
      double s = 0.0;
      for (int k = 0; k < b; ++k) s += X[i * b + k] * Y[j * b + k];
      Z[i * b + j] = s;
    }
}
static void mv(int b, const double* X, const double* v, double* w) {
  for (int i = 0; i < b; ++i) {
    double s = 0.0;
    for (int k = 0; k < b; ++k) s += X[i * b + k] * v[k];
    w[i] = s;
  }
}
static void sym(int b, double* X) {
  for (int i = 0; i < b; ++i)
    for (int j = 0; j < i; ++j) {
      double a = 0.5 * (X[i * b + j] + X[j * b + i]);
      X[i * b + j] = a;
      X[j * b + i] = a;
    }
}
/* Solve M X = R for X (M b x b, R b x m, row-major), Gaussian elimination with partial pivoting.
 * Returns log|det M| in *logabsdet (if not NULL) and 0, or -1 if M is singular. */
static int solve(int b, const double* M, double* R, int m, double* logabsdet) {
  double* a = malloc(sizeof(double) * b * b);
  if (!a) return -1;
  memcpy(a, M, sizeof(double) * b * b);
  double ld = 0.0;
  for (int c = 0; c < b; ++c) {
    int p = c;
    for (int r = c + 1; r < b; ++r)
      if (fabs(a[r * b + c]) > fabs(a[p * b + c])) p = r;
    if (a[p * b + c] == 0.0) {
      free(a);
      return -1;
    }
    if (p != c) {
      for (int k = 0; k < b; ++k) { double t = a[c * b + k]; a[c * b + k] = a[p * b + k]; a[p * b + k] = t; }
      for (int k = 0; k < m; ++k) { double t = R[c * m + k]; R[c * m + k] = R[p * m + k]; R[p * m + k] = t; }
    }
    ld += log(fabs(a[c * b + c]));
    for (int r = c + 1; r < b; ++r) {
      double f = a[r * b + c] / a[c * b + c];
      if (f == 0.0) continue;
      for (int k = c; k < b; ++k) a[r * b + k] -= f * a[c * b + k];
      for (int k = 0; k < m; ++k) R[r * m + k] -= f * R[c * m + k];
    }
  }
  for (int c = b - 1; c >= 0; --c) {
    for (int k = 0; k < m; ++k) {
      double s = R[c * m + k];
      for (int j = c + 1; j < b; ++j) s -= a[c * b + j] * R[j * m + k];
      R[c * m + k] = s / a[c * b + c];
    }
  }
  if (logabsdet) *logabsdet = ld;
  free(a);
  return 0;
}

/* ---------------- squared-exponential approximation ---------------- */
/* Monic coefficients (s^0 .. s^(n-1)) of prod_k (s - r_k) over the stable roots r_k of
   sum_{m<=n} (-r^2/2)^m / m! (n even): the truncated exponential's roots u_k found by
   Durand-Kerner iteration, r_k = the square root of -2 u_k with negative real part. */
static int se_unit_coeffs(int n, double* coef) {
  if (n < 2 || n % 2 || n > 16) return -1;
  double complex c[17], z[16];
  double fact = 1.0;
  for (int m = 0; m <= n; ++m) {
    if (m > 0) fact *= m;
    c[m] = 1.0 / fact;                         /* u^m coefficient */
  }
  for (int m = 0; m <= n; ++m) c[m] /= (1.0 / fact);   /* monic in u */
  for (int k = 0; k < n; ++k) z[k] = cpow(0.4 + 0.9 * I, k);
  for (int it = 0; it < 2000; ++it) {
    double moved = 0.0;
    for (int k = 0; k < n; ++k) {
      double complex pv = c[n];
      for (int m = n - 1; m >= 0; --m) pv = pv * z[k] + c[m];
      double complex den = 1.0;
      for (int j = 0; j < n; ++j)
        if (j != k) den *= (z[k] - z[j]);
      double complex dz = pv / den;
      z[k] -= dz;
      moved = fmax(moved, cabs(dz) / fmax(1.0, cabs(z[k])));
    }
    if (moved < 1e-16) break;
  }
  double complex poly[17];
  poly[0] = 1.0;
  for (int m = 1; m <= n; ++m) poly[m] = 0.0;
  for (int k = 0; k < n; ++k) {
    double complex r = csqrt(-2.0 * z[k]);
    if (creal(r) > 0) r = -r;
    /* multiply by (s - r): poly holds coefficients of s^0 .. s^k */
    for (int m = k + 1; m >= 1; --m) poly[m] = poly[m - 1] - r * poly[m];
    poly[0] = -r * poly[0];
  }
  for (int m = 0; m < n; ++m) coef[m] = creal(poly[m]);
  return 0;
}

/* exp(X) by scaling and squaring of the Taylor series (b x b). */
static void expm_taylor(int b, const double* X, double* E) {
  double nrm = 0.0;
  for (int i = 0; i < b; ++i) {
    double r = 0.0;
    for (int j = 0; j < b; ++j) r += fabs(X[i * b + j]);
    if (r > nrm) nrm = r;
  }
  int sq = 0;
  while (nrm > 0.25) {
    nrm *= 0.5;
    ++sq;
  }
  double Y[MAXB * MAXB], T[MAXB * MAXB], U[MAXB * MAXB];
  double sc = ldexp(1.0, -sq);
  for (int k = 0; k < b * b; ++k) Y[k] = X[k] * sc;
  for (int k = 0; k < b * b; ++k) { E[k] = (k / b == k % b) ? 1.0 : 0.0; T[k] = E[k]; }
  for (int m = 1; m <= 24; ++m) {
    mm(b, T, Y, U);
    for (int k = 0; k < b * b; ++k) { T[k] = U[k] / m; E[k] += T[k]; }
  }
  for (int q = 0; q < sq; ++q) {
    mm(b, E, E, U);
    memcpy(E, U, sizeof(double) * b * b);
  }
}

/* Stationary covariance: F P + P F^T + q e_n e_n^T = 0 solved for the n(n+1)/2 entries of the
   symmetric P (companion F). */
static int lyap_companion(int n, const double* F, double q, double* P) {
  int nu = n * (n + 1) / 2;
  if (n > 16) return -1;
  double* M = calloc((size_t)nu * nu, sizeof(double));
  double* R = malloc(sizeof(double) * nu);
  if (!M || !R) {
    free(M);
    free(R);
    return -1;
  }
  int idx[16][16];
  for (int i = 0, k = 0; i < n; ++i)
    for (int j = i; j < n; ++j, ++k) idx[i][j] = idx[j][i] = k;
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) {
      int row = idx[i][j];
      for (int k = 0; k < n; ++k) {
        M[row * nu + idx[k][j]] += F[i * n + k];   /* (F P)_ij */
        M[row * nu + idx[i][k]] += F[j * n + k];   /* (P F^T)_ij */
      }
      R[row] = (i == n - 1 && j == n - 1) ? -q : 0.0;
    }
  const int rc = solve(nu, M, R, 1, NULL);
  if (rc == 0)
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) P[i * n + j] = R[idx[i][j]];
  free(M);
  free(R);
  return rc;
}

/* F of the squared-exponential term at lam = 1 / l. */
static void se_F(const model_t* m, int i, double* F) {
  int n = m->dim[i];
  double l = m->lam[i];
  memset(F, 0, sizeof(double) * n * n);
  for (int r = 0; r + 1 < n; ++r) F[r * n + r + 1] = 1.0;
  for (int c = 0; c < n; ++c) F[(n - 1) * n + c] = -m->se_coef[i][c] * pow(l, n - c);
}

/* ---------------- model ---------------- */
/* e^{-z} I_j(z) by its power series, terms summed in log space. */
static double bessel_ive(int j, double z) {
  if (j < 0) j = -j;
  if (z == 0.0) return j == 0 ? 1.0 : 0.0;
  double s = 0.0;
  double lz2 = log(0.5 * z);
  for (int k = 0; k < 2000; ++k) {
    double lt = (2.0 * k + j) * lz2 - lgamma(k + 1.0) - lgamma(k + j + 1.0) - z;
    double term = exp(lt);
    s += term;
    if (k > z && term < 1e-18 * s) break;
  }
  return s;
}

static int model_init(model_t* m, int n_terms, const int* kinds, const int* harm, const double* hyper) {
  if (n_terms < 1 || n_terms > 8) return -1;
  memset(m, 0, sizeof(*m));
  m->n_parts = n_terms;
  int b = 0, p = 0;
  for (int i = 0; i < n_terms; ++i) {
    m->kind[i] = kinds[i];
    m->harm[i] = harm[i];
    m->off[i] = b;
    m->pidx[i] = p;
    if (kinds[i] == 1 || kinds[i] == 2 || kinds[i] == 4 || kinds[i] == 5) {
      /* Matern nu = dim - 1/2: kinds 4, 1, 2, 5 are nu = 1/2, 3/2, 5/2, 7/2 */
      m->dim[i] = kinds[i] == 4 ? 1 : kinds[i] == 1 ? 2 : kinds[i] == 2 ? 3 : 4;
      m->ell[i] = hyper[p];
      m->var[i] = hyper[p + 1];
      m->lam[i] = sqrt(2.0 * m->dim[i] - 1.0) / m->ell[i];
      p += 2;
    } else if (kinds[i] == 7) {
      /* squared exponential through its spectral approximation of order harm[i] */
      m->dim[i] = harm[i];
      m->ell[i] = hyper[p];
      m->var[i] = hyper[p + 1];
      m->lam[i] = 1.0 / m->ell[i];
      if (se_unit_coeffs(harm[i], m->se_coef[i])) return -1;
      p += 2;
    } else if (kinds[i] == 3 || kinds[i] == 6) {
      /* periodic; kind 6 (quasi-periodic) also decays every harmonic by exp(-dt / decay) */
      m->dim[i] = 2 * (harm[i] + 1);
      m->ell[i] = hyper[p];
      m->var[i] = hyper[p + 1];
      m->period[i] = hyper[p + 2];
      if (kinds[i] == 6) {
        m->decay[i] = hyper[p + 3];
        p += 1;
      }
      double z = 1.0 / (m->ell[i] * m->ell[i]);
      for (int j = 0; j <= harm[i]; ++j) {
        double c = j == 0 ? 1.0 : 2.0;
        m->q2[i][j] = c * bessel_ive(j, z);
        m->dq2[i][j] = c * (0.5 * (bessel_ive(j - 1, z) + bessel_ive(j + 1, z)) - bessel_ive(j, z));
      }
      p += 3;
    } else {
      return -1;
    }
    b += m->dim[i];
  }
  if (b > MAXB || p + 1 > MAXP) return -1;
  m->b = b;
  m->n_kernel_params = p;
  m->noise = hyper[p];
  /* stationary covariance, its parameter derivatives and h */
  for (int i = 0; i < n_terms; ++i) {
    int o = m->off[i];
    int pi = m->pidx[i];
    if (m->kind[i] == 7) {
      /* q = var sqrt(2 pi) n! 2^n lam^(2n - 1); P_rc scales as lam^(r+c) */
      int n = m->dim[i];
      double l = m->lam[i], dl = -l / m->ell[i], fact = 1.0;
      for (int k = 2; k <= n; ++k) fact *= k;
      double q = m->var[i] * sqrt(2.0 * M_PI) * fact * pow(2.0, n) * pow(l, 2 * n - 1);
      double F[MAXB * MAXB], Ps[MAXB * MAXB];
      se_F(m, i, F);
      if (lyap_companion(n, F, q, Ps)) return -1;
      for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) {
          double v = 0.5 * (Ps[r * n + c] + Ps[c * n + r]);
          m->P[(o + r) * b + o + c] = v;
          m->dP[pi][(o + r) * b + o + c] = (r + c) * v / l * dl;
          m->dP[pi + 1][(o + r) * b + o + c] = v / m->var[i];
        }
      m->h[o] = 1.0;
    } else if (m->kind[i] == 4) {
      m->P[o * b + o] = m->var[i];
      m->dP[pi + 1][o * b + o] = 1.0;
      m->h[o] = 1.0;
    } else if (m->kind[i] == 5) {
      /* entry (r, c) = (-1)^c times the (r + c)-th derivative of k at 0; those are
         -v l^2/5 (second), v l^4/5 (fourth), -v l^6 (sixth) */
      double l = m->lam[i], v = m->var[i], dl = -l / m->ell[i];
      double l2 = l * l, l4 = l2 * l2;
      double Pm[16] = {1.0, 0.0, -l2 / 5.0, 0.0, 0.0, l2 / 5.0, 0.0, -l4 / 5.0,
                       -l2 / 5.0, 0.0, l4 / 5.0, 0.0, 0.0, -l4 / 5.0, 0.0, l4 * l2};
      double dPm[16] = {0.0, 0.0, -2.0 * l / 5.0, 0.0, 0.0, 2.0 * l / 5.0, 0.0, -4.0 * l2 * l / 5.0,
                        -2.0 * l / 5.0, 0.0, 4.0 * l2 * l / 5.0, 0.0, 0.0, -4.0 * l2 * l / 5.0, 0.0,
                        6.0 * l4 * l};
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
          m->P[(o + r) * b + o + c] = v * Pm[r * 4 + c];
          m->dP[pi][(o + r) * b + o + c] = v * dPm[r * 4 + c] * dl;
          m->dP[pi + 1][(o + r) * b + o + c] = Pm[r * 4 + c];
        }
      m->h[o] = 1.0;
    } else if (m->kind[i] == 1) {
      double l = m->lam[i], v = m->var[i], dl = -l / m->ell[i];
      m->P[o * b + o] = v;
      m->P[(o + 1) * b + o + 1] = v * l * l;
      m->dP[pi][(o + 1) * b + o + 1] = v * 2.0 * l * dl;
      m->dP[pi + 1][o * b + o] = 1.0;
      m->dP[pi + 1][(o + 1) * b + o + 1] = l * l;
      m->h[o] = 1.0;
    } else if (m->kind[i] == 2) {
      double l = m->lam[i], v = m->var[i], dl = -l / m->ell[i];
      double Pm[9] = {1.0, 0.0, -l * l / 3.0, 0.0, l * l / 3.0, 0.0, -l * l / 3.0, 0.0, l * l * l * l};
      double dPm[9] = {0.0, 0.0, -2.0 * l / 3.0, 0.0, 2.0 * l / 3.0, 0.0, -2.0 * l / 3.0, 0.0, 4.0 * l * l * l};
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          m->P[(o + r) * b + o + c] = v * Pm[r * 3 + c];
          m->dP[pi][(o + r) * b + o + c] = v * dPm[r * 3 + c] * dl;
          m->dP[pi + 1][(o + r) * b + o + c] = Pm[r * 3 + c];
        }
      m->h[o] = 1.0;
    } else {
      double dz = -2.0 / (m->ell[i] * m->ell[i] * m->ell[i]);
      for (int j = 0; j <= m->harm[i]; ++j)
        for (int r = 0; r < 2; ++r) {
          int d = o + 2 * j + r;
          m->P[d * b + d] = m->var[i] * m->q2[i][j];
          m->dP[pi][d * b + d] = m->var[i] * m->dq2[i][j] * dz;
          m->dP[pi + 1][d * b + d] = m->q2[i][j];
        }
      for (int j = 0; j <= m->harm[i]; ++j) m->h[o + 2 * j] = 1.0;
    }
  }
  return 0;
}

/* A[dt] and (optionally) dA[dt]/dtheta_k for every kernel parameter k. */
static void model_A(const model_t* m, double dt, double* A, double (*dA)[MAXB * MAXB]) {
  int b = m->b;
  memset(A, 0, sizeof(double) * b * b);
  if (dA)
    for (int k = 0; k < m->n_kernel_params; ++k) memset(dA[k], 0, sizeof(double) * b * b);
  for (int i = 0; i < m->n_parts; ++i) {
    int o = m->off[i], pi = m->pidx[i];
    if (m->kind[i] == 7) {
      /* A = expm(F dt); with F = lam D C1 D^-1 (D = diag(lam^r)) and x = lam dt,
         dA/dlam = ((r - c) / lam) A_rc + (dt / lam) (F A)_rc */
      int n = m->dim[i];
      double l = m->lam[i], dl = -l / m->ell[i];
      double F[MAXB * MAXB], X[MAXB * MAXB], E[MAXB * MAXB], FE[MAXB * MAXB];
      se_F(m, i, F);
      for (int k = 0; k < n * n; ++k) X[k] = F[k] * dt;
      expm_taylor(n, X, E);
      mm(n, F, E, FE);
      for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) {
          A[(o + r) * b + o + c] = E[r * n + c];
          if (dA) dA[pi][(o + r) * b + o + c] = ((r - c) / l * E[r * n + c] + dt / l * FE[r * n + c]) * dl;
        }
    } else if (m->kind[i] != 3 && m->kind[i] != 6) {
      /* Matern: F is the companion matrix of (s + l)^d; N = F + l I is nilpotent (N^d = 0) and
         A = e^{-l dt} (I + N dt + N^2 dt^2/2 + N^3 dt^3/6); dN/dl = dF/dl + I */
      int d = m->dim[i];
      double l = m->lam[i];
      double N[16] = {0}, Nd[16] = {0};
      for (int r = 0; r + 1 < d; ++r) {
        N[r * d + r] = l;
        N[r * d + r + 1] = 1.0;
        Nd[r * d + r] = 1.0;
      }
      for (int c = 0; c < d; ++c) {
        /* last row of F: -C(d, c) l^(d - c) */
        double binom = 1.0;
        for (int q = 0; q < c; ++q) binom = binom * (d - q) / (q + 1);
        N[(d - 1) * d + c] = -binom * pow(l, d - c);
        Nd[(d - 1) * d + c] = -binom * (d - c) * pow(l, d - c - 1);
      }
      N[(d - 1) * d + d - 1] += l;
      Nd[(d - 1) * d + d - 1] += 1.0;
      double N2[16], N3[16], NdN[16], NNd[16], T1[16], T2[16], T3[16];
      mm(d, N, N, N2);
      mm(d, N2, N, N3);
      mm(d, Nd, N, NdN);
      mm(d, N, Nd, NNd);
      mm(d, Nd, N2, T1);    /* Nd N^2 */
      mm(d, N, NdN, T2);    /* N Nd N */
      mm(d, N2, Nd, T3);    /* N^2 Nd */
      double e = exp(-l * dt);
      double dl = -l / m->ell[i];
      for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
          int q = r * d + c;
          double poly = (r == c ? 1.0 : 0.0) + N[q] * dt + 0.5 * N2[q] * dt * dt + N3[q] * dt * dt * dt / 6.0;
          double a = e * poly;
          A[(o + r) * b + o + c] = a;
          if (dA) {
            double dpoly = Nd[q] * dt + 0.5 * (NdN[q] + NNd[q]) * dt * dt + (T1[q] + T2[q] + T3[q]) * dt * dt * dt / 6.0;
            dA[pi][(o + r) * b + o + c] = (-dt * a + e * dpoly) * dl;
          }
        }
    } else {
      double w0 = 2.0 * M_PI / m->period[i];
      int quasi = m->kind[i] == 6;
      double e = quasi ? exp(-dt / m->decay[i]) : 1.0;
      double de = quasi ? e * dt / (m->decay[i] * m->decay[i]) : 0.0;   /* d e / d decay */
      for (int j = 0; j <= m->harm[i]; ++j) {
        double ang = j * w0 * dt;
        double c = cos(ang), s = sin(ang);
        int d = o + 2 * j;
        A[d * b + d] = e * c;
        A[d * b + d + 1] = -e * s;
        A[(d + 1) * b + d] = e * s;
        A[(d + 1) * b + d + 1] = e * c;
        if (dA) {
          double dang = -ang / m->period[i];
          dA[pi + 2][d * b + d] = -e * s * dang;
          dA[pi + 2][d * b + d + 1] = -e * c * dang;
          dA[pi + 2][(d + 1) * b + d] = e * c * dang;
          dA[pi + 2][(d + 1) * b + d + 1] = -e * s * dang;
          if (quasi) {
            dA[pi + 3][d * b + d] = de * c;
            dA[pi + 3][d * b + d + 1] = -de * s;
            dA[pi + 3][(d + 1) * b + d] = de * s;
            dA[pi + 3][(d + 1) * b + d + 1] = de * c;
          }
        }
      }
    }
  }
}

static void model_Q(const model_t* m, const double* A, double* Q) {
  int b = m->b;
  double T[MAXB * MAXB], U[MAXB * MAXB];
  mm(b, A, m->P, T);
  mmt(b, T, A, U);
  for (int i = 0; i < b * b; ++i) Q[i] = m->P[i] - U[i];
  sym(b, Q);
}

/* ---------------- exported entry points ---------------- */
int spo_state_dim(int n_terms, const int* kinds, const int* harm, const double* hyper) {
  model_t m;
  if (model_init(&m, n_terms, kinds, harm, hyper)) return -1;
  return m.b;
}

/* Closed-form A_n, Q_n (row-major b x b per edge) and the stationary covariance. */
int spo_edges(int n_terms, const int* kinds, const int* harm, const double* hyper, int64_t n,
              const double* t, double* A, double* Q, double* Pinf, double* h) {
  model_t m;
  if (model_init(&m, n_terms, kinds, harm, hyper)) return -1;
  int b = m.b;
  for (int64_t i = 0; i + 1 < n; ++i) {
    model_A(&m, t[i + 1] - t[i], A + i * b * b, NULL);
    model_Q(&m, A + i * b * b, Q + i * b * b);
  }
  if (Pinf) memcpy(Pinf, m.P, sizeof(double) * b * b);
  if (h) memcpy(h, m.h, sizeof(double) * b);
  return 0;
}

/*
 * Sequential BTD elimination (factored pivots).  Outputs may be NULL.
 * scalars[0..2] = logML, data fit y^T K_y^-1 y, log det K_y.
 * z_mean: n x b, S_diag: n x b x b, S_sub: (n-1) x b x b with S_sub[n] = Cov(z_{n+1}, z_n | y).
 */
int spo_btd_factored(int n_terms, const int* kinds, const int* harm, const double* hyper, int64_t n,
                     const double* t, const double* y, double* scalars, double* f_mean, double* f_var,
                     double* z_mean, double* S_diag, double* S_sub) {
  model_t m;
  if (n < 1 || model_init(&m, n_terms, kinds, harm, hyper)) return -1;
  const int b = m.b, bb = b * b;
  const double s2 = m.noise;
  double* C = (double*)malloc(sizeof(double) * bb * n);
  double* xf = (double*)malloc(sizeof(double) * b * n);
  if (!C || !xf) { free(C); free(xf); return -2; }
  double Vprev[MAXB * MAXB], xpred[MAXB], Mx[MAXB * MAXB], R[MAXB * (MAXB + 1)];
  double A[MAXB * MAXB], Q[MAXB * MAXB], T[MAXB * MAXB];
  memcpy(Vprev, m.P, sizeof(double) * bb);
  memset(xpred, 0, sizeof(xpred));
  double logdet_terms = 0.0;
  int bad = 0;
  for (int64_t i = 0; i < n; ++i) {
    /* Mx = I + V J, J = h h^T / s2 */
    double Vh[MAXB];
    mv(b, Vprev, m.h, Vh);
    for (int r = 0; r < b; ++r)
      for (int c = 0; c < b; ++c) Mx[r * b + c] = (r == c ? 1.0 : 0.0) + Vh[r] * m.h[c] / s2;
    /* R = [V | V eta + A x^f] and solve Mx [C | x^f] = R */
    for (int r = 0; r < b; ++r) {
      for (int c = 0; c < b; ++c) R[r * (b + 1) + c] = Vprev[r * b + c];
      R[r * (b + 1) + b] = Vh[r] * y[i] / s2 + xpred[r];
    }
    double ld;
    if (solve(b, Mx, R, b + 1, &ld)) { bad = 1; break; }
    logdet_terms += ld;
    for (int r = 0; r < b; ++r) {
      for (int c = 0; c < b; ++c) C[i * bb + r * b + c] = R[r * (b + 1) + c];
      xf[i * b + r] = R[r * (b + 1) + b];
    }
    sym(b, C + i * bb);
    if (i + 1 < n) {
      model_A(&m, t[i + 1] - t[i], A, NULL);
      model_Q(&m, A, Q);
      mm(b, A, C + i * bb, T);
      mmt(b, T, A, Vprev);
      for (int k = 0; k < bb; ++k) Vprev[k] += Q[k];
      sym(b, Vprev);
      mv(b, A, xf + i * b, xpred);
    }
  }
  if (bad) { free(C); free(xf); return -3; }
  /* back substitution and Takahashi recursion, newest first */
  double x[MAXB], xn[MAXB], S[MAXB * MAXB], Sn[MAXB * MAXB], G[MAXB * MAXB], GT[MAXB * MAXB];
  double datafit_quad = 0.0, yy = 0.0;
  memcpy(xn, xf + (n - 1) * b, sizeof(double) * b);
  memcpy(Sn, C + (n - 1) * bb, sizeof(double) * bb);
  for (int64_t i = n - 1; i >= 0; --i) {
    if (i == n - 1) {
      memcpy(x, xn, sizeof(double) * b);
      memcpy(S, Sn, sizeof(double) * bb);
    } else {
      double V[MAXB * MAXB], Ax[MAXB], d[MAXB], U[MAXB * MAXB], W[MAXB * MAXB];
      model_A(&m, t[i + 1] - t[i], A, NULL);
      model_Q(&m, A, Q);
      mm(b, A, C + i * bb, T);            /* T = A C */
      mmt(b, T, A, V);
      for (int k = 0; k < bb; ++k) V[k] += Q[k];
      sym(b, V);
      memcpy(GT, T, sizeof(double) * bb); /* G^T = V^-1 A C */
      if (solve(b, V, GT, b, NULL)) { free(C); free(xf); return -3; }
      for (int r = 0; r < b; ++r)
        for (int c = 0; c < b; ++c) G[r * b + c] = GT[c * b + r];
      mv(b, A, xf + i * b, Ax);
      for (int r = 0; r < b; ++r) d[r] = xn[r] - Ax[r];
      mv(b, G, d, x);
      for (int r = 0; r < b; ++r) x[r] += xf[i * b + r];
      for (int k = 0; k < bb; ++k) U[k] = Sn[k] - V[k];
      mm(b, G, U, W);
      mmt(b, W, G, S);
      for (int k = 0; k < bb; ++k) S[k] += C[i * bb + k];
      sym(b, S);
      if (S_sub) mm(b, Sn, GT, S_sub + i * bb);
    }
    double fm = 0.0, fv = 0.0;
    for (int r = 0; r < b; ++r) {
      fm += m.h[r] * x[r];
      for (int c = 0; c < b; ++c) fv += m.h[r] * S[r * b + c] * m.h[c];
    }
    if (f_mean) f_mean[i] = fm;
    if (f_var) f_var[i] = fv;
    if (z_mean) memcpy(z_mean + i * b, x, sizeof(double) * b);
    if (S_diag) memcpy(S_diag + i * bb, S, sizeof(double) * bb);
    datafit_quad += (y[i] / s2) * fm;
    yy += y[i] * y[i];
    memcpy(xn, x, sizeof(double) * b);
    memcpy(Sn, S, sizeof(double) * bb);
  }
  double logdet = logdet_terms + (double)n * log(s2);
  double datafit = yy / s2 - datafit_quad;
  if (scalars) {
    scalars[0] = -0.5 * datafit - 0.5 * logdet - 0.5 * (double)n * log(2.0 * M_PI);
    scalars[1] = datafit;
    scalars[2] = logdet;
  }
  free(C);
  free(xf);
  return 0;
}

/* logML and its tangent-linear gradient (kernel parameters in order, then s2). */
int spo_tangent_grad(int n_terms, const int* kinds, const int* harm, const double* hyper, int64_t n,
                     const double* t, const double* y, double* logml, double* grad) {
  model_t m;
  if (n < 1 || model_init(&m, n_terms, kinds, harm, hyper)) return -1;
  const int b = m.b, bb = b * b, np_ = m.n_kernel_params + 1;
  const double s2 = m.noise;
  double mu[MAXB] = {0}, P[MAXB * MAXB];
  static __thread double dm[MAXP][MAXB], dP[MAXP][MAXB * MAXB], dA[MAXP][MAXB * MAXB];
  memcpy(P, m.P, sizeof(double) * bb);
  for (int k = 0; k < np_; ++k) {
    memset(dm[k], 0, sizeof(dm[k]));
    if (k < m.n_kernel_params) memcpy(dP[k], m.dP[k], sizeof(double) * bb);
    else memset(dP[k], 0, sizeof(dP[k]));
  }
  double ll = 0.0, g[MAXP] = {0};
  double A[MAXB * MAXB], Q[MAXB * MAXB], T[MAXB * MAXB], U[MAXB * MAXB], W[MAXB * MAXB];
  for (int64_t i = 0; i < n; ++i) {
    if (i > 0) {
      model_A(&m, t[i] - t[i - 1], A, dA);
      model_Q(&m, A, Q);
      for (int k = 0; k < np_; ++k) {
        double v1[MAXB], v2[MAXB];
        if (k < m.n_kernel_params) {
          /* dQ = dP0 - dA P0 A^T - A dP0 A^T - A P0 dA^T */
          double dQ[MAXB * MAXB], X[MAXB * MAXB];
          mm(b, dA[k], m.P, T);
          mmt(b, T, A, U);
          mm(b, A, m.dP[k], X);
          mmt(b, X, A, W);
          for (int e = 0; e < bb; ++e) dQ[e] = m.dP[k][e] - U[e] - W[e];
          for (int r = 0; r < b; ++r)
            for (int c = 0; c < b; ++c) dQ[r * b + c] -= U[c * b + r];
          /* dP' = dA P A^T + A dP A^T + A P dA^T + dQ */
          mm(b, dA[k], P, T);
          mmt(b, T, A, U);
          mm(b, A, dP[k], X);
          mmt(b, X, A, W);
          for (int r = 0; r < b; ++r)
            for (int c = 0; c < b; ++c) dP[k][r * b + c] = U[r * b + c] + U[c * b + r] + W[r * b + c] + dQ[r * b + c];
          mv(b, dA[k], mu, v1);
          mv(b, A, dm[k], v2);
          for (int r = 0; r < b; ++r) dm[k][r] = v1[r] + v2[r];
        } else {
          double X[MAXB * MAXB];
          mm(b, A, dP[k], X);
          mmt(b, X, A, dP[k]);
          mv(b, A, dm[k], v2);
          memcpy(dm[k], v2, sizeof(double) * b);
        }
        sym(b, dP[k]);
      }
      double mn[MAXB];
      mv(b, A, mu, mn);
      memcpy(mu, mn, sizeof(double) * b);
      mm(b, A, P, T);
      mmt(b, T, A, U);
      for (int e = 0; e < bb; ++e) P[e] = U[e] + Q[e];
      sym(b, P);
    }
    double u[MAXB];
    mv(b, P, m.h, u);
    double s = s2, v = y[i];
    for (int r = 0; r < b; ++r) { s += m.h[r] * u[r]; v -= m.h[r] * mu[r]; }
    ll += -0.5 * log(2.0 * M_PI * s) - 0.5 * v * v / s;
    for (int k = 0; k < np_; ++k) {
      double du[MAXB];
      mv(b, dP[k], m.h, du);
      double ds = (k == np_ - 1) ? 1.0 : 0.0, dv = 0.0;
      for (int r = 0; r < b; ++r) { ds += m.h[r] * du[r]; dv -= m.h[r] * dm[k][r]; }
      g[k] += -0.5 * ds / s - v * dv / s + 0.5 * v * v * ds / (s * s);
      for (int r = 0; r < b; ++r) {
        double dK = (du[r] - u[r] * ds / s) / s;
        dm[k][r] += dK * v + (u[r] / s) * dv;
      }
      for (int r = 0; r < b; ++r)
        for (int c = 0; c < b; ++c)
          dP[k][r * b + c] += -(du[r] * u[c] + u[r] * du[c]) / s + u[r] * u[c] * ds / (s * s);
    }
    for (int r = 0; r < b; ++r) mu[r] += u[r] / s * v;
    for (int r = 0; r < b; ++r)
      for (int c = 0; c < b; ++c) P[r * b + c] -= u[r] * u[c] / s;
    sym(b, P);
  }
  if (logml) *logml = ll;
  if (grad) memcpy(grad, g, sizeof(double) * np_);
  return 0;
}
