// Device building blocks for temporal-GP inference in sparse-precision form (gfx950).
//
// The posterior precision of the stacked states is block tridiagonal (Theorem 1 of
// Grigorievskiy, Lawrence & Sarkka, arXiv:1610.08035).  It is kept in the factored form
// the theorem gives, Kinv = A^-T Q^-1 A^-1, i.e. per edge n (nodes n -> n+1) the pair
// (A_n, Q_n) and per node the observation information J = h h^T / s2, eta_n = h y_n / s2.
// Eliminating a node of that chain is a Gaussian integral that never needs Q^-1:
//
//   element  E(i -> j) = exp(c - 1/2 z_i^T J z_i + eta^T z_i) N(z_j; A z_i + b, Q)
//   E1 (x) E2 integrates the junction node k of E1(i -> k) E2(k -> j) with
//      Gam = (I + Q1 J2)^-1,  P+ = Gam Q1,  W = J2 Gam,
//      A = A2 Gam A1,  b = A2 Gam (b1 + Q1 eta2) + b2,  Q = A2 P+ A2^T + Q2,
//      J = J1 + A1^T W A1,  eta = eta1 + A1^T (Gam^T eta2 - W b1),
//      c = c1 + c2 - 1/2 log det(I + Q1 J2) - 1/2 b1^T W b1 + eta2^T Gam b1 + 1/2 eta2^T P+ eta2
//
// which is the Schur complement of the block-tridiagonal matrix at node k written in
// conditional (Woodbury) form.  It is associative, so odd-even cyclic reduction over the
// chain is a balanced tree of (x); a lane's run of consecutive nodes is folded with the
// cheaper rank-one case J2 = h h^T / s2.  The log marginal likelihood is the sum of the
// c's plus the per-node constants (eq. ml2 through the determinant lemma eq. det_1).
//
// The reverse sweep inside a chunk is the natural-order elimination (Thomas) seeded with
// the exact pivot the reduction hands to the chunk's first node, followed by its
// hand-written adjoint.  With lam = dL/dm, Lam = dL/dP of a state N(m, P) and
// Lhat = lam lam^T - 2 Lam (carried by its own recursion, never by that difference):
//   mean       mu = m + P lam,                      (subproblem 1)
//   covariance S = P - P Lhat P,                    (subproblem 2, diagonal blocks)
//   lag one    S_{n+1,n} = (I - P_{n+1} Lhat_{n+1}) A_n P+_n,
// and the edge adjoints A_bar, Q_bar, which contract with dA/dtheta and dP0/dtheta into
// d logML / d theta (subproblem 4 / eq. dd1 without forming any trace).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spg {

#define SPG_DEV __device__ __forceinline__
#define SPG_UNROLL _Pragma("unroll")

constexpr double kLog2Pi = 1.8378770664093454836;

// Work-group barrier that orders LDS accesses only: global loads and stores issued before it stay
// in flight (a plain __syncthreads also waits for every outstanding global access of the
// thread).  For exchanges through LDS; data passed through global memory needs __syncthreads.
SPG_DEV void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ------------------------------------------------------------------ small dense algebra
// All matrices are row-major register arrays with compile-time sizes; every loop unrolls.
template <int B>
SPG_DEV void mat_copy(const double (&X)[B][B], double (&Y)[B][B]) {
  SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j) Y[i][j] = X[i][j];
}
template <int B>
SPG_DEV void mat_zero(double (&X)[B][B]) {
  SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j) X[i][j] = 0.0;
}
template <int B>
SPG_DEV void mat_eye(double (&X)[B][B]) {
  SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j) X[i][j] = (i == j) ? 1.0 : 0.0;
}
// Z = X Y
template <int B>
SPG_DEV void mm(const double (&X)[B][B], const double (&Y)[B][B], double (&Z)[B][B]) {
  SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j) {
    double s = X[i][0] * Y[0][j];
    SPG_UNROLL for (int k = 1; k < B; ++k) s = fma(X[i][k], Y[k][j], s);
    Z[i][j] = s;
  }
}
// Z = X^T Y
template <int B>
SPG_DEV void mtm(const double (&X)[B][B], const double (&Y)[B][B], double (&Z)[B][B]) {
  SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j) {
    double s = X[0][i] * Y[0][j];
    SPG_UNROLL for (int k = 1; k < B; ++k) s = fma(X[k][i], Y[k][j], s);
    Z[i][j] = s;
  }
}
// Z = X Y^T, symmetric result assumed (upper computed, mirrored)
template <int B>
SPG_DEV void mmt_sym(const double (&X)[B][B], const double (&Y)[B][B], double (&Z)[B][B]) {
  SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = i; j < B; ++j) {
    double s = X[i][0] * Y[j][0];
    SPG_UNROLL for (int k = 1; k < B; ++k) s = fma(X[i][k], Y[j][k], s);
    Z[i][j] = s;
  }
  SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < i; ++j) Z[i][j] = Z[j][i];
}
// Z = X^T Y, symmetric result assumed
template <int B>
SPG_DEV void mtm_sym(const double (&X)[B][B], const double (&Y)[B][B], double (&Z)[B][B]) {
  SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = i; j < B; ++j) {
    double s = X[0][i] * Y[0][j];
    SPG_UNROLL for (int k = 1; k < B; ++k) s = fma(X[k][i], Y[k][j], s);
    Z[i][j] = s;
  }
  SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < i; ++j) Z[i][j] = Z[j][i];
}
template <int B>
SPG_DEV void mv(const double (&X)[B][B], const double (&v)[B], double (&w)[B]) {
  SPG_UNROLL for (int i = 0; i < B; ++i) {
    double s = X[i][0] * v[0];
    SPG_UNROLL for (int k = 1; k < B; ++k) s = fma(X[i][k], v[k], s);
    w[i] = s;
  }
}
template <int B>
SPG_DEV void mtv(const double (&X)[B][B], const double (&v)[B], double (&w)[B]) {
  SPG_UNROLL for (int i = 0; i < B; ++i) {
    double s = X[0][i] * v[0];
    SPG_UNROLL for (int k = 1; k < B; ++k) s = fma(X[k][i], v[k], s);
    w[i] = s;
  }
}
template <int B>
SPG_DEV double dot(const double (&a)[B], const double (&b)[B]) {
  double s = a[0] * b[0];
  SPG_UNROLL for (int k = 1; k < B; ++k) s = fma(a[k], b[k], s);
  return s;
}
template <int B>
SPG_DEV double frob(const double (&X)[B][B], const double (&Y)[B][B]) {
  double s = 0.0;
  SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j) s = fma(X[i][j], Y[i][j], s);
  return s;
}
template <int B>
SPG_DEV void symmetrize(double (&X)[B][B]) {
  SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = i + 1; j < B; ++j) {
    double a = 0.5 * (X[i][j] + X[j][i]);
    X[i][j] = a;
    X[j][i] = a;
  }
}

// Inverse of a general B x B matrix by Gauss-Jordan elimination with partial pivoting;
// returns log|det|.  Row exchanges are done with selects so every index stays static.
// Used on M = I + Q J with Q, J >= 0, whose eigenvalues are all >= 1.
template <int B>
SPG_DEV double inv_logdet(const double (&Min)[B][B], double (&G)[B][B]) {
  double a[B][B];
  mat_copy<B>(Min, a);
  mat_eye<B>(G);
  double pivprod = 1.0;
  SPG_UNROLL for (int c = 0; c < B; ++c) {
    // pivot row p >= c with the largest |a[p][c]|; exchange rows c and p of a and G
    SPG_UNROLL for (int r = c + 1; r < B; ++r) {
      const bool sw = fabs(a[r][c]) > fabs(a[c][c]);
      SPG_UNROLL for (int k = 0; k < B; ++k) {
        const double x = a[c][k], y = a[r][k];
        a[c][k] = sw ? y : x;
        a[r][k] = sw ? x : y;
        const double gx = G[c][k], gy = G[r][k];
        G[c][k] = sw ? gy : gx;
        G[r][k] = sw ? gx : gy;
      }
    }
    const double piv = a[c][c];
    pivprod *= piv;
    const double ip = 1.0 / piv;
    SPG_UNROLL for (int k = 0; k < B; ++k) {
      a[c][k] *= ip;
      G[c][k] *= ip;
    }
    SPG_UNROLL for (int r = 0; r < B; ++r) {
      if (r == c) continue;
      const double f = a[r][c];
      SPG_UNROLL for (int k = 0; k < B; ++k) {
        a[r][k] = fma(-f, a[c][k], a[r][k]);
        G[r][k] = fma(-f, G[c][k], G[r][k]);
      }
    }
  }
  // |det| = product of the pivots; for b <= 16 and M = I + Q J it stays far from overflow
  return log(fabs(pivprod));
}

// a b - c d with one rounding error on each product folded back (Kahan's 2x2 determinant):
// accurate to a few ulps of the result even when the two products nearly cancel.
SPG_DEV double diff_of_products(double a, double b, double c, double d) {
  const double w = c * d;
  const double e = fma(-c, d, w);
  const double f = fma(a, b, -w);
  return f + e;
}

template <>
SPG_DEV double inv_logdet<1>(const double (&M)[1][1], double (&G)[1][1]) {
  G[0][0] = 1.0 / M[0][0];
  return log(fabs(M[0][0]));
}

// b = 2 and b = 3: the inverse through the adjugate, one division and a short dependency
// chain (the pivoted elimination above needs one division per column in sequence).
template <>
SPG_DEV double inv_logdet<2>(const double (&M)[2][2], double (&G)[2][2]) {
  const double det = diff_of_products(M[0][0], M[1][1], M[0][1], M[1][0]);
  const double id = 1.0 / det;
  G[0][0] = M[1][1] * id;
  G[0][1] = -M[0][1] * id;
  G[1][0] = -M[1][0] * id;
  G[1][1] = M[0][0] * id;
  return log(fabs(det));
}
template <>
SPG_DEV double inv_logdet<3>(const double (&M)[3][3], double (&G)[3][3]) {
  // cofactor C[i][j]; the inverse is C^T / det
  const double c00 = diff_of_products(M[1][1], M[2][2], M[1][2], M[2][1]);
  const double c01 = diff_of_products(M[1][2], M[2][0], M[1][0], M[2][2]);
  const double c02 = diff_of_products(M[1][0], M[2][1], M[1][1], M[2][0]);
  const double c10 = diff_of_products(M[0][2], M[2][1], M[0][1], M[2][2]);
  const double c11 = diff_of_products(M[0][0], M[2][2], M[0][2], M[2][0]);
  const double c12 = diff_of_products(M[0][1], M[2][0], M[0][0], M[2][1]);
  const double c20 = diff_of_products(M[0][1], M[1][2], M[0][2], M[1][1]);
  const double c21 = diff_of_products(M[0][2], M[1][0], M[0][0], M[1][2]);
  const double c22 = diff_of_products(M[0][0], M[1][1], M[0][1], M[1][0]);
  const double det = fma(M[0][0], c00, fma(M[0][1], c01, M[0][2] * c02));
  const double id = 1.0 / det;
  G[0][0] = c00 * id;
  G[0][1] = c10 * id;
  G[0][2] = c20 * id;
  G[1][0] = c01 * id;
  G[1][1] = c11 * id;
  G[1][2] = c21 * id;
  G[2][0] = c02 * id;
  G[2][1] = c12 * id;
  G[2][2] = c22 * id;
  return log(fabs(det));
}

// ------------------------------------------------------------------ state-space models
// Per-series constants.  Matern-nu (nu = 3/2 -> b = 2, nu = 5/2 -> b = 3), observation
// vector h = e_0.  With lam = sqrt(2 nu) / l and x = lam dt, the transition
// A[dt] = expm(F dt) = e^-x (I + dt N + dt^2/2 N^2), N = F + lam I nilpotent, is written out
// entry by entry, together with its lam-derivative.  P0 holds k(0), -k''(0), k''''(0).
struct SeriesPar {
  double lam;     // sqrt(2 nu) / lengthscale
  double var;     // signal variance
  double s2;      // noise variance
  double ell;     // lengthscale
};

template <int B>
struct Matern;

// Matern-1/2 (b = 1, lam = 1 / l): the Ornstein-Uhlenbeck state, A = e^{-lam dt}.
template <>
struct Matern<1> {
  static constexpr int B = 1;
  SPG_DEV static void pinf(const SeriesPar& p, double (&P)[1][1]) { P[0][0] = p.var; }
  SPG_DEV static void dpinf_dlam(const SeriesPar&, double (&P)[1][1]) { P[0][0] = 0.0; }
  SPG_DEV static void transition(const SeriesPar& p, double dt, double& e, double (&A)[1][1]) {
    e = exp(-p.lam * dt);
    A[0][0] = e;
  }
  SPG_DEV static void transition_e(const SeriesPar&, double, double e, double (&A)[1][1]) { A[0][0] = e; }
  SPG_DEV static double dA_dlam_dot(const SeriesPar&, double dt, double e, const double (&Ab)[1][1]) {
    return -dt * e * Ab[0][0];
  }
};

template <>
struct Matern<2> {
  static constexpr int B = 2;
  SPG_DEV static void pinf(const SeriesPar& p, double (&P)[2][2]) {
    P[0][0] = p.var;
    P[0][1] = P[1][0] = 0.0;
    P[1][1] = p.var * p.lam * p.lam;
  }
  SPG_DEV static void dpinf_dlam(const SeriesPar& p, double (&P)[2][2]) {
    P[0][0] = 0.0;
    P[0][1] = P[1][0] = 0.0;
    P[1][1] = 2.0 * p.var * p.lam;
  }
  SPG_DEV static void transition(const SeriesPar& p, double dt, double& e, double (&A)[2][2]) {
    e = exp(-p.lam * dt);
    transition_e(p, dt, e, A);
  }
  SPG_DEV static void transition_e(const SeriesPar& p, double dt, double e, double (&A)[2][2]) {
    const double x = p.lam * dt;
    A[0][0] = e * (1.0 + x);
    A[0][1] = e * dt;
    A[1][0] = -e * p.lam * x;
    A[1][1] = e * (1.0 - x);
  }
  // <Abar, dA/dlam>
  SPG_DEV static double dA_dlam_dot(const SeriesPar& p, double dt, double e, const double (&Ab)[2][2]) {
    const double x = p.lam * dt;
    const double d00 = -dt * x, d01 = -dt * dt, d10 = x * (x - 2.0), d11 = dt * (x - 2.0);
    return e * (Ab[0][0] * d00 + Ab[0][1] * d01 + Ab[1][0] * d10 + Ab[1][1] * d11);
  }
};

template <>
struct Matern<3> {
  static constexpr int B = 3;
  SPG_DEV static void pinf(const SeriesPar& p, double (&P)[3][3]) {
    const double l2 = p.lam * p.lam, v = p.var;
    P[0][0] = v;
    P[0][1] = P[1][0] = 0.0;
    P[0][2] = P[2][0] = -v * l2 * (1.0 / 3.0);
    P[1][1] = v * l2 * (1.0 / 3.0);
    P[1][2] = P[2][1] = 0.0;
    P[2][2] = v * l2 * l2;
  }
  SPG_DEV static void dpinf_dlam(const SeriesPar& p, double (&P)[3][3]) {
    const double l = p.lam, v = p.var;
    P[0][0] = 0.0;
    P[0][1] = P[1][0] = 0.0;
    P[0][2] = P[2][0] = -v * l * (2.0 / 3.0);
    P[1][1] = v * l * (2.0 / 3.0);
    P[1][2] = P[2][1] = 0.0;
    P[2][2] = 4.0 * v * l * l * l;
  }
  SPG_DEV static void transition(const SeriesPar& p, double dt, double& e, double (&A)[3][3]) {
    e = exp(-p.lam * dt);
    transition_e(p, dt, e, A);
  }
  SPG_DEV static void transition_e(const SeriesPar& p, double dt, double e, double (&A)[3][3]) {
    const double l = p.lam, x = l * dt, x2 = x * x;
    A[0][0] = e * (1.0 + x + 0.5 * x2);
    A[0][1] = e * dt * (1.0 + x);
    A[0][2] = e * 0.5 * dt * dt;
    A[1][0] = -e * 0.5 * l * x2;
    A[1][1] = e * (1.0 + x - x2);
    A[1][2] = e * dt * (1.0 - 0.5 * x);
    A[2][0] = e * l * l * (0.5 * x2 - x);
    A[2][1] = e * l * (x2 - 3.0 * x);
    A[2][2] = e * (1.0 - 2.0 * x + 0.5 * x2);
  }
  SPG_DEV static double dA_dlam_dot(const SeriesPar& p, double dt, double e, const double (&Ab)[3][3]) {
    const double l = p.lam, x = l * dt, x2 = x * x;
    double s = Ab[0][0] * (-0.5 * dt * x2);
    s = fma(Ab[0][1], -dt * dt * x, s);
    s = fma(Ab[0][2], -0.5 * dt * dt * dt, s);
    s = fma(Ab[1][0], -0.5 * x2 * (3.0 - x), s);
    s = fma(Ab[1][1], dt * x * (x - 3.0), s);
    s = fma(Ab[1][2], 0.5 * dt * dt * (x - 3.0), s);
    s = fma(Ab[2][0], l * x * (3.0 * x - 0.5 * x2 - 3.0), s);
    s = fma(Ab[2][1], x * (6.0 * x - x2 - 6.0), s);
    s = fma(Ab[2][2], dt * (-3.0 + 3.0 * x - 0.5 * x2), s);
    return e * s;
  }
};

// Matern-7/2 (b = 4, lam = sqrt(7) / l): the state holds f and its first three derivatives, F
// is the companion matrix of (s + lam)^4.  N = F + lam I is nilpotent (N^4 = 0), so
// A = e^{-lam dt} (I + N dt + N^2 dt^2 / 2 + N^3 dt^3 / 6); the entries below are that sum
// multiplied out in x = lam dt.  P0 holds the derivatives of k at 0: entry (i, j) is
// (-1)^j k^(i+j)(0), with k''(0) = -var lam^2 / 5, k''''(0) = var lam^4 / 5,
// k^(6)(0) = -var lam^6.
template <>
struct Matern<4> {
  static constexpr int B = 4;
  SPG_DEV static void pinf(const SeriesPar& p, double (&P)[4][4]) {
    const double v = p.var, l2 = p.lam * p.lam, l4 = l2 * l2;
    SPG_UNROLL for (int i = 0; i < 4; ++i) SPG_UNROLL for (int j = 0; j < 4; ++j) P[i][j] = 0.0;
    P[0][0] = v;
    P[0][2] = P[2][0] = -v * l2 * 0.2;
    P[1][1] = v * l2 * 0.2;
    P[1][3] = P[3][1] = -v * l4 * 0.2;
    P[2][2] = v * l4 * 0.2;
    P[3][3] = v * l4 * l2;
  }
  SPG_DEV static void dpinf_dlam(const SeriesPar& p, double (&P)[4][4]) {
    const double v = p.var, l = p.lam, l3 = l * l * l;
    SPG_UNROLL for (int i = 0; i < 4; ++i) SPG_UNROLL for (int j = 0; j < 4; ++j) P[i][j] = 0.0;
    P[0][2] = P[2][0] = -v * l * 0.4;
    P[1][1] = v * l * 0.4;
    P[1][3] = P[3][1] = -v * l3 * 0.8;
    P[2][2] = v * l3 * 0.8;
    P[3][3] = 6.0 * v * l3 * l * l;
  }
  SPG_DEV static void transition(const SeriesPar& p, double dt, double& e, double (&A)[4][4]) {
    e = exp(-p.lam * dt);
    transition_e(p, dt, e, A);
  }
  SPG_DEV static void transition_e(const SeriesPar& p, double dt, double e, double (&A)[4][4]) {
    const double l = p.lam, x = l * dt, x2 = x * x, x3 = x2 * x, l2 = l * l;
    const double c6 = e * (1.0 / 6.0), c2 = 0.5 * e;
    A[0][0] = c6 * (x3 + 3.0 * x2 + 6.0 * x + 6.0);
    A[0][1] = c2 * dt * (x2 + 2.0 * x + 2.0);
    A[0][2] = c2 * dt * dt * (x + 1.0);
    A[0][3] = c6 * dt * dt * dt;
    A[1][0] = -c6 * l * x3;
    A[1][1] = -c2 * (x3 - x2 - 2.0 * x - 2.0);
    A[1][2] = -c2 * dt * (x2 - 2.0 * x - 2.0);
    A[1][3] = -c6 * dt * dt * (x - 3.0);
    A[2][0] = c6 * l2 * x2 * (x - 3.0);
    A[2][1] = c2 * l * x2 * (x - 4.0);
    A[2][2] = c2 * (x - 1.0) * (x2 - 4.0 * x - 2.0);
    A[2][3] = c6 * dt * (x2 - 6.0 * x + 6.0);
    A[3][0] = -c6 * l2 * l * x * (x2 - 6.0 * x + 6.0);
    A[3][1] = -c2 * l2 * x * (x2 - 7.0 * x + 8.0);
    A[3][2] = -c2 * l * x * (x - 6.0) * (x - 2.0);
    A[3][3] = -c6 * (x3 - 9.0 * x2 + 18.0 * x - 6.0);
  }
  // <Abar, dA/dlam> at fixed dt
  SPG_DEV static double dA_dlam_dot(const SeriesPar& p, double dt, double e, const double (&Ab)[4][4]) {
    const double l = p.lam, x = l * dt, x2 = x * x, x3 = x2 * x;
    const double u = x - 4.0, w = (x - 6.0) * (x - 2.0), z = x3 - 12.0 * x2 + 36.0 * x - 24.0;
    double s = Ab[0][0] * (-dt * x3 * (1.0 / 6.0));
    s = fma(Ab[0][1], -0.5 * dt * dt * x2, s);
    s = fma(Ab[0][2], -0.5 * dt * dt * dt * x, s);
    s = fma(Ab[0][3], -dt * dt * dt * dt * (1.0 / 6.0), s);
    s = fma(Ab[1][0], x3 * u * (1.0 / 6.0), s);
    s = fma(Ab[1][1], 0.5 * dt * x2 * u, s);
    s = fma(Ab[1][2], 0.5 * dt * dt * x * u, s);
    s = fma(Ab[1][3], dt * dt * dt * u * (1.0 / 6.0), s);
    s = fma(Ab[2][0], -l * x2 * w * (1.0 / 6.0), s);
    s = fma(Ab[2][1], -0.5 * x2 * w, s);
    s = fma(Ab[2][2], -0.5 * dt * x * w, s);
    s = fma(Ab[2][3], -dt * dt * w * (1.0 / 6.0), s);
    s = fma(Ab[3][0], l * l * x * z * (1.0 / 6.0), s);
    s = fma(Ab[3][1], 0.5 * l * x * z, s);
    s = fma(Ab[3][2], 0.5 * x * z, s);
    s = fma(Ab[3][3], dt * z * (1.0 / 6.0), s);
    return e * s;
  }
};

// ------------------------------------------------------------------ chain elements
template <int B>
struct Elem {
  double A[B][B];
  double b[B];
  double Q[B][B];
  double J[B][B];
  double eta[B];
  double cf;   // quadratic-in-y part of the log normaliser
  double cl;   // log-determinant part of the log normaliser (includes -1/2 log 2 pi terms)
};

template <int B>
SPG_DEV void elem_identity(Elem<B>& E) {
  mat_eye<B>(E.A);
  mat_zero<B>(E.Q);
  mat_zero<B>(E.J);
  SPG_UNROLL for (int i = 0; i < B; ++i) {
    E.b[i] = 0.0;
    E.eta[i] = 0.0;
  }
  E.cf = 0.0;
  E.cl = 0.0;
}

// General combine E1 (x) E2 (tree levels of the cyclic reduction).
template <int B>
SPG_DEV void elem_combine(const Elem<B>& E1, const Elem<B>& E2, Elem<B>& R) {
  double M[B][B], G[B][B];
  mm<B>(E1.Q, E2.J, M);
  SPG_UNROLL for (int i = 0; i < B; ++i) M[i][i] += 1.0;
  const double ld = inv_logdet<B>(M, G);
  double Pp[B][B], W[B][B], GA[B][B];
  mm<B>(G, E1.Q, Pp);
  symmetrize<B>(Pp);
  mm<B>(E2.J, G, W);
  symmetrize<B>(W);
  mm<B>(G, E1.A, GA);
  double Gb[B], Ppe[B], g[B], Gte[B], Wb[B], r[B];
  mv<B>(G, E1.b, Gb);
  mv<B>(Pp, E2.eta, Ppe);
  mtv<B>(G, E2.eta, Gte);
  mv<B>(W, E1.b, Wb);
  SPG_UNROLL for (int i = 0; i < B; ++i) {
    g[i] = Gb[i] + Ppe[i];
    r[i] = Gte[i] - Wb[i];
  }
  const double cf = -0.5 * dot<B>(E1.b, Wb) + dot<B>(E2.eta, Gb) + 0.5 * dot<B>(E2.eta, Ppe);
  // new edge
  double T[B][B];
  mm<B>(E2.A, GA, R.A);
  double Ag[B];
  mv<B>(E2.A, g, Ag);
  mm<B>(E2.A, Pp, T);
  mmt_sym<B>(T, E2.A, R.Q);
  SPG_UNROLL for (int i = 0; i < B; ++i) {
    R.b[i] = Ag[i] + E2.b[i];
    SPG_UNROLL for (int j = 0; j < B; ++j) R.Q[i][j] += E2.Q[i][j];
  }
  // information pushed back to the left node
  double WA[B][B], AWA[B][B], Ar[B];
  mm<B>(W, E1.A, WA);
  mtm_sym<B>(E1.A, WA, AWA);
  mtv<B>(E1.A, r, Ar);
  SPG_UNROLL for (int i = 0; i < B; ++i) {
    R.eta[i] = E1.eta[i] + Ar[i];
    SPG_UNROLL for (int j = 0; j < B; ++j) R.J[i][j] = E1.J[i][j] + AWA[i][j];
  }
  R.cf = E1.cf + E2.cf + cf;
  R.cl = E1.cl + E2.cl - 0.5 * ld;
}

// The two halves of E1 (x) E2, for two lanes on different wavefronts (a tree level then takes
// about half the issue time of one lane doing the whole join).  Both form Gam = (I + Q1 J2)^-1;
// the forward half sets the new edge (A, b, Q) of R, the backward half the information pushed
// back to the left node (J, eta) and the normaliser (cf, cl).  Same arithmetic, in the same
// order, as elem_combine.
template <int B>
SPG_DEV void elem_combine_fwd(const Elem<B>& E1, const Elem<B>& E2, Elem<B>& R) {
  double M[B][B], G[B][B];
  mm<B>(E1.Q, E2.J, M);
  SPG_UNROLL for (int i = 0; i < B; ++i) M[i][i] += 1.0;
  (void)inv_logdet<B>(M, G);
  double Pp[B][B], GA[B][B];
  mm<B>(G, E1.Q, Pp);
  symmetrize<B>(Pp);
  mm<B>(G, E1.A, GA);
  double Gb[B], Ppe[B], g[B];
  mv<B>(G, E1.b, Gb);
  mv<B>(Pp, E2.eta, Ppe);
  SPG_UNROLL for (int i = 0; i < B; ++i) g[i] = Gb[i] + Ppe[i];
  double T[B][B], Ag[B];
  mm<B>(E2.A, GA, R.A);
  mv<B>(E2.A, g, Ag);
  mm<B>(E2.A, Pp, T);
  mmt_sym<B>(T, E2.A, R.Q);
  SPG_UNROLL for (int i = 0; i < B; ++i) {
    R.b[i] = Ag[i] + E2.b[i];
    SPG_UNROLL for (int j = 0; j < B; ++j) R.Q[i][j] += E2.Q[i][j];
  }
}
template <int B>
SPG_DEV void elem_combine_bwd(const Elem<B>& E1, const Elem<B>& E2, Elem<B>& R) {
  double M[B][B], G[B][B];
  mm<B>(E1.Q, E2.J, M);
  SPG_UNROLL for (int i = 0; i < B; ++i) M[i][i] += 1.0;
  const double ld = inv_logdet<B>(M, G);
  double Pp[B][B], W[B][B];
  mm<B>(G, E1.Q, Pp);
  symmetrize<B>(Pp);
  mm<B>(E2.J, G, W);
  symmetrize<B>(W);
  double Gb[B], Ppe[B], Gte[B], Wb[B], r[B];
  mv<B>(G, E1.b, Gb);
  mv<B>(Pp, E2.eta, Ppe);
  mtv<B>(G, E2.eta, Gte);
  mv<B>(W, E1.b, Wb);
  SPG_UNROLL for (int i = 0; i < B; ++i) r[i] = Gte[i] - Wb[i];
  const double cf = -0.5 * dot<B>(E1.b, Wb) + dot<B>(E2.eta, Gb) + 0.5 * dot<B>(E2.eta, Ppe);
  double WA[B][B], AWA[B][B], Ar[B];
  mm<B>(W, E1.A, WA);
  mtm_sym<B>(E1.A, WA, AWA);
  mtv<B>(E1.A, r, Ar);
  SPG_UNROLL for (int i = 0; i < B; ++i) {
    R.eta[i] = E1.eta[i] + Ar[i];
    SPG_UNROLL for (int j = 0; j < B; ++j) R.J[i][j] = E1.J[i][j] + AWA[i][j];
  }
  R.cf = E1.cf + E2.cf + cf;
  R.cl = E1.cl + E2.cl - 0.5 * ld;
}

// Prefix combine: (m, P) = predicted state N(z; m, P) at the left node of E, pushed through E.
// Returns the increment of the log normaliser (fit and log-det parts).
template <int B>
SPG_DEV void prefix_combine(const double (&m)[B], const double (&P)[B][B], const Elem<B>& E,
                            double (&mo)[B], double (&Po)[B][B], double& dcf, double& dcl) {
  double M[B][B], G[B][B];
  mm<B>(P, E.J, M);
  SPG_UNROLL for (int i = 0; i < B; ++i) M[i][i] += 1.0;
  const double ld = inv_logdet<B>(M, G);
  double Pp[B][B], W[B][B];
  mm<B>(G, P, Pp);
  symmetrize<B>(Pp);
  mm<B>(E.J, G, W);
  symmetrize<B>(W);
  double Gm[B], Ppe[B], g[B], Wm[B];
  mv<B>(G, m, Gm);
  mv<B>(Pp, E.eta, Ppe);
  mv<B>(W, m, Wm);
  SPG_UNROLL for (int i = 0; i < B; ++i) g[i] = Gm[i] + Ppe[i];
  dcf = -0.5 * dot<B>(m, Wm) + dot<B>(E.eta, Gm) + 0.5 * dot<B>(E.eta, Ppe) + E.cf;
  dcl = -0.5 * ld + E.cl;
  double Ag[B], T[B][B];
  mv<B>(E.A, g, Ag);
  mm<B>(E.A, Pp, T);
  mmt_sym<B>(T, E.A, Po);
  SPG_UNROLL for (int i = 0; i < B; ++i) {
    mo[i] = Ag[i] + E.b[i];
    SPG_UNROLL for (int j = 0; j < B; ++j) Po[i][j] += E.Q[i][j];
  }
}

// Suffix combine: information (Jb, etab) on the right node of E, pulled back to E's left node.
template <int B>
SPG_DEV void suffix_combine(const Elem<B>& E, const double (&Jb)[B][B], const double (&etab)[B],
                            double (&Jo)[B][B], double (&etao)[B]) {
  double M[B][B], G[B][B];
  mm<B>(E.Q, Jb, M);
  SPG_UNROLL for (int i = 0; i < B; ++i) M[i][i] += 1.0;
  (void)inv_logdet<B>(M, G);
  double W[B][B];
  mm<B>(Jb, G, W);
  symmetrize<B>(W);
  double Gte[B], Wb[B], r[B];
  mtv<B>(G, etab, Gte);
  mv<B>(W, E.b, Wb);
  SPG_UNROLL for (int i = 0; i < B; ++i) r[i] = Gte[i] - Wb[i];
  double WA[B][B], AWA[B][B], Ar[B];
  mm<B>(W, E.A, WA);
  mtm_sym<B>(E.A, WA, AWA);
  mtv<B>(E.A, r, Ar);
  SPG_UNROLL for (int i = 0; i < B; ++i) {
    etao[i] = E.eta[i] + Ar[i];
    SPG_UNROLL for (int j = 0; j < B; ++j) Jo[i][j] = E.J[i][j] + AWA[i][j];
  }
}

// ------------------------------------------------------------------ element storage (SoA)
// Field layout of one element: A (B*B), b (B), Q upper (B(B+1)/2), J upper, eta (B), cf, cl.
template <int B>
struct ElemLayout {
  static constexpr int kSym = B * (B + 1) / 2;
  static constexpr int kA = 0;
  static constexpr int kb = B * B;
  static constexpr int kQ = kb + B;
  static constexpr int kJ = kQ + kSym;
  static constexpr int keta = kJ + kSym;
  static constexpr int kcf = keta + B;
  static constexpr int kcl = kcf + 1;
  static constexpr int kFields = kcl + 1;
};

template <int B>
SPG_DEV void elem_store(double* base, int64_t ld, int64_t i, const Elem<B>& E) {
  using L = ElemLayout<B>;
  SPG_UNROLL for (int r = 0; r < B; ++r) SPG_UNROLL for (int c = 0; c < B; ++c)
    base[(L::kA + r * B + c) * ld + i] = E.A[r][c];
  SPG_UNROLL for (int r = 0; r < B; ++r) {
    base[(L::kb + r) * ld + i] = E.b[r];
    base[(L::keta + r) * ld + i] = E.eta[r];
  }
  int s = 0;
  SPG_UNROLL for (int r = 0; r < B; ++r) SPG_UNROLL for (int c = r; c < B; ++c) {
    base[(L::kQ + s) * ld + i] = E.Q[r][c];
    base[(L::kJ + s) * ld + i] = E.J[r][c];
    ++s;
  }
  base[L::kcf * ld + i] = E.cf;
  base[L::kcl * ld + i] = E.cl;
}

// The fields each half of a split join produces: forward (A, b, Q), backward (J, eta, cf, cl).
template <int B>
SPG_DEV void elem_store_half(double* base, int64_t ld, int64_t i, const Elem<B>& E, bool fwd) {
  using L = ElemLayout<B>;
  if (fwd) {
    SPG_UNROLL for (int r = 0; r < B; ++r) SPG_UNROLL for (int c = 0; c < B; ++c)
      base[(L::kA + r * B + c) * ld + i] = E.A[r][c];
    SPG_UNROLL for (int r = 0; r < B; ++r) base[(L::kb + r) * ld + i] = E.b[r];
    int s = 0;
    SPG_UNROLL for (int r = 0; r < B; ++r) SPG_UNROLL for (int c = r; c < B; ++c) base[(L::kQ + s++) * ld + i] = E.Q[r][c];
  } else {
    SPG_UNROLL for (int r = 0; r < B; ++r) base[(L::keta + r) * ld + i] = E.eta[r];
    int s = 0;
    SPG_UNROLL for (int r = 0; r < B; ++r) SPG_UNROLL for (int c = r; c < B; ++c) base[(L::kJ + s++) * ld + i] = E.J[r][c];
    base[L::kcf * ld + i] = E.cf;
    base[L::kcl * ld + i] = E.cl;
  }
}

template <int B>
SPG_DEV void elem_load(const double* base, int64_t ld, int64_t i, Elem<B>& E) {
  using L = ElemLayout<B>;
  SPG_UNROLL for (int r = 0; r < B; ++r) SPG_UNROLL for (int c = 0; c < B; ++c)
    E.A[r][c] = base[(L::kA + r * B + c) * ld + i];
  SPG_UNROLL for (int r = 0; r < B; ++r) {
    E.b[r] = base[(L::kb + r) * ld + i];
    E.eta[r] = base[(L::keta + r) * ld + i];
  }
  int s = 0;
  SPG_UNROLL for (int r = 0; r < B; ++r) SPG_UNROLL for (int c = r; c < B; ++c) {
    const double q = base[(L::kQ + s) * ld + i];
    const double j = base[(L::kJ + s) * ld + i];
    E.Q[r][c] = q;
    E.Q[c][r] = q;
    E.J[r][c] = j;
    E.J[c][r] = j;
    ++s;
  }
  E.cf = base[L::kcf * ld + i];
  E.cl = base[L::kcl * ld + i];
}

}  // namespace spg
