// Wide-state path for one series: a sum of covariance terms (Matern-1/2 .. 7/2, periodic and
// quasi-periodic with any number of harmonics, squared exponential by its spectral
// approximation of even order up to 10), state dimension b up to 16, in state-space form
// (Sec. 2.1); the model is described at run time (spingp_sumdesc.hpp), the kernels are
// compiled once per b.  The paper's kernels are such sums: Matern-3/2 + 10th-order squared
// exponential (b = 12, Sec. 4.2), the CO2 kernel (Sec. 4.3).
//
// The per-lane kernels keep a whole chain element in registers; at b = 10 an element has 322
// doubles, so here one wavefront (a "team" of 64 lanes, one work-group) works on one element
// operation at a time with its b x b blocks staged in LDS, its products on the matrix cores.
// The cyclic reduction runs level by level over all N nodes (one node per leaf), one launch
// per level:
//   up-sweep   level k element i = E(k-1, 2i) (x) E(k-1, 2i+1)      (odd-even reduction)
//   down-sweep messages of level k-1 from those of level k: the predicted state (m, P)
//              entering an element's left node (prefix) and the information (J, eta) that
//              all later data put on its right node (suffix)
//   node step  with the exact predicted state at node n and the exact information on node
//              n+1, the filtered state, the smoothed moments and the derivatives of the log
//              marginal likelihood with respect to the edge n -> n+1 are all local:
//                lam = Gam^T eta' - W m',  Lam = 1/2 (lam lam^T - W)   (dL/dm', dL/dP')
//                mu = m+ + P+ A^T lam,  S = P+ - P+ A^T W A P+,  S_sub = (I - P' W) A P+
//                A_bar = lam m+^T + 2 Lam A (P+ - P0),  P0_bar += Lam - A^T Lam A
//              and the noise variance by the posterior expectation of d log N(y; h z, s2).
//
// State basis.  The model's natural state is block diagonal (one block per term) with an
// observation vector h of ones and zeros.  The kernels run in the basis z' = T z with T = I
// except row 0 = h^T (state 0, the first state of the first term, is always observed), where
// the observation is e_0 (so the node information is rank one in entry (0, 0)); A' = T A T^-1,
// Q' = T Q T^T, P0' = T P0 T^T.  State outputs are mapped back with T^-1, gradients with
// T^T (.) T^-T.
#pragma once
#include "spingp_device.hpp"
#include "spingp_sqexp_tables.hpp"
#include "spingp_sumdesc.hpp"

namespace spg {
namespace wide {

constexpr int kW = 64;  // lanes per team (one wavefront, one work-group)
static_assert(kSqExpMaxOrder == kMaxSqExpOrder, "generated tables cover every supported order");

// A team is one wavefront (every team kernel is launched with kW threads), whose LDS operations
// execute in issue order: a wavefront-scope fence (no wait instruction) orders the LDS writes
// of one phase before the reads of the next, and the wave barrier keeps the compiler from
// moving them across it.
static_assert(kW == 64, "a team is one wave64");
SPG_DEV void tsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// ---------------------------------------------------------------------------- layouts
template <int B>
struct Lay {
  static constexpr int BB = B * B;
  // element (item-major in global memory, same order in LDS): A, b, Q, J, eta, cf, cl
  static constexpr int kA = 0, kb = BB, kQ = BB + B, kJ = 2 * BB + B, keta = 3 * BB + B;
  static constexpr int kcf = 3 * BB + 2 * B, kcl = kcf + 1;
  static constexpr int kE = kcl + 1;
  static constexpr int kEs = (kE + 7) / 8 * 8;        // item stride (64-byte multiple)
  // message: m, P (prefix) and J, eta (suffix)
  static constexpr int km = 0, kP = B, kMJ = B + BB, kMeta = 2 * BB + B;
  static constexpr int kM = 2 * BB + 2 * B;
  static constexpr int kMs = (kM + 7) / 8 * 8;
  // scratch of one element operation: a join takes 3 matrices and 6 vectors (and reuses the
  // blocks of its operands that it has consumed), a prefix or suffix step 3 matrices and 5
  // vectors; kTmp covers any of them
  static constexpr int kTmp = 8 * BB + 10 * B;
  static constexpr int kTmpJoin = 3 * BB + 6 * B;
  static constexpr int kTmpStep = 3 * BB + 5 * B;
};

// ---------------------------------------------------------------------------- team algebra
// Row-major B x B matrices in LDS.  Outputs never alias inputs.  Every call ends with a
// barrier, so its result is visible to the whole team.
//
// Matrix products run on the matrix cores: op(X) op(Y) for B <= 16 is one 16 x 16 tile, built
// from 16 x 16 x 4 FP64 MFMA steps over k (operands zero past B).  In each step lane l supplies
// op(X)[l % 16][k] and op(Y)[k][l % 16] for k = 4 s + l / 16, and the 16 x 16 result ends with
// entry (l / 16 + 4 r, l % 16) in component r of lane l.  The whole wavefront takes part, so
// products are only formed in uniform control flow.
typedef double v4d __attribute__((ext_vector_type(4)));

template <int B, bool TX, bool TY>
SPG_DEV v4d mx(const double* X, const double* Y) {
  static_assert(B <= 16, "one 16 x 16 tile");
  const int l = threadIdx.x, i = l & 15, kq = l >> 4;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  SPG_UNROLL for (int s = 0; s < (B + 3) / 4; ++s) {
    const int k = 4 * s + kq;
    const bool in = i < B && k < B;
    // every lane loads (a clamped, valid index), then the padding is zeroed
    const int ix = in ? (TX ? k * B + i : i * B + k) : 0;
    const int iy = in ? (TY ? i * B + k : k * B + i) : 0;
    const double xv = X[ix], yv = Y[iy];
    const double a = in ? xv : 0.0;
    const double b = in ? yv : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  return acc;
}
// The symmetric part (Z + Z^T) / 2 of Z = op(X) op(Y): Z^T = op(Y)^T op(X)^T is a second tile.
template <int B, bool TX, bool TY>
SPG_DEV v4d mx_sym(const double* X, const double* Y) {
  return 0.5 * (mx<B, TX, TY>(X, Y) + mx<B, !TY, !TX>(Y, X));
}
// f(i, j, value) for the entries of the lane's results inside the B x B block.
template <int B, class F>
SPG_DEV void mx_each(const v4d& d, F&& f) {
  const int l = threadIdx.x, j = l & 15, i0 = l >> 4;
  if (j < B) {
    SPG_UNROLL for (int r = 0; r < 4; ++r) {
      const int i = i0 + 4 * r;
      if (i < B) f(i, j, d[r]);
    }
  }
}
template <int B>
SPG_DEV void mx_store(const v4d& d, double* Z) {
  mx_each<B>(d, [&](int i, int j, double v) { Z[i * B + j] = v; });
}
template <int B>
SPG_DEV void t_copy(const double* __restrict__ X, double* __restrict__ Y, int n) {
  for (int e = threadIdx.x; e < n; e += kW) Y[e] = X[e];
  tsync();
}
template <int B>
SPG_DEV void t_mm(const double* X, const double* Y, double* Z) {        // Z = X Y
  mx_store<B>(mx<B, false, false>(X, Y), Z);
  tsync();
}
template <int B>
SPG_DEV void t_mtm(const double* X, const double* Y, double* Z) {       // Z = X^T Y
  mx_store<B>(mx<B, true, false>(X, Y), Z);
  tsync();
}
template <int B>
SPG_DEV void t_mtv(const double* X, const double* v, double* w) {       // w = X^T v
  if (threadIdx.x < B) {
    const int i = threadIdx.x;
    double s = 0.0;
    SPG_UNROLL for (int k = 0; k < B; ++k) s = fma(X[k * B + i], v[k], s);
    w[i] = s;
  }
  tsync();
}
template <int B>
SPG_DEV void t_sym(double* X) {                                          // X = (X + X^T) / 2
  for (int e = threadIdx.x; e < B * B; e += kW) {
    const int i = e / B, j = e - i * B;
    if (i < j) {
      const double a = 0.5 * (X[i * B + j] + X[j * B + i]);
      X[i * B + j] = a;
      X[j * B + i] = a;
    }
  }
  tsync();
}
template <int B>
SPG_DEV void t_add_eye(double* X) {
  if (threadIdx.x < B) X[threadIdx.x * (B + 1)] += 1.0;
  tsync();
}
// Every lane returns the same value (broadcast reads, fixed order).
template <int B>
SPG_DEV double t_dot(const double* a, const double* b) {
  double s = 0.0;
  SPG_UNROLL for (int k = 0; k < B; ++k) s = fma(a[k], b[k], s);
  return s;
}

// Value of x in lane C of the caller's row of 16 lanes, for every lane of that row (DPP
// row_newbcast, one 64-bit move; the lane index must be a constant, so callers pass an
// unrolled loop index).  Every lane of every row is written, so no old value is needed.
template <int C>
SPG_DEV double row_bcast_c(double x) {
  return __builtin_amdgcn_mov_dpp(x, 0x150 + C, 0xF, 0xF, false);
}
SPG_DEV double row_bcast(double x, int c) {
  switch (c) {
    case 0: return row_bcast_c<0>(x);
    case 1: return row_bcast_c<1>(x);
    case 2: return row_bcast_c<2>(x);
    case 3: return row_bcast_c<3>(x);
    case 4: return row_bcast_c<4>(x);
    case 5: return row_bcast_c<5>(x);
    case 6: return row_bcast_c<6>(x);
    case 7: return row_bcast_c<7>(x);
    case 8: return row_bcast_c<8>(x);
    case 9: return row_bcast_c<9>(x);
    case 10: return row_bcast_c<10>(x);
    case 11: return row_bcast_c<11>(x);
    case 12: return row_bcast_c<12>(x);
    case 13: return row_bcast_c<13>(x);
    case 14: return row_bcast_c<14>(x);
    default: return row_bcast_c<15>(x);
  }
}

// G = M^-1 by Gauss-Jordan with partial pivoting over columns; returns log |det M| (the same in
// every lane).  Lane r < B of every row of 16 lanes keeps row r of [M | G] in registers (lanes
// past B shadow row B - 1 and write nothing).  At step c the pivot is the largest entry of row c
// (a search inside lane c), every lane swaps the two columns in its own row, and the pivot row
// reaches the other lanes by DPP broadcasts from the fixed lane c: no cross-lane traffic
// depends on the pivot.  Pivot rows stay unscaled until the end (each later update is linear
// in the row, so the scale carries through).  M P = E^-1 for the column permutation P, so
// M^-1 = P E: the rows are written to their permuted places.  G may be M: every row is read
// into registers before the first is written (one wavefront, in program order).
template <int B>
SPG_DEV double t_inv_logdet(const double* M, double* G, double* /*unused*/ = nullptr) {
  static_assert(B <= 16, "one row of 16 lanes holds the matrix");
  const int tid = threadIdx.x;
  const int lr = tid & 15;
  const int r = lr < B ? lr : B - 1;
  double a[B], g[B];
  SPG_UNROLL for (int k = 0; k < B; ++k) {
    a[k] = M[r * B + k];
    g[k] = (r == k) ? 1.0 : 0.0;
  }
  int qs[B];
  double mant = 1.0;   // product of the pivots as mantissa and binary exponent: one log at the end
  int expo = 0;
  double own_piv = 1.0;
  SPG_UNROLL for (int c = 0; c < B; ++c) {
    // pivot column: the first k >= c with the largest |a[k]| in row c, found by lane c
    int q = c;
    double best = fabs(a[c]);
    SPG_UNROLL for (int k = c + 1; k < B; ++k) {
      const double v = fabs(a[k]);
      if (v > best) {
        best = v;
        q = k;
      }
    }
    q = __builtin_amdgcn_readlane(q, c);
    qs[c] = q;
    SPG_UNROLL for (int k = c + 1; k < B; ++k) {
      if (q == k) {   // uniform
        const double x = a[c];
        a[c] = a[k];
        a[k] = x;
      }
    }
    const double piv = row_bcast(a[c], c);
    int e;
    mant *= frexp(piv, &e);
    expo += e;
    const bool mine = lr == c;
    if (mine) own_piv = piv;
    // multiplier of this row (0 for the pivot row itself, which keeps its scale)
    const double l = mine ? 0.0 : a[c] / piv;
    SPG_UNROLL for (int k = c + 1; k < B; ++k) a[k] = fma(-l, row_bcast(a[k], c), a[k]);
    SPG_UNROLL for (int k = 0; k <= c; ++k) g[k] = fma(-l, row_bcast(g[k], c), g[k]);
  }
  // scale every row by its own pivot, then undo the column swaps (last swap first)
  const double is = 1.0 / own_piv;
  int pos = r;
  SPG_UNROLL for (int c = B - 1; c >= 0; --c) {
    const int q = qs[c];
    pos = pos == c ? q : (pos == q ? c : pos);
  }
  if (tid < B) {
    SPG_UNROLL for (int k = 0; k < B; ++k) G[pos * B + k] = g[k] * is;
  }
  tsync();
  return log(fabs(mant)) + expo * 0.69314718055994530942;
}

// G = (I + X J)^-1 for a leaf's node information J = s e0 e0^T (rank one, entry (0, 0) only):
// X J = s X[:, 0] e0^T, so G = I - s X[:, 0] e0^T / (1 + s X[0][0]) (Sherman-Morrison) and
// log det = log(1 + s X[0][0]).  Every lane returns the log-determinant.
template <int B>
SPG_DEV double t_inv_rank1(const double* X, double s, double* G) {
  const double d = fma(s, X[0], 1.0);
  const double f = s / d;
  for (int e = threadIdx.x; e < B * B; e += kW) {
    const int i = e / B, j = e - i * B;
    G[e] = (i == j ? 1.0 : 0.0) - (j == 0 ? f * X[i * B] : 0.0);
  }
  tsync();
  return log(d);
}

// G = (I + Q J)^-1 for a Q confined to the leading 2 x 2 block (a leaf edge of the Matern-3/2 +
// periodic model: the rotation blocks have Q = 0): with C = Q[0:2, 0:2], Q J = E2 C E2^T J, and
// Woodbury gives G = I - E2 K C E2^T J with the 2 x 2 K = (I + C J[0:2, 0:2])^-1.  Every lane
// forms K C from the eight entries it needs.
template <int B>
SPG_DEV void t_inv_q2(const double* Q, const double* J, double* G) {
  const double n00 = 1.0 + fma(Q[0], J[0], Q[1] * J[B]), n01 = fma(Q[0], J[1], Q[1] * J[B + 1]);
  const double n10 = fma(Q[B], J[0], Q[B + 1] * J[B]), n11 = 1.0 + fma(Q[B], J[1], Q[B + 1] * J[B + 1]);
  const double id = 1.0 / diff_of_products(n00, n11, n01, n10);
  // K = id [[n11, -n01], [-n10, n00]];  KC = K C
  const double kc00 = id * diff_of_products(n11, Q[0], n01, Q[B]);
  const double kc01 = id * diff_of_products(n11, Q[1], n01, Q[B + 1]);
  const double kc10 = id * diff_of_products(n00, Q[B], n10, Q[0]);
  const double kc11 = id * diff_of_products(n00, Q[B + 1], n10, Q[1]);
  for (int e = threadIdx.x; e < B * B; e += kW) {
    const int i = e / B, j = e - i * B;
    double g = (i == j) ? 1.0 : 0.0;
    if (i == 0) g -= fma(kc00, J[j], kc01 * J[B + j]);
    if (i == 1) g -= fma(kc10, J[j], kc11 * J[B + j]);
    G[e] = g;
  }
  tsync();
}

// ---------------------------------------------------------------------------- element ops
// The element operations below run as a few phases, one barrier each: the independent
// products of a phase on the matrix cores, and lanes < B the vectors.

// R = E1 (x) E2 (join at the shared node; see spingp_device.hpp).
// LEAF2: E2 is a leaf, whose J is rank one (the inverse in closed form).
// Scratch: M, its inverse G and later A2 P+ share one block; E1's Q1 takes G A1 once P+ = G Q1
// is formed, E2's J2 takes W A1 once W = J2 G is formed (both operands are consumed).  A team
// is one wavefront, so a block's last reads precede its next writes in program order (the
// pointers may alias, so the compiler keeps that order).
template <int B, bool LEAF2 = false>
SPG_DEV void t_combine(double* E1, double* E2, double* R, double* tmp) {
  using Y = Lay<B>;
  constexpr int BB = B * B;
  double *M = tmp, *G = tmp, *T = tmp, *Pp = tmp + BB, *W = tmp + 2 * BB;
  double* v = tmp + 3 * BB;   // three matrices and six vectors: 3 b^2 + 6 b doubles of scratch
  double *Gb = v, *Ppe = v + B, *g = v + 2 * B, *Gte = v + 3 * B, *Wb = v + 4 * B, *r = v + 5 * B;
  const double *A1 = E1 + Y::kA, *b1 = E1 + Y::kb, *Q1 = E1 + Y::kQ, *J1 = E1 + Y::kJ, *eta1 = E1 + Y::keta;
  const double *A2 = E2 + Y::kA, *b2 = E2 + Y::kb, *Q2 = E2 + Y::kQ, *J2 = E2 + Y::kJ, *eta2 = E2 + Y::keta;
  double* GA = E1 + Y::kQ;
  double* WA = E2 + Y::kJ;
  const int tid = threadIdx.x;
  double ld;
  if (LEAF2) {
    ld = t_inv_rank1<B>(Q1, J2[0], G);
  } else {
    mx_each<B>(mx<B, false, false>(Q1, J2), [&](int i, int j, double v) { M[i * B + j] = v + (i == j ? 1.0 : 0.0); });
    tsync();
    ld = t_inv_logdet<B>(M, G, nullptr);
  }
  // P+ = G Q1, W = J2 G (both symmetric), G A1 (into Q1's block, after its last read); G b1,
  // G^T eta2
  mx_store<B>(mx_sym<B, false, false>(G, Q1), Pp);
  mx_store<B>(mx_sym<B, false, false>(J2, G), W);
  mx_store<B>(mx<B, false, false>(G, A1), GA);
  if (tid < B) {
    double s1 = 0.0, s3 = 0.0;
    SPG_UNROLL for (int k = 0; k < B; ++k) {
      s1 = fma(G[tid * B + k], b1[k], s1);
      s3 = fma(G[k * B + tid], eta2[k], s3);
    }
    Gb[tid] = s1;
    Gte[tid] = s3;
  }
  tsync();
  // new transition A2 G A1, A2 P+ (into G's block), W A1 (into J2's block); P+ eta2, W b1 and
  // the vectors g, r
  mx_store<B>(mx<B, false, false>(A2, GA), R + Y::kA);
  mx_store<B>(mx<B, false, false>(A2, Pp), T);
  mx_store<B>(mx<B, false, false>(W, A1), WA);
  if (tid < B) {
    double s2 = 0.0, s4 = 0.0;
    SPG_UNROLL for (int k = 0; k < B; ++k) {
      s2 = fma(Pp[tid * B + k], eta2[k], s2);
      s4 = fma(W[tid * B + k], b1[k], s4);
    }
    Ppe[tid] = s2;
    Wb[tid] = s4;
    g[tid] = Gb[tid] + s2;
    r[tid] = Gte[tid] - s4;
  }
  tsync();
  // new noise A2 P+ A2^T + Q2, information J1 + A1^T W A1 (both symmetric), new offset and eta
  mx_each<B>(mx_sym<B, false, true>(T, A2), [&](int i, int j, double v) { R[Y::kQ + i * B + j] = v + Q2[i * B + j]; });
  mx_each<B>(mx_sym<B, true, false>(A1, WA), [&](int i, int j, double v) { R[Y::kJ + i * B + j] = J1[i * B + j] + v; });
  if (tid < B) {
    double s5 = 0.0, s6 = 0.0;
    SPG_UNROLL for (int k = 0; k < B; ++k) {
      s5 = fma(A2[tid * B + k], g[k], s5);
      s6 = fma(A1[k * B + tid], r[k], s6);
    }
    R[Y::kb + tid] = s5 + b2[tid];
    R[Y::keta + tid] = eta1[tid] + s6;
  }
  if (tid == 0) {
    const double cf = -0.5 * t_dot<B>(b1, Wb) + t_dot<B>(eta2, Gb) + 0.5 * t_dot<B>(eta2, Ppe);
    R[Y::kcf] = E1[Y::kcf] + E2[Y::kcf] + cf;
    R[Y::kcl] = E1[Y::kcl] + E2[Y::kcl] - 0.5 * ld;
  }
  tsync();
}

// Prefix: the predicted state N(m, P) at E's left node pushed through E -> (mo, Po); returns
// the log-normaliser increments in dcf, dcl (uniform over the team).
// LEAF: E is a leaf, whose J is rank one (the inverse in closed form).
template <int B, bool LEAF = false>
SPG_DEV void t_prefix(const double* m, const double* P, const double* E, double* mo, double* Po, double* tmp,
                      double& dcf, double& dcl) {
  using Y = Lay<B>;
  constexpr int BB = B * B;
  // M and its inverse G share a block (see t_combine)
  double *M = tmp, *G = tmp, *Pp = tmp + BB, *T = tmp + 2 * BB;
  double* v = tmp + 3 * BB;   // three matrices and five vectors: 3 b^2 + 5 b doubles of scratch
  double *Gm = v, *Ppe = v + B, *g = v + 2 * B, *Wm = v + 3 * B, *Jm = v + 4 * B;
  const double *A = E + Y::kA, *bb = E + Y::kb, *Q = E + Y::kQ, *J = E + Y::kJ, *eta = E + Y::keta;
  const int tid = threadIdx.x;
  double ld;
  if (LEAF) {
    ld = t_inv_rank1<B>(P, J[0], G);
  } else {
    mx_each<B>(mx<B, false, false>(P, J), [&](int i, int j, double v) { M[i * B + j] = v + (i == j ? 1.0 : 0.0); });
    tsync();
    ld = t_inv_logdet<B>(M, G, nullptr);
  }
  // P+ = sym(G P); W = sym(J G) enters only through W m = (J G m + G^T J m) / 2
  mx_store<B>(mx_sym<B, false, false>(G, P), Pp);
  if (tid < B) {
    double s1 = 0.0, s5 = 0.0;
    SPG_UNROLL for (int k = 0; k < B; ++k) {
      s1 = fma(G[tid * B + k], m[k], s1);
      s5 = fma(J[tid * B + k], m[k], s5);
    }
    Gm[tid] = s1;
    Jm[tid] = s5;
  }
  tsync();
  mx_store<B>(mx<B, false, false>(A, Pp), T);
  if (tid < B) {
    double s2 = 0.0, s3 = 0.0, s6 = 0.0;
    SPG_UNROLL for (int k = 0; k < B; ++k) {
      s2 = fma(Pp[tid * B + k], eta[k], s2);
      s3 = fma(J[tid * B + k], Gm[k], s3);
      s6 = fma(G[k * B + tid], Jm[k], s6);
    }
    Ppe[tid] = s2;
    Wm[tid] = 0.5 * (s3 + s6);
    g[tid] = Gm[tid] + s2;
  }
  tsync();
  mx_each<B>(mx_sym<B, false, true>(T, A), [&](int i, int j, double v) { Po[i * B + j] = v + Q[i * B + j]; });
  if (tid < B) {
    double s4 = 0.0;
    SPG_UNROLL for (int k = 0; k < B; ++k) s4 = fma(A[tid * B + k], g[k], s4);
    mo[tid] = s4 + bb[tid];
  }
  dcf = -0.5 * t_dot<B>(m, Wm) + t_dot<B>(eta, Gm) + 0.5 * t_dot<B>(eta, Ppe) + E[Y::kcf];
  dcl = -0.5 * ld + E[Y::kcl];
  tsync();
}

// Suffix: information (Jb, etab) on E's right node pulled back to its left node -> (Jo, etao).
// Q2: E's Q is confined to the leading 2 x 2 block (the inverse in closed form).
template <int B, bool Q2 = false>
SPG_DEV void t_suffix(const double* E, const double* Jb, const double* etab, double* Jo, double* etao, double* tmp) {
  using Y = Lay<B>;
  constexpr int BB = B * B;
  // M, its inverse G and later W A share a block (see t_combine)
  double *M = tmp, *G = tmp, *WA = tmp, *W = tmp + BB;
  double* v = tmp + 2 * BB;   // two matrices and two vectors: 2 b^2 + 2 b doubles of scratch
  double *s1v = v, *r = v + B;
  const double *A = E + Y::kA, *bb = E + Y::kb, *Q = E + Y::kQ, *J = E + Y::kJ, *eta = E + Y::keta;
  const int tid = threadIdx.x;
  if (Q2) {
    t_inv_q2<B>(Q, Jb, G);
  } else {
    mx_each<B>(mx<B, false, false>(Q, Jb), [&](int i, int j, double v) { M[i * B + j] = v + (i == j ? 1.0 : 0.0); });
    tsync();
    (void)t_inv_logdet<B>(M, G, nullptr);
  }
  mx_store<B>(mx_sym<B, false, false>(Jb, G), W);
  if (tid < B) {
    double s1 = 0.0;
    SPG_UNROLL for (int k = 0; k < B; ++k) s1 = fma(G[k * B + tid], etab[k], s1);
    s1v[tid] = s1;
  }
  tsync();
  mx_store<B>(mx<B, false, false>(W, A), WA);
  if (tid < B) {
    double s2 = 0.0;
    SPG_UNROLL for (int k = 0; k < B; ++k) s2 = fma(W[tid * B + k], bb[k], s2);
    r[tid] = s1v[tid] - s2;
  }
  tsync();
  mx_each<B>(mx_sym<B, true, false>(A, WA), [&](int i, int j, double v) { Jo[i * B + j] = J[i * B + j] + v; });
  if (tid < B) {
    double s3 = 0.0;
    SPG_UNROLL for (int k = 0; k < B; ++k) s3 = fma(A[k * B + tid], r[k], s3);
    etao[tid] = eta[tid] + s3;
  }
  tsync();
}

// Items of a level kernel are fetched one iteration ahead: each lane loads its share of the next
// item's operands (consecutive doubles over the lanes) into registers while the team works on
// the current one, so the global-memory latency overlaps the element operation.  Above b = 12
// the level kernels' registers are taken by the element operations and their operands are
// loaded when used.
template <int B>
struct Ahead {
  static constexpr bool kOn = B <= 12;
  // the node step prefetches at every b (above b = 12 it runs one team per SIMD, which leaves
  // the registers for it)
  static constexpr bool kNode = true;
};
// Waves per SIMD the team kernels are compiled for (register budget of 512 / waves per lane,
// MFMA accumulators included): at b <= 12 three teams of the up and down kernels, two of the
// node step and four of the leaves stay resident, above b = 12 two, one and three (the LDS
// per team allows as many, except for the leaves at b = 15 and 16, which stage their element
// in LDS: two).
template <int B>
struct Occ {
  static constexpr int kLevel = B <= 12 ? 3 : 2;
  static constexpr int kNode = B <= 12 ? 2 : 1;
  static constexpr int kLeaf = B <= 12 ? 4 : 3;
};

// ---------------------------------------------------------------------------- the model
// A sum of terms (spingp_sumdesc.hpp), each a block of the state:
//   Matern-nu, m = nu + 1/2 states (f and its derivatives), lam = sqrt(2 nu) / l: the closed
//     forms of spingp_device.hpp (transition, stationary covariance, d/dlam);
//   periodic with J harmonics: the truncated cosine series of the periodic kernel with weights
//     q_h^2 = var_P c_h exp(-x) I_h(x), x = 1 / l_P^2, c_0 = 1, c_h = 2; harmonic h is a
//     rotation by h w dt (w = 2 pi / period) with Q = 0;
//   quasi-periodic: the periodic term times exp(-|tau| / l_D): every harmonic block is
//     e^{-dt / l_D} times the rotation and has Q = q_h^2 (1 - e^{-2 dt / l_D}) I;
//   squared exponential of even order n by its spectral approximation (state f, f', ...,
//     f^(n-1), lam = 1 / l), kept in the scaled state f^(k) / lam^k: there the transition is
//     expm(C1 lam dt) = 2 Re sum_k Z_k e^{r_k lam dt} over the stable roots with Im r_k > 0
//     and P0 = var P1 (tables from the unit-lengthscale companion matrix C1), with no powers
//     of lam (in the original basis P0 spans lam^(2 n - 2), which FP64 cannot carry for short
//     lengthscales); its Q is formed as P0 - A P0 A^T.  State outputs are scaled back by lam^k.
// Hyperparameters per term in list order: Matern (l, var), periodic (l_P, var_P, period),
// quasi-periodic (l_P, var_P, period, l_D), squared exponential (l, var); then s2.
// Term constants (from c0): Matern lam, var, l; periodic and quasi-periodic l_P, var_P,
// period, w, x, lam_D (quasi-periodic), q_h^2 (J + 1), dq_h^2/dx (J + 1); squared exp. lam, var.
template <int B>
struct Consts {
  // s2, at most 64 doubles of term constants, the output scale, P0', P0
  static constexpr int kMax = 1 + 64 + B + 2 * B * B;
  static constexpr int kNoP0o = kMax - B * B;   // all but the original-basis P0 (the last block)
};

SPG_DEV bool observed(const SumDesc& d, int k) { return ((d.obs >> k) & 1u) != 0u; }
// T (row 0 = h^T, identity below) and T^-1 (row 0 = (1, -h_1, ..., -h_{B-1}), identity below)
SPG_DEV double T_at(const SumDesc& d, int i, int j) {
  return i == 0 ? (observed(d, j) ? 1.0 : 0.0) : (i == j ? 1.0 : 0.0);
}
SPG_DEV double Ti_at(const SumDesc& d, int i, int j) {
  if (i == 0) return j == 0 ? 1.0 : (observed(d, j) ? -1.0 : 0.0);
  return i == j ? 1.0 : 0.0;
}
// entry (i, j) of T^T X T^-T for a row-major X in LDS, from the sparsity of T:
// (X T^-T)[k][0] = X[k][0] - sum over observed l >= 1 of X[k][l], (X T^-T)[k][j] = X[k][j]
// for j >= 1; (T^T Y)[i][j] = Y[i][j] + [i >= 1 observed] Y[0][j]
template <int B>
SPG_DEV double abar_orig(const SumDesc& d, const double* X, int i, int j) {
  auto y = [&](int k) {
    double v = X[k * B + j];
    if (j == 0)
      for (int l = 1; l < B; ++l)
        if (observed(d, l)) v -= X[k * B + l];
    return v;
  };
  double r = y(i);
  if (i >= 1 && observed(d, i)) r += y(0);
  return r;
}

// Matern block of order m (1..4) over dt, written to eb (m^2 each, row-major): with DERIV the
// derivative dA/dlam at eb[2 m^2] (the node step), else the transition A at eb[0] and
// Q = P0 - A P0 A^T at eb[m^2] (the leaves).
template <int M, bool DERIV>
SPG_DEV void matern_block_m(const double* ct, double dt, double* eb) {
  SeriesPar p;
  p.lam = ct[0];
  p.var = ct[1];
  p.ell = ct[2];
  p.s2 = 1.0;
  double e, A[M][M];
  Matern<M>::transition(p, dt, e, A);
  if (DERIV) {
    SPG_UNROLL for (int r = 0; r < M; ++r) SPG_UNROLL for (int c = 0; c < M; ++c) {
      double Ab[M][M];
      SPG_UNROLL for (int k = 0; k < M; ++k) SPG_UNROLL for (int l = 0; l < M; ++l) Ab[k][l] = (k == r && l == c) ? 1.0 : 0.0;
      eb[2 * M * M + r * M + c] = Matern<M>::dA_dlam_dot(p, dt, e, Ab);
    }
  } else {
    double P[M][M];
    Matern<M>::pinf(p, P);
    SPG_UNROLL for (int r = 0; r < M; ++r) {
      double T[M];
      SPG_UNROLL for (int c = 0; c < M; ++c) {
        double s = 0.0;
        SPG_UNROLL for (int k = 0; k < M; ++k) s = fma(A[r][k], P[k][c], s);
        T[c] = s;
      }
      SPG_UNROLL for (int c = 0; c < M; ++c) {
        double s = P[r][c];
        SPG_UNROLL for (int k = 0; k < M; ++k) s = fma(-T[k], A[c][k], s);
        eb[r * M + c] = A[r][c];
        eb[M * M + r * M + c] = s;
      }
    }
  }
}
template <bool DERIV>
SPG_DEV void matern_block(int m, const double* ct, double dt, double* eb) {
  switch (m) {
    case 1: matern_block_m<1, DERIV>(ct, dt, eb); break;
    case 2: matern_block_m<2, DERIV>(ct, dt, eb); break;
    case 3: matern_block_m<3, DERIV>(ct, dt, eb); break;
    default: matern_block_m<4, DERIV>(ct, dt, eb); break;
  }
}
template <int M>
SPG_DEV double matern_p0_m(const double* ct, int r, int c) {
  SeriesPar p;
  p.lam = ct[0];
  p.var = ct[1];
  p.ell = ct[2];
  p.s2 = 1.0;
  double P[M][M];
  Matern<M>::pinf(p, P);
  double v = 0.0;
  SPG_UNROLL for (int k = 0; k < M; ++k) SPG_UNROLL for (int l = 0; l < M; ++l) v = (k == r && l == c) ? P[k][l] : v;
  return v;
}
SPG_DEV double matern_p0(int m, const double* ct, int r, int c) {
  switch (m) {
    case 1: return matern_p0_m<1>(ct, r, c);
    case 2: return matern_p0_m<2>(ct, r, c);
    case 3: return matern_p0_m<3>(ct, r, c);
    default: return matern_p0_m<4>(ct, r, c);
  }
}
// <Pb block, P0 / var> and <Pb block, dP0/dlam> of a Matern block
template <int M>
SPG_DEV void matern_grad_m(const double* ct, const double* Pb, int ld, double& gvar, double& glam) {
  SeriesPar p;
  p.lam = ct[0];
  p.var = ct[1];
  p.ell = ct[2];
  p.s2 = 1.0;
  double P[M][M], dP[M][M];
  Matern<M>::pinf(p, P);
  Matern<M>::dpinf_dlam(p, dP);
  gvar = glam = 0.0;
  SPG_UNROLL for (int r = 0; r < M; ++r) SPG_UNROLL for (int c = 0; c < M; ++c) {
    gvar = fma(Pb[r * ld + c], P[r][c] / p.var, gvar);
    glam = fma(Pb[r * ld + c], dP[r][c], glam);
  }
}
SPG_DEV void matern_grad(int m, const double* ct, const double* Pb, int ld, double& gvar, double& glam) {
  switch (m) {
    case 1: matern_grad_m<1>(ct, Pb, ld, gvar, glam); break;
    case 2: matern_grad_m<2>(ct, Pb, ld, gvar, glam); break;
    case 3: matern_grad_m<3>(ct, Pb, ld, gvar, glam); break;
    default: matern_grad_m<4>(ct, Pb, ld, gvar, glam); break;
  }
}

// The transcendental part of an edge of length dt, formed by one lane: into es (two doubles
// per scalar) (cos, sin) of h w dt per harmonic and exp(-dt / l_D) (quasi-periodic),
// e^{r_k lam dt} as (re, im) per root (squared exponential); into eb every Matern term's block
// (A, Q = P0 - A P0 A^T and dA/dlam).  es and eb may be global memory.
SPG_DEV void edge_row(const SumDesc& d, const double* c, double dt, double* es, double* eb) {
  for (int u = 0; u < d.nt; ++u) {
    const TermInfo& T = d.t[u];
    const double* ct = c + T.c0;
    if (T.type == kTermMatern) {
      matern_block<false>(T.order, ct, dt, eb + T.blk0);
      matern_block<true>(T.order, ct, dt, eb + T.blk0);
    } else if (T.type == kTermSqExp) {
      const double x = ct[0] * dt;
      const int o = kSqExpRootOff[T.order / 2 - 1];
      for (int q = 0; q < T.njob; ++q) {
        const double m = exp(kSqExpRootRe[o + q] * x);
        double sn, cs;
        sincos(kSqExpRootIm[o + q] * x, &sn, &cs);
        es[2 * (T.job0 + q)] = m * cs;
        es[2 * (T.job0 + q) + 1] = m * sn;
      }
    } else {
      for (int q = 0; q <= T.order; ++q) {
        double sn, cs;
        sincos((double)q * ct[3] * dt, &sn, &cs);
        es[2 * (T.job0 + q)] = cs;
        es[2 * (T.job0 + q) + 1] = sn;
      }
      if (T.type == kTermQuasi) {
        es[2 * (T.job0 + T.order + 1)] = exp(-ct[5] * dt);
        es[2 * (T.job0 + T.order + 1) + 1] = 0.0;
      }
    }
  }
}
// Doubles of one edge row: the scalars, then the Matern blocks.
SPG_DEV int edge_row_size(const SumDesc& d) { return 2 * d.njob + d.nblk; }

// Support index of block-local entry (r, c) of term T, or -1.
SPG_DEV int support_index(const TermInfo& T, int r, int c) {
  if (T.type == kTermMatern || T.type == kTermSqExp) return T.sup0 + r * T.n + c;
  if ((r >> 1) != (c >> 1)) return -1;
  return T.sup0 + 4 * (r >> 1) + 2 * (r & 1) + (c & 1);
}

// Entry (r, c) of term T's block (block-local indices; 0 outside the harmonic 2 x 2 blocks).
SPG_DEV void term_entry(const TermInfo& T, const double* c, const double* es, const double* eb, double dt, int r,
                        int cc, double& a, double& q, double& da0, double& da1) {
  a = q = da0 = da1 = 0.0;
  const double* ct = c + T.c0;
  if (T.type == kTermMatern) {
    const int m = T.n, o = T.blk0 + r * m + cc;
    a = eb[o];
    q = eb[o + m * m];
    da0 = eb[o + 2 * m * m];
  } else if (T.type == kTermSqExp) {
    // scaled state: A = E(lam dt) = expm(C1 lam dt), dA/dlam = dt C1 E(lam dt)
    const int n = T.order, h = n / 2;
    const int zo = kSqExpZOff[h - 1] + (r * n + cc) * h, ro = kSqExpRootOff[h - 1];
    double s = 0.0, ds = 0.0;
    for (int k = 0; k < h; ++k) {
      const double er = es[2 * (T.job0 + k)], ei = es[2 * (T.job0 + k) + 1];
      const double zr = kSqExpZRe[zo + k], zi = kSqExpZIm[zo + k];
      const double pr = zr * er - zi * ei, pi = zr * ei + zi * er;   // Z e^{r x}
      s += pr;
      ds += kSqExpRootRe[ro + k] * pr - kSqExpRootIm[ro + k] * pi;  // Re(r Z e^{r x})
    }
    a = 2.0 * s;
    da0 = 2.0 * dt * ds;
  } else {
    const int h = r >> 1;
    if ((cc >> 1) != h) return;
    const int ri = r & 1, rj = cc & 1;
    const double cs = es[2 * (T.job0 + h)], sn = es[2 * (T.job0 + h) + 1];
    // [[cos, -sin], [sin, cos]] and its derivative in the angle [[-sin, -cos], [cos, -sin]],
    // times d angle / d period
    const double rv = ri == rj ? cs : (ri == 0 ? -sn : sn);
    const double drv = ri == rj ? -sn : (ri == 0 ? -cs : cs);
    const double th = (double)h * ct[3] * dt;
    const bool quasi = T.type == kTermQuasi;
    const double ed = quasi ? es[2 * (T.job0 + T.order + 1)] : 1.0;
    a = ed * rv;
    da0 = ed * drv * (-th / ct[2]);
    if (quasi) {
      da1 = -dt * a;
      if (ri == rj) q = ct[6 + h] * (1.0 - ed * ed);
    }
  }
}
// Entry (i, j) of the whole transition: term_of[k] is the term of state k (block diagonal).
SPG_DEV void edge_entry(const TermInfo* tt, const int* term_of, const double* c, const double* es, const double* eb,
                        double dt, int i, int j, double& a, double& q, double& da0, double& da1) {
  const int u = term_of[i];
  if (u != term_of[j]) {
    a = q = da0 = da1 = 0.0;
    return;
  }
  const TermInfo& T = tt[u];
  term_entry(T, c, es, eb, dt, i - T.s0, j - T.s0, a, q, da0, da1);
}

// Entry (i, j) of the original-basis stationary covariance P0.
SPG_DEV double p0_entry(const SumDesc& d, const TermInfo* tt, const double* c, int i, int j) {
  double v = 0.0;
  for (int u = 0; u < d.nt; ++u) {
    const TermInfo T = tt[u];
    const int r = i - T.s0, cc = j - T.s0;
    if (r < 0 || r >= T.n || cc < 0 || cc >= T.n) continue;
    const double* ct = c + T.c0;
    if (T.type == kTermMatern) v = matern_p0(T.order, ct, r, cc);
    else if (T.type == kTermSqExp) v = ct[1] * kSqExpP1[kSqExpP1Off[T.order / 2 - 1] + r * T.n + cc];
    else v = r == cc ? ct[6 + (r >> 1)] : 0.0;
  }
  return v;
}

// Support entry s (an entry of the transition with a derivative) -> (i, j) and its term.
SPG_DEV int support(const SumDesc& d, const TermInfo* tt, int s, int& i, int& j) {
  int term = 0;
  i = j = 0;
  for (int u = 0; u < d.nt; ++u) {
    const TermInfo T = tt[u];
    const int l = s - T.sup0;
    if (l < 0 || l >= T.nsup) continue;
    term = u;
    if (T.type == kTermMatern || T.type == kTermSqExp) {
      i = T.s0 + l / T.n;
      j = T.s0 + l % T.n;
    } else {
      const int h = l >> 2;
      i = T.s0 + 2 * h + ((l >> 1) & 1);
      j = T.s0 + 2 * h + (l & 1);
    }
  }
  return term;
}

// Gradient of the raw hyperparameters from the summed partials: tot[B*B + f] are the channel
// sums, tot[B*B + na] the noise sum, Pb the original-basis P0_bar (one lane).
template <int B>
SPG_DEV void final_grad(const SumDesc& d, const TermInfo* tt, const double* c, const double* tot, const double* Pb, double* grad) {
  constexpr int BB = B * B;
  for (int u = 0; u < d.nt; ++u) {
    const TermInfo T = tt[u];
    const double* ct = c + T.c0;
    const double* pb = Pb + T.s0 * B + T.s0;
    double* g = grad + T.h0;
    if (T.type == kTermMatern) {
      double gvar, glam;
      matern_grad(T.order, ct, pb, B, gvar, glam);
      const double lam = ct[0], ell = ct[2];
      g[0] = (tot[BB + T.ch0] + glam) * (-lam / ell);   // d lam / d l = -lam / l
      g[1] = gvar;
    } else if (T.type == kTermSqExp) {
      // in the scaled state P0 = var P1 does not depend on lam
      const double lam = ct[0];
      const int po = kSqExpP1Off[T.order / 2 - 1];
      double gv = 0.0;
      for (int r = 0; r < T.n; ++r)
        for (int cc = 0; cc < T.n; ++cc) gv = fma(pb[r * B + cc], kSqExpP1[po + r * T.n + cc], gv);
      g[0] = tot[BB + T.ch0] * (-lam * lam);   // d lam / d l = -lam^2
      g[1] = gv;
    } else {
      // P0 is diagonal in the harmonic blocks
      const double ell = ct[0], var = ct[1];
      double gl = 0.0, gv = 0.0;
      for (int r = 0; r < T.n; ++r) {
        const int h = r >> 1;
        const double v = pb[r * B + r];
        gl = fma(v, ct[7 + T.order + h] * (-2.0 / (ell * ell * ell)), gl);
        gv = fma(v, ct[6 + h] / var, gv);
      }
      g[0] = gl;
      g[1] = gv;
      g[2] = tot[BB + T.ch0];
      if (T.type == kTermQuasi) g[3] = tot[BB + T.ch0 + 1] * (-ct[5] * ct[5]);   // d lam_D / d l_D
    }
  }
  grad[d.nh - 1] = tot[BB + d.na];
}

// exp(-x) I_j(x) by its power series, summed in log space (no overflow for large x).
SPG_DEV double bessel_ive(int j, double x) {
  if (j < 0) j = -j;
  if (!(x > 0.0)) return j == 0 ? 1.0 : 0.0;
  const double lh = log(0.5 * x);
  double lt = j * lh - lgamma(j + 1.0) - x;
  double s = 0.0;
  for (int k = 0; k < 200000; ++k) {
    const double tk = exp(lt);
    s += tk;
    if (k > 0.5 * x + 8.0 && tk <= 1e-18 * s) break;
    lt += 2.0 * lh - log((double)(k + 1)) - log((double)(k + 1 + j));
  }
  return s;
}

// ---------------------------------------------------------------------------- kernels
// Model constants from the hyperparameter row (one work-group).
template <int B>
__global__ __launch_bounds__(kW) void k_wide_setup(SumDesc d, const double* __restrict__ hyper,
                                                   double* __restrict__ cst) {
  constexpr int BB = B * B;
  __shared__ double c[Consts<B>::kMax];
  __shared__ double X[BB];
  __shared__ TermInfo tt[kMaxTerms];
  const int tid = threadIdx.x;
  if (tid < d.nt) tt[tid] = d.t[tid];
  for (int e = tid; e < d.kConst; e += kW) c[e] = 0.0;
  tsync();
  if (tid == 0) {
    c[d.kS2] = hyper[d.nh - 1];
    for (int u = 0; u < d.nt; ++u) {
      const TermInfo T = tt[u];
      const double* h = hyper + T.h0;
      double* ct = c + T.c0;
      if (T.type == kTermMatern) {
        const double nu2 = 2.0 * T.order - 1.0;   // 2 nu
        ct[0] = sqrt(nu2) / h[0];
        ct[1] = h[1];
        ct[2] = h[0];
      } else if (T.type == kTermSqExp) {
        ct[0] = 1.0 / h[0];
        ct[1] = h[1];
      } else {
        ct[0] = h[0];
        ct[1] = h[1];
        ct[2] = h[2];
        ct[3] = 6.283185307179586477 / h[2];
        ct[4] = 1.0 / (h[0] * h[0]);
        ct[5] = T.type == kTermQuasi ? 1.0 / h[3] : 0.0;
      }
    }
  }
  tsync();
  // q_h^2 and dq_h^2 / dx, with d(e^-x I_h)/dx = (I_{h-1} + I_{h+1}) e^-x / 2 - e^-x I_h
  for (int u = 0; u < d.nt; ++u) {
    const TermInfo T = tt[u];
    if (T.type != kTermPeriodic && T.type != kTermQuasi) continue;
    double* ct = c + T.c0;
    if (tid <= T.order) {
      const double x = ct[4], cj = tid == 0 ? 1.0 : 2.0;
      const double i0 = bessel_ive(tid, x), im = bessel_ive(tid - 1, x), ip = bessel_ive(tid + 1, x);
      ct[6 + tid] = ct[1] * cj * i0;
      ct[7 + T.order + tid] = ct[1] * cj * (0.5 * (im + ip) - i0);
    }
    tsync();
  }
  // output scale: lam^k on the squared-exponential blocks
  if (tid < B) {
    double sc = 1.0;
    for (int u = 0; u < d.nt; ++u) {
      const TermInfo T = tt[u];
      const int r = tid - T.s0;
      if (T.type == kTermSqExp && r >= 0 && r < T.n) sc = pow(c[T.c0], (double)r);
    }
    c[d.kScale + tid] = sc;
  }
  for (int e = tid; e < BB; e += kW) c[d.kP0o + e] = p0_entry(d, tt, c, e / B, e % B);
  tsync();
  // P0' = T P0 T^T
  for (int e = tid; e < BB; e += kW) {
    const int i = e / B, j = e - i * B;
    double s = 0.0;
    for (int k = 0; k < B; ++k) s = fma(T_at(d, i, k), c[d.kP0o + k * B + j], s);
    X[e] = s;
  }
  tsync();
  for (int e = tid; e < BB; e += kW) {
    const int i = e / B, j = e - i * B;
    double s = 0.0;
    for (int k = 0; k < B; ++k) s = fma(X[i * B + k], T_at(d, j, k), s);
    c[d.kP0 + e] = s;
  }
  tsync();
  for (int e = tid; e < d.kConst; e += kW) cst[e] = c[e];
}

// Edges, one lane each: the transcendental part of edge n -> n+1 (zero after the last node)
// into row n of edges (edge_row_size doubles), read by the leaves.
constexpr int kEdgeThreads = 128;
template <int B>
__global__ __launch_bounds__(kEdgeThreads) void k_wide_edges(SumDesc d, const double* __restrict__ t, int64_t n_pts,
                                                             const double* __restrict__ cst,
                                                             double* __restrict__ edges) {
  const int64_t n = (int64_t)blockIdx.x * kEdgeThreads + threadIdx.x;
  if (n >= n_pts) return;
  const int rs = edge_row_size(d);
  double* row = edges + n * rs;
  if (n + 1 < n_pts) {
    edge_row(d, cst, t[n + 1] - t[n], row, row + 2 * d.njob);
  } else {
    for (int e = 0; e < rs; ++e) row[e] = 0.0;
  }
}

// Leaf n: node n's information and the edge n -> n+1 (A = 0, Q = 0 after the last node).
template <int B>
__global__ __launch_bounds__(kW, Occ<B>::kLeaf) void k_wide_leaf(SumDesc d, const double* __restrict__ t,
                                                  const double* __restrict__ y, int64_t n_pts,
                                                  const double* __restrict__ cst, const double* __restrict__ edges,
                                                  double* __restrict__ elems, double* __restrict__ deriv) {
  constexpr int BB = B * B;
  using Y = Lay<B>;
  __shared__ double c[Consts<B>::kMax];
  // A, Q and one product block are staged here; the element goes straight to global memory up
  // to b = 14 and through LDS above (measured: 12 % faster at b = 13 and 14 without the
  // staging, 3 % slower at b = 15 and 16)
  constexpr bool kStage = B >= 15;
  __shared__ double Ao[BB], Qo[BB], X[BB], es[2 * kMaxJobs], eb[kMaxBlk], Es[kStage ? Y::kEs : 1];
  __shared__ TermInfo tt[kMaxTerms];
  __shared__ int term_of[B];
  const int tid = threadIdx.x;
  if (tid < d.nt) tt[tid] = d.t[tid];
  if (tid < B) {
    int u = 0;
    for (int v = 1; v < d.nt; ++v)
      if (tid >= d.t[v].s0) u = v;
    term_of[tid] = u;
  }
  for (int e = tid; e < d.kConst; e += kW) c[e] = cst[e];
  tsync();
  const double s2 = c[d.kS2];
  const double* P0o = c + d.kP0o;
  for (int64_t n = blockIdx.x; n < n_pts; n += gridDim.x) {
    const bool edge = n + 1 < n_pts;
    const double dt = edge ? t[n + 1] - t[n] : 0.0;
    {
      const int rs = edge_row_size(d), ns2 = 2 * d.njob;
      const double* row = edges + n * rs;
      for (int e = tid; e < rs; e += kW) {
        if (e < ns2) es[e] = row[e];
        else eb[e - ns2] = row[e];
      }
    }
    tsync();
    // the transition's derivatives on the support go to deriv (the term's channels per entry),
    // for the node step of the same edge
    double* dv = deriv + n * d.ndv;
    for (int e = tid; e < BB; e += kW) {
      const int i = e / B, j = e - i * B;
      double a = 0.0, q = 0.0, d0 = 0.0, d1 = 0.0;
      if (edge) edge_entry(tt, term_of, c, es, eb, dt, i, j, a, q, d0, d1);
      Ao[e] = a;
      Qo[e] = q;
      const int u = term_of[i];
      if (u == term_of[j]) {
        const TermInfo& T = tt[u];
        const int sidx = support_index(T, i - T.s0, j - T.s0);
        if (sidx >= 0) {
          const int o = T.dv0 + (sidx - T.sup0) * T.nch;
          dv[o] = d0;
          if (T.nch == 2) dv[o + 1] = d1;
        }
      }
    }
    tsync();
    if (d.has_se) {
      // squared-exponential blocks: Q = P0 - A P0 A^T (block diagonal, so the full products
      // give each block's own)
      mx_store<B>(mx<B, false, false>(Ao, P0o), X);
      tsync();
      const v4d apa = mx<B, false, true>(X, Ao);
      mx_each<B>(apa, [&](int i, int j, double v) {
        const int u = term_of[i];
        if (u == term_of[j] && tt[u].type == kTermSqExp) Qo[i * B + j] = edge ? P0o[i * B + j] - v : 0.0;
      });
      tsync();
    }
    // A' = T A T^-1 and Q' = T Q T^T from the sparsity of T (identity but row 0 = h^T):
    // (T X)[0][j] = sum over observed k of X[k][j], (X T^-1)[i][j] = X[i][j] - X[i][0] for an
    // observed j >= 1, (X T^T)[i][0] = sum over observed k of X[i][k]; other entries unchanged.
    // The sums load every term and add the observed ones (in the same order).
    double* const gout = elems + n * Y::kEs;
    double* const out = kStage ? Es : gout;
    for (int e = tid; e < BB; e += kW) {
      const int i = e / B, j = e - i * B;
      double s = Ao[e];
      if (i == 0)
        SPG_UNROLL for (int k = 1; k < B; ++k) {
          const double v = Ao[k * B + j];
          s = observed(d, k) ? s + v : s;
        }
      X[e] = s;
    }
    tsync();
    for (int e = tid; e < BB; e += kW) {
      const int i = e / B, j = e - i * B;
      out[Y::kA + e] = (j >= 1 && observed(d, j)) ? -X[i * B] + X[e] : X[e];
    }
    for (int e = tid; e < BB; e += kW) {
      const int i = e / B, j = e - i * B;
      double s = Qo[e];
      if (i == 0)
        SPG_UNROLL for (int k = 1; k < B; ++k) {
          const double v = Qo[k * B + j];
          s = observed(d, k) ? s + v : s;
        }
      X[e] = s;
    }
    tsync();
    // Q' = (T Q) T^T into A's block (no longer read), then written out symmetrised
    for (int e = tid; e < BB; e += kW) {
      const int i = e / B;
      double s = X[e];
      if (e - i * B == 0)
        SPG_UNROLL for (int k = 1; k < B; ++k) {
          const double v = X[i * B + k];
          s = observed(d, k) ? s + v : s;
        }
      Ao[e] = s;
    }
    tsync();
    // a NaN observation marks a node without one (a prediction time): no information
    const double yn = y[n];
    const bool obs = yn == yn;
    for (int e = tid; e < BB; e += kW) {
      const int i = e / B, j = e - i * B;
      out[Y::kQ + e] = i == j ? Ao[e] : 0.5 * (Ao[e] + Ao[j * B + i]);
      out[Y::kJ + e] = (e == 0 && obs) ? 1.0 / s2 : 0.0;
    }
    if (tid < B) {
      out[Y::kb + tid] = 0.0;
      out[Y::keta + tid] = (tid == 0 && obs) ? yn / s2 : 0.0;
    }
    if (tid == 0) {
      out[Y::kcf] = obs ? -0.5 * yn * yn / s2 : 0.0;
      out[Y::kcl] = obs ? -0.5 * (kLog2Pi + log(s2)) : 0.0;
    }
    if (kStage) {
      tsync();
      for (int e = tid; e < Y::kEs; e += kW) gout[e] = e < Y::kE ? Es[e] : 0.0;
    } else {
      for (int e = Y::kE + tid; e < Y::kEs; e += kW) gout[e] = 0.0;
    }
    tsync();
  }
}

// Up-sweep: level k (n_cur elements at off_cur) from level k - 1 (n_prev at off_prev).
// LEAF: level k - 1 is the leaf level (every right operand is a leaf).
template <int B, bool LEAF = false>
__global__ __launch_bounds__(kW, Occ<B>::kLevel) void k_wide_up(double* __restrict__ elems, int64_t off_prev, int64_t n_prev,
                                                int64_t off_cur, int64_t n_cur) {
  using Y = Lay<B>;
  __shared__ double E1[Y::kEs], E2[Y::kEs], tmp[Y::kTmpJoin];
  const int tid = threadIdx.x;
  constexpr int kTwo = 2 * Y::kEs;                 // the two operands are adjacent in memory
  constexpr int NP = Ahead<B>::kOn ? (kTwo + kW - 1) / kW : 1;
  double pre[NP];
  auto fetch = [&](int64_t it) {
    if (it >= n_cur) return;
    const double* a = elems + (off_prev + 2 * it) * Y::kEs;
    const int lim = 2 * it + 1 < n_prev ? kTwo : Y::kEs;
    SPG_UNROLL for (int j = 0; j < NP; ++j) {
      const int e = tid + j * kW;
      if (e < lim) pre[j] = a[e];
    }
  };
  if (Ahead<B>::kOn) fetch(blockIdx.x);
  for (int64_t i = blockIdx.x; i < n_cur; i += gridDim.x) {
    const double* a = elems + (off_prev + 2 * i) * Y::kEs;
    double* out = elems + (off_cur + i) * Y::kEs;
    const bool paired = 2 * i + 1 < n_prev;
    if (Ahead<B>::kOn) {
      SPG_UNROLL for (int j = 0; j < NP; ++j) {
        const int e = tid + j * kW;
        if (e < Y::kEs) E1[e] = pre[j];
        else if (e < kTwo && paired) E2[e - Y::kEs] = pre[j];
      }
      tsync();
      fetch(i + gridDim.x);
    } else {
      for (int e = tid; e < Y::kEs; e += kW) {
        E1[e] = a[e];
        if (paired) E2[e] = a[Y::kEs + e];
      }
      tsync();
    }
    if (!paired) {                             // unpaired tail: passes through
      for (int e = tid; e < Y::kEs; e += kW) out[e] = E1[e];
      tsync();
      continue;
    }
    t_combine<B, LEAF>(E1, E2, out, tmp);     // the result goes straight to global memory
    for (int e = Y::kE + tid; e < Y::kEs; e += kW) out[e] = 0.0;
    tsync();
  }
}

// Root: messages of the root element (prefix = the prior N(0, P0'), suffix = nothing) and the
// log marginal likelihood (the prior pushed through the whole chain).
template <int B>
__global__ __launch_bounds__(kW) void k_wide_root(SumDesc d, const double* __restrict__ cst,
                                                  const double* __restrict__ elems, int64_t off_root,
                                                  double* __restrict__ msgs, double* __restrict__ scal) {
  constexpr int BB = B * B;
  using Y = Lay<B>;
  __shared__ double E[Y::kEs], m0[B], P0[BB], mo[B], Po[BB], tmp[Y::kTmp];
  const int tid = threadIdx.x;
  for (int e = tid; e < Y::kEs; e += kW) E[e] = elems[off_root * Y::kEs + e];
  for (int e = tid; e < BB; e += kW) P0[e] = cst[d.kP0 + e];
  if (tid < B) m0[tid] = 0.0;
  tsync();
  double* msg = msgs + off_root * Y::kMs;
  for (int e = tid; e < Y::kMs; e += kW) {
    double v = 0.0;
    if (e >= Y::kP && e < Y::kP + BB) v = P0[e - Y::kP];
    msg[e] = v;
  }
  double dcf, dcl;
  t_prefix<B>(m0, P0, E, mo, Po, tmp, dcf, dcl);
  if (tid == 0) {
    scal[0] = dcf + dcl;
    scal[1] = dcf;
    scal[2] = dcl;
  }
}

// Down-sweep: messages of level k - 1 (n_child at off_child) from level k (at off_par).
// LEAF: the children are leaves (the left sibling a right child is pushed through is a leaf).
// Q2: and the right sibling a left child pulls back through has Q in the leading 2 x 2 block.
template <int B, bool LEAF = false, bool Q2 = false>
__global__ __launch_bounds__(kW, Occ<B>::kLevel) void k_wide_down(const double* __restrict__ elems, double* __restrict__ msgs,
                                                  int64_t off_par, int64_t off_child, int64_t n_child) {
  using Y = Lay<B>;
  constexpr int BB = B * B;
  __shared__ double par[Y::kMs], E[Y::kEs], tmp[Y::kTmpStep];
  const int tid = threadIdx.x;
  // parent message, then the sibling element (absent for an unpaired tail)
  constexpr int kAll = Y::kMs + Y::kEs;
  constexpr int NP = Ahead<B>::kOn ? (kAll + kW - 1) / kW : 1;
  double pre[NP];
  auto fetch = [&](int64_t it) {
    if (it >= n_child) return;
    const double* pm = msgs + (off_par + (it >> 1)) * Y::kMs;
    const bool lft = (it & 1) == 0;
    const bool tail = lft && it + 1 >= n_child;
    const double* sib = elems + (off_child + (lft ? it + 1 : it - 1)) * Y::kEs;
    SPG_UNROLL for (int j = 0; j < NP; ++j) {
      const int e = tid + j * kW;
      if (e < Y::kMs) pre[j] = pm[e];
      else if (e < kAll && !tail) pre[j] = sib[e - Y::kMs];
    }
  };
  if (Ahead<B>::kOn) fetch(blockIdx.x);
  for (int64_t c = blockIdx.x; c < n_child; c += gridDim.x) {
    const double* pm = msgs + (off_par + (c >> 1)) * Y::kMs;
    double* om = msgs + (off_child + c) * Y::kMs;
    const bool left = (c & 1) == 0;
    const bool tail = left && c + 1 >= n_child;   // unpaired tail: same messages as its parent
    const double* sib = elems + (off_child + (left ? c + 1 : c - 1)) * Y::kEs;
    if (Ahead<B>::kOn) {
      SPG_UNROLL for (int j = 0; j < NP; ++j) {
        const int e = tid + j * kW;
        if (e < Y::kMs) par[e] = pre[j];
        else if (e < kAll && !tail) E[e - Y::kMs] = pre[j];
      }
    } else {
      for (int e = tid; e < Y::kMs; e += kW) par[e] = pm[e];
      if (!tail)
        for (int e = tid; e < Y::kEs; e += kW) E[e] = sib[e];
    }
    tsync();
    if (Ahead<B>::kOn) fetch(c + gridDim.x);
    if (tail) {
      for (int e = tid; e < Y::kMs; e += kW) om[e] = par[e];
      tsync();
      continue;
    }
    // the new message goes straight to global memory: the half that does not change, the
    // padding, then the half the step forms
    for (int e = tid; e < B + BB; e += kW) {
      const int h = left ? e : Y::kMJ + e;
      om[h] = par[h];
    }
    for (int e = Y::kM + tid; e < Y::kMs; e += kW) om[e] = 0.0;
    if (left) {
      // prefix unchanged; suffix pulled back through the right sibling
      t_suffix<B, LEAF && Q2>(E, par + Y::kMJ, par + Y::kMeta, om + Y::kMJ, om + Y::kMeta, tmp);
    } else {
      // prefix pushed through the left sibling; suffix unchanged
      double dcf, dcl;
      t_prefix<B, LEAF>(par + Y::km, par + Y::kP, E, om + Y::km, om + Y::kP, tmp, dcf, dcl);
    }
  }
}

struct WideOut {
  double* f_mean;
  double* f_var;
  double* z_mean;
  double* S_diag;
  double* S_sub;
  int64_t ld;
  double* part;      // [gridDim.x][B*B + na + 1] per-work-group gradient partials
  const unsigned long long* status;   // the status word: a data error poisons the outputs (NaN)
};

// Node step (see the file comment).  Gradient partials per work-group: P0'_bar (B*B), the
// channel sums <A_bar, dA/dtheta> (na), d/ds2.
template <int B, int MODE>
__global__ __launch_bounds__(kW, Occ<B>::kNode) void k_wide_node(SumDesc d, const double* __restrict__ t,
                                                                 const double* __restrict__ y, int64_t n_pts,
                                                                 const double* __restrict__ cst,
                                                                 const double* __restrict__ elems,
                                                                 const double* __restrict__ msgs,
                                                                 const double* __restrict__ deriv, WideOut out) {
  constexpr int BB = B * B;
  using Y = Lay<B>;
  constexpr bool kGrad = (MODE & kWantGrad) != 0;
  constexpr bool kCov = (MODE & (kWantVar | kWantSub)) != 0;
  constexpr bool kSub = (MODE & kWantSub) != 0;
  const int kPart = BB + d.na + 1;
  __shared__ double c[Consts<B>::kNoP0o];
  __shared__ double dvs[2 * kMaxSupport];   // the edge's transition derivatives on the support
  __shared__ double E[Y::kEs], G_[Y::kMs];   // leaf element; messages (prefix at n, suffix on n + 1)
  __shared__ double mp[B], mn[B], Mx[BB], W[BB], lam[B], Lam[BB], X2[BB], mu[B], fcol[B];
  // the inverse overwrites its input (see t_inv_logdet); Mx is free again once W and lam are formed
  double* Gm = Mx;
  // the final team reduction reuses X2 (not read after the node loop) when it is large enough
  constexpr bool kRedInX2 = BB >= kW;
  __shared__ double red_[kRedInX2 ? 1 : kW];
  double* red = kRedInX2 ? X2 : red_;
  // P+, P', X1 = A P+ and X3 share one block with the scratch of the first node's suffix step
  // (t_suffix needs 2 b^2 + 2 b), which runs after their last use in that iteration
  __shared__ double quad[4 * BB];
  double *Pp = quad, *Pn = quad + BB, *X1 = quad + 2 * BB, *X3 = quad + 3 * BB, *tmp = quad;
  __shared__ TermInfo tt[kMaxTerms];
  __shared__ unsigned short sup[kMaxSupport];   // support entry s: i | j << 5 | term << 10
  const int tid = threadIdx.x;
  if (tid < d.nt) tt[tid] = d.t[tid];
  for (int e = tid; e < d.kP0 + BB; e += kW) c[e] = cst[e];   // all but the original-basis P0
  tsync();
  for (int sidx = tid; sidx < d.ns; sidx += kW) {
    int si, sj;
    const int u = support(d, tt, sidx, si, sj);
    sup[sidx] = si | (sj << 5) | (u << 10);
  }
  tsync();
  const double* P0 = c + d.kP0;
  const double s2 = c[d.kS2];
  const bool poison = *out.status != ~0ull;
  constexpr int kRows = (BB + kW - 1) / kW;
  double acc_p0[kRows], acc_s2 = 0.0;
  SPG_UNROLL for (int r = 0; r < kRows; ++r) acc_p0[r] = 0.0;
  // transition derivatives: each lane owns up to two support entries s = tid + 64 q (their
  // place and term are looked up when used), with one accumulator per channel of their term
  double acc_a[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  // the leaf element, the messages and (gradient) the edge's derivatives of node n, fetched
  // one node ahead (see Ahead)
  const int kDv = kGrad ? d.ndv : 0;
  const int kAll = Y::kEs + Y::kMs + kDv;
  // registers for the element, the messages and the first 64 or more derivative entries (the
  // rest of a larger support loads with the node itself)
  constexpr int NP = Ahead<B>::kNode ? (Y::kEs + Y::kMs + (kGrad ? kW : 0) + kW - 1) / kW : 1;
  double pre[NP];
  auto fetch = [&](int64_t it) {
    if (it >= n_pts) return;
    SPG_UNROLL for (int j = 0; j < NP; ++j) {
      const int e = tid + j * kW;
      if (e < Y::kEs) pre[j] = elems[it * Y::kEs + e];
      else if (e < Y::kEs + Y::kMs) pre[j] = msgs[it * Y::kMs + e - Y::kEs];
      else if (e < kAll) pre[j] = deriv[it * kDv + e - Y::kEs - Y::kMs];
    }
  };
  constexpr bool ahead = Ahead<B>::kNode;
  static_assert(!ahead || Y::kEs + Y::kMs <= NP * kW, "the element and the messages fit the registers");
  if (ahead) fetch(blockIdx.x);
  for (int64_t n = blockIdx.x; n < n_pts; n += gridDim.x) {
    const bool edge = n + 1 < n_pts;
    if (ahead) {
      SPG_UNROLL for (int j = 0; j < NP; ++j) {
        const int e = tid + j * kW;
        if (e < Y::kEs) E[e] = pre[j];
        else if (e < Y::kEs + Y::kMs) G_[e - Y::kEs] = pre[j];
        else if (e < kAll) dvs[e - Y::kEs - Y::kMs] = pre[j];
      }
      for (int e = NP * kW + tid; e < kAll; e += kW) dvs[e - Y::kEs - Y::kMs] = deriv[n * kDv + e - Y::kEs - Y::kMs];
    } else {
      for (int e = tid; e < Y::kEs; e += kW) E[e] = elems[n * Y::kEs + e];
      for (int e = tid; e < Y::kMs; e += kW) G_[e] = msgs[n * Y::kMs + e];
      for (int e = tid; e < kDv; e += kW) dvs[e] = deriv[n * kDv + e];
    }
    tsync();
    if (ahead) fetch(n + gridDim.x);
    const double* m = G_ + Y::km;
    const double* P = G_ + Y::kP;
    const double* A = E + Y::kA;
    // filtered state at n: K = P e0 / s, v = y - m_0
    const double yn = y[n];
    const bool obs = yn == yn;                 // NaN: a node without observation (zero gain)
    const double s = P[0] + s2, is = obs ? 1.0 / s : 0.0, v = obs ? yn - m[0] : 0.0;
    for (int e = tid; e < BB; e += kW) {
      const int i = e / B, j = e - i * B;
      Pp[e] = P[e] - P[i * B] * P[j * B] * is;
    }
    if (tid < B) mp[tid] = m[tid] + P[tid * B] * is * v;
    tsync();
    t_sym<B>(Pp);
    // predicted state at n + 1 and the suffix information on it
    const double* Js = G_ + Y::kMJ;
    const double* es = G_ + Y::kMeta;
    // predicted state m' = A m+ (b = 0 at a leaf), P' = sym(A P+ A^T) + Q; seed at n + 1:
    // Gam = (I + P' J')^-1, W = sym(J' Gam), lam = Gam^T eta' - W m', Lam
    mx_store<B>(mx<B, false, false>(A, Pp), X1);
    if (tid < B) {
      double sacc = 0.0;
      for (int k = 0; k < B; ++k) sacc = fma(A[tid * B + k], mp[k], sacc);
      mn[tid] = sacc;
    }
    tsync();
    mx_each<B>(mx_sym<B, false, true>(X1, A), [&](int i, int j, double v) { Pn[i * B + j] = v + E[Y::kQ + i * B + j]; });
    tsync();
    mx_each<B>(mx<B, false, false>(Pn, Js), [&](int i, int j, double v) { Mx[i * B + j] = v + (i == j ? 1.0 : 0.0); });
    tsync();
    (void)t_inv_logdet<B>(Mx, Gm, fcol);
    mx_store<B>(mx_sym<B, false, false>(Js, Gm), W);
    tsync();
    if (tid < B) {
      const int i = tid;
      double s1 = 0.0, s3 = 0.0;
      for (int k = 0; k < B; ++k) {
        s1 = fma(Gm[k * B + i], es[k], s1);
        s3 = fma(W[i * B + k], mn[k], s3);
      }
      lam[i] = s1 - s3;
    }
    tsync();
    for (int e = tid; e < BB; e += kW) {
      const int i = e / B, j = e - i * B;
      Lam[e] = 0.5 * (lam[i] * lam[j] - W[e]);
    }
    tsync();
    // smoothed mean mu = m+ + P+ A^T lam
    t_mtv<B>(A, lam, fcol);
    if (tid < B) {
      double sacc = mp[tid];
      for (int k = 0; k < B; ++k) sacc = fma(Pp[tid * B + k], fcol[k], sacc);
      mu[tid] = sacc;
    }
    tsync();
    // smoothed covariance S = P+ - (A P+)^T W (A P+)   (X1 = A P+)
    double S00 = 0.0;
    if (kCov) {
      t_mm<B>(W, X1, X2);                // W A P+
      t_mtm<B>(X1, X2, X3);              // (A P+)^T W A P+
      for (int e = tid; e < BB; e += kW) X3[e] = Pp[e] - X3[e];
      tsync();
      t_sym<B>(X3);
      S00 = X3[0];
    } else if (kGrad) {
      // only S_00 is needed: P+_00 - x^T W x with x = (A P+) e_0, in the order of the products
      if (tid < B) {
        double v = 0.0;
        for (int k = 0; k < B; ++k) v = fma(W[tid * B + k], X1[k * B], v);
        fcol[tid] = v;
      }
      tsync();
      double q = 0.0;
      for (int k = 0; k < B; ++k) q = fma(X1[k * B], fcol[k], q);
      S00 = Pp[0] - q;
    }
    if (out.f_mean && tid == 0) out.f_mean[n] = poison ? kPoison : mu[0];
    if (out.f_var && tid == 0) out.f_var[n] = poison ? kPoison : S00;
    if (out.z_mean && tid < B) {
      double z = mu[tid];
      if (tid == 0) for (int k = 1; k < B; ++k) z = fma(Ti_at(d, 0, k), mu[k], z);
      out.z_mean[tid * out.ld + n] = poison ? kPoison : z * c[d.kScale + tid];
    }
    if (out.S_diag || (kSub && out.S_sub && edge)) {
      // back to the original basis: S_o = T^-1 S' T^-T, S_sub_o = T^-1 S_sub' T^-T
      if (out.S_diag) {
        for (int e = tid; e < BB; e += kW) {
          const int i = e / B, j = e - i * B;
          double sacc = 0.0;
          for (int k = 0; k < B; ++k) sacc = fma(Ti_at(d, i, k), X3[k * B + j], sacc);
          X2[e] = sacc;
        }
        tsync();
        for (int e = tid; e < BB; e += kW) {
          const int i = e / B, j = e - i * B;
          if (j < i) continue;
          double sacc = 0.0;
          for (int k = 0; k < B; ++k) sacc = fma(X2[i * B + k], Ti_at(d, j, k), sacc);
          const int pk = i * B - i * (i - 1) / 2 + (j - i);     // packed upper, row-major
          out.S_diag[(int64_t)pk * out.ld + n] = poison ? kPoison : sacc * (c[d.kScale + i] * c[d.kScale + j]);
        }
        tsync();
      }
      if (kSub && out.S_sub && edge) {
        // S_sub' = (I - P' W) A P+ = X1 - Pn (W X1)
        t_mm<B>(W, X1, X2);
        t_mm<B>(Pn, X2, Mx);
        for (int e = tid; e < BB; e += kW) Mx[e] = X1[e] - Mx[e];
        tsync();
        for (int e = tid; e < BB; e += kW) {
          const int i = e / B, j = e - i * B;
          double sacc = 0.0;
          for (int k = 0; k < B; ++k) sacc = fma(Ti_at(d, i, k), Mx[k * B + j], sacc);
          X2[e] = sacc;
        }
        tsync();
        for (int e = tid; e < BB; e += kW) {
          const int i = e / B, j = e - i * B;
          double sacc = 0.0;
          for (int k = 0; k < B; ++k) sacc = fma(X2[i * B + k], Ti_at(d, j, k), sacc);
          out.S_sub[(int64_t)e * out.ld + n] = poison ? kPoison : sacc * (c[d.kScale + i] * c[d.kScale + j]);
        }
        tsync();
      }
    }
    if (kGrad) {
      // noise: E[d/ds2 log N(y; z_0, s2)] = -1/(2 s2) + ((y - mu_0)^2 + S_00) / (2 s2^2)
      if (tid == 0 && obs) {
        const double r = yn - mu[0];
        acc_s2 += -0.5 / s2 + 0.5 * (r * r + S00) / (s2 * s2);
      }
      if (edge) {
        // A_bar = lam m+^T + 2 (Lam A)(P+ - P0) into Mx, with X3 = Lam A kept for P0_bar below
        // (the smoothed covariance X3 held is written out above and not needed any more)
        t_mm<B>(Lam, A, X3);
        for (int e = tid; e < BB; e += kW) X2[e] = Pp[e] - P0[e];
        tsync();
        t_mm<B>(X3, X2, Mx);
        for (int e = tid; e < BB; e += kW) {
          const int i = e / B, j = e - i * B;
          Mx[e] = fma(lam[i], mp[j], 2.0 * Mx[e]);
        }
        tsync();
        // original basis: A_bar_o = T^T A_bar T^-T, needed only on the support of the
        // transition derivatives (each lane's own support entries)
        SPG_UNROLL for (int q = 0; q < 2; ++q) {
          const int sidx = tid + q * kW;
          if (sidx < d.ns) {
            const int sv = sup[sidx], si = sv & 31, sj = (sv >> 5) & 31;
            const TermInfo& T = tt[sv >> 10];
            const int o = T.dv0 + (sidx - T.sup0) * T.nch;
            const double ab = abar_orig<B>(d, Mx, si, sj);
            acc_a[q][0] = fma(ab, dvs[o], acc_a[q][0]);
            if (T.nch == 2) acc_a[q][1] = fma(ab, dvs[o + 1], acc_a[q][1]);
          }
        }
        // P0_bar += Lam - A^T (Lam A)
        t_mtm<B>(A, X3, X2);
        for (int e = tid, r = 0; e < BB; e += kW, ++r) acc_p0[r] += Lam[e] - X2[e];
      }
      if (n == 0) {
        // the first state is drawn from N(0, P0'): P0_bar += Lam_0, the seed of the prior
        // against all the information on node 0 (its own and the suffix pulled back).  The
        // suffix step's scratch shares its block with P+, P', A P+ and X3: the barrier orders
        // their last reads above before its first writes.
        tsync();
        t_suffix<B>(E, Js, es, X2, mn, tmp);
        t_mm<B>(P0, X2, Mx);
        t_add_eye<B>(Mx);
        (void)t_inv_logdet<B>(Mx, Gm, fcol);
        t_mm<B>(X2, Gm, W);
        t_sym<B>(W);
        t_mtv<B>(Gm, mn, lam);
        for (int e = tid, r = 0; e < BB; e += kW, ++r) {
          const int i = e / B, j = e - i * B;
          acc_p0[r] += 0.5 * (lam[i] * lam[j] - W[e]);
        }
      }
    }
    tsync();
  }
  if (kGrad) {
    // per-work-group partials: lane-owned entries of P0_bar, then the scalar sums reduced over
    // the team in a fixed order
    double* pw = out.part + (int64_t)blockIdx.x * kPart;
    for (int e = tid, r = 0; e < BB; e += kW, ++r) pw[e] = acc_p0[r];
    for (int f = 0; f <= d.na; ++f) {
      // channel f: this lane's accumulators of that channel; f = na: the noise variance
      double v = 0.0;
      if (f == d.na) {
        v = acc_s2;
      } else {
        SPG_UNROLL for (int q = 0; q < 2; ++q) {
          const int sidx = tid + q * kW;
          if (sidx < d.ns) {
            const TermInfo& T = tt[sup[sidx] >> 10];
            if (T.ch0 == f) v += acc_a[q][0];
            if (T.nch == 2 && T.ch0 + 1 == f) v += acc_a[q][1];
          }
        }
      }
      red[tid] = v;
      tsync();
      if (tid == 0) {
        double sacc = 0.0;
        for (int k = 0; k < kW; ++k) sacc += red[k];
        pw[BB + f] = sacc;
      }
      tsync();
    }
  }
}

// Sum of the per-work-group partials: work-group f adds field f over all node work-groups
// (lane-strided, then a fixed tree over the lanes), so the result is independent of timing.
template <int B>
__global__ __launch_bounds__(kW) void k_wide_sum(const double* __restrict__ part, int n_part, int kPart,
                                                 double* __restrict__ tot) {
  __shared__ double red[kW];
  const int tid = threadIdx.x, f = blockIdx.x;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  int w = tid;
  for (; w + 3 * kW < n_part; w += 4 * kW) {
    SPG_UNROLL for (int u = 0; u < 4; ++u) a[u] += part[(int64_t)(w + u * kW) * kPart + f];
  }
  for (; w < n_part; w += kW) a[0] += part[(int64_t)w * kPart + f];
  red[tid] = (a[0] + a[1]) + (a[2] + a[3]);
  tsync();
  for (int st = kW / 2; st > 0; st /= 2) {
    if (tid < st) red[tid] += red[tid + st];
    tsync();
  }
  if (tid == 0) tot[f] = red[0];
}

// Gradient with respect to the raw hyperparameters (the model's row) from the summed
// partials; also copies the log likelihood.
template <int B>
__global__ __launch_bounds__(kW) void k_wide_final(SumDesc d, const double* __restrict__ cst,
                                                   const double* __restrict__ totg,
                                                   const double* __restrict__ scal, double* __restrict__ logml,
                                                   double* __restrict__ grad,
                                                   const unsigned long long* __restrict__ status, uint32_t gmask) {
  constexpr int BB = B * B;
  const int kPart = BB + d.na + 1;
  __shared__ double c[Consts<B>::kMax], tot[BB + kMaxChannels + 1], X[BB], Pb[BB];
  __shared__ TermInfo tt[kMaxTerms];
  const int tid = threadIdx.x;
  if (tid < d.nt) tt[tid] = d.t[tid];
  for (int e = tid; e < d.kConst; e += kW) c[e] = cst[e];
  for (int e = tid; e < kPart; e += kW) tot[e] = totg[e];
  tsync();
  // P0_bar in the original basis: T^T P0'_bar T
  for (int e = tid; e < BB; e += kW) {
    const int i = e / B, j = e - i * B;
    double sacc = 0.0;
    for (int k = 0; k < B; ++k) sacc = fma(T_at(d, k, i), tot[k * B + j], sacc);
    X[e] = sacc;
  }
  tsync();
  for (int e = tid; e < BB; e += kW) {
    const int i = e / B, j = e - i * B;
    double sacc = 0.0;
    for (int k = 0; k < B; ++k) sacc = fma(X[i * B + k], T_at(d, k, j), sacc);
    Pb[e] = sacc;
  }
  tsync();
  if (tid == 0) {
    double g[3 * kMaxTerms + 2 * kMaxTerms + 1];   // at most four per term and s2
    final_grad<B>(d, tt, c, tot, Pb, g);
    // gradient components outside gmask are 0; a data error poisons everything (NaN)
    const bool poison = *status != ~0ull;
    for (int k = 0; k < d.nh; ++k) grad[k] = poison ? kPoison : (((gmask >> k) & 1u) ? g[k] : 0.0);
    if (logml) logml[0] = poison ? kPoison : scal[0];
  }
}

}  // namespace wide
}  // namespace spg
