// Kernels of the hot path: chunk fold + work-group tree (k_fwd), banded reduction of the
// work-group aggregates (k_top_bands), top-level path walk + work-group down-sweep + chunk
// elimination + adjoint sweep (k_bwd), and for several series a fixed-order per-series sum
// (k_series_reduce) plus the assemble-time chunk map.
//
// Work decomposition, R points per lane and L lanes per work-group.  A chunk is R consecutive
// nodes of one series (the last chunk of a series may be shorter); its element spans from the
// chunk's first node to the next chunk's first node.  Series are concatenated: the edge after
// the last node of a series carries A = 0 and Q = P0 of the next series (no information crosses
// it, and the next series starts from its own prior), the edge after the very last node A = 0,
// Q = 0.  Work-group g owns chunk slots [g L, (g+1) L).  The reduction tree is a sequential fold
// inside a lane (R nodes), a balanced tree over the L lanes in LDS, and a banded tree over the
// work-group aggregates.  The reverse kernel hands every chunk the predicted state (m, P) at its
// first node (prefix from the prior) and the information (J, eta) on its successor (suffix from
// the end); those seed the chunk's elimination and its adjoint sweep.
#pragma once
#include "spingp_device.hpp"

namespace spg {

// Hyperparameter row: (lengthscale, signal variance, noise variance).  Read from device memory,
// so replays of a captured launch pick up new values.
template <int B>
SPG_DEV SeriesPar load_par(const double* hyper) {
  SeriesPar p;
  p.ell = hyper[0];
  p.var = hyper[1];
  p.s2 = hyper[2];
  // lam = sqrt(2 nu) / l with nu = B - 1/2
  p.lam = (B == 1 ? 1.0 : B == 2 ? 1.7320508075688772935 : B == 3 ? 2.2360679774997896964 : 2.6457513110645905905) /
          p.ell;
  return p;
}

// Layout of several series (device arrays built by spingp_assemble); unused for one series.
struct SeriesMap {
  const int64_t* offsets;       // [S + 1] first node of every series, offsets[S] = N
  const int32_t* chunk_series;  // [slots] series of every chunk slot, -1 past the last chunk
  const int64_t* chunk_first;   // [S + 1] first chunk of every series
  int64_t slots;                // entries of chunk_series (launched chunk slots)
  int32_t n_series;
  uint32_t* bad;                // [S] nonzero for a series whose inputs failed the device checks
};

// Device-detected data errors poison the outputs they affect with NaN.  One series: any error in
// the status word (minimum of (index << 4) | code over the offending points, all ones when none)
// poisons everything; several series: the series flagged in bad, or all of them when the offsets
// themselves are invalid (code 1 in the status word).
constexpr double kPoison = __builtin_nan("");
SPG_DEV bool status_poisons_all(const unsigned long long* status, bool batched) {
  const unsigned long long st = *status;
  return st != ~0ull && (!batched || (st & 15ull) == 1ull);
}

// Hyperparameter row of the series that owns node 0 (its prior is the root of the chain): the
// series of chunk 0, which skips leading empty series.
template <bool BATCHED>
SPG_DEV const double* root_hyper(const double* __restrict__ hyper, const SeriesMap& sm) {
  if (!BATCHED) return hyper;
  const int32_t s = sm.chunk_series[0];
  return hyper + 3 * (int64_t)(s < 0 ? 0 : s);
}

// What a lane works on.
template <int B>
struct Lane {
  SeriesPar p;          // hyperparameters of the lane's series
  int64_t series;       // its index
  int64_t start;        // first node of the chunk
  int len;              // nodes in the chunk (0 for a padding slot)
  int64_t s_begin;      // first node of the series
  int64_t s_end;        // one past its last node
  bool has_next;        // another series follows (boundary edge carries its prior)
  const double* hyper_next;
  bool next_clean;      // that series passed the device checks
  bool clean;           // this series passed the device checks (several series)
};

// A series that failed the device checks is run on neutral stand-in data (times 0, 1, 2, ...
// from its first node, no observations, unit hyperparameters): its outputs are NaN anyway, and
// its non-finite values would otherwise reach the next series through the boundary edge
// (0 * NaN is NaN).
template <int B>
SPG_DEV SeriesPar neutral_par() {
  const double one[3] = {1.0, 1.0, 1.0};
  return load_par<B>(one);
}

template <int B, int R, bool BATCHED>
SPG_DEV Lane<B> lane_of(int64_t chunk, int64_t n_pts, const double* __restrict__ hyper, const SeriesMap& sm) {
  Lane<B> ln;
  if (!BATCHED) {
    ln.series = 0;
    ln.start = chunk * R;
    ln.len = ln.start < n_pts ? (int)((n_pts - ln.start) < R ? (n_pts - ln.start) : R) : 0;
    ln.s_begin = 0;
    ln.s_end = n_pts;
    ln.has_next = false;
    ln.hyper_next = hyper;
    ln.next_clean = true;
    ln.clean = true;
    ln.p = load_par<B>(hyper);
    return ln;
  }
  const int32_t s = sm.chunk_series[chunk];
  if (s < 0) {
    ln.series = 0;
    ln.start = 0;
    ln.len = 0;
    ln.s_begin = 0;
    ln.s_end = 0;
    ln.has_next = false;
    ln.hyper_next = hyper;
    ln.next_clean = true;
    ln.clean = true;
    ln.p = load_par<B>(hyper);
    return ln;
  }
  // clamped so that invalid offsets (reported by the assemble-time checks) never index outside
  // [0, n_pts); valid offsets pass through unchanged
  ln.series = s;
  const int64_t ob = sm.offsets[s], oe = sm.offsets[s + 1];
  ln.s_begin = ob < 0 ? 0 : (ob > n_pts ? n_pts : ob);
  ln.s_end = oe < ln.s_begin ? ln.s_begin : (oe > n_pts ? n_pts : oe);
  ln.start = ln.s_begin + (chunk - sm.chunk_first[s]) * R;
  if (ln.start < ln.s_begin || ln.start > ln.s_end) ln.start = ln.s_end;
  ln.len = (int)((ln.s_end - ln.start) < R ? (ln.s_end - ln.start) : R);
  // the node after the series' last one opens the next non-empty series, whose first chunk is
  // the next slot
  ln.has_next = false;
  ln.hyper_next = hyper;
  ln.next_clean = true;
  if (ln.start + ln.len == ln.s_end && chunk + 1 < sm.slots) {
    const int32_t s2 = sm.chunk_series[chunk + 1];
    if (s2 >= 0) {
      ln.has_next = true;
      ln.hyper_next = hyper + 3 * (int64_t)s2;
      ln.next_clean = sm.bad == nullptr || sm.bad[s2] == 0u;
    }
  }
  ln.clean = sm.bad == nullptr || sm.bad[s] == 0u;
  ln.p = ln.clean ? load_par<B>(hyper + 3 * (int64_t)s) : neutral_par<B>();
  return ln;
}

// Edge n -> n+1: the transition and e = exp(-lam dt) for a model edge (returns true); the
// boundary or terminal edge after a series' last node has A = 0 (returns false).
template <int B>
SPG_DEV bool edge_at(const Lane<B>& ln, const double* __restrict__ t, int64_t n, double& dt, double& e,
                     double (&A)[B][B]) {
  if (n + 1 < ln.s_end) {
    dt = ln.clean ? t[n + 1] - t[n] : 1.0;
    Matern<B>::transition(ln.p, dt, e, A);
    return true;
  }
  dt = 0.0;
  e = 0.0;
  mat_zero<B>(A);
  return false;
}

// A chunk's times (and the next node's) and observations, loaded together at the start so that
// a lane waits on memory once, not once per node.  Indices are clamped into [0, n_pts); entries
// past the chunk are never used.
template <int R>
struct ChunkData {
  double t[R + 1];
  double y[R];
};
template <int B, int R>
SPG_DEV void load_chunk(const Lane<B>& ln, const double* __restrict__ t, const double* __restrict__ y, int64_t n_pts,
                        ChunkData<R>& cd) {
  SPG_UNROLL for (int k = 0; k <= R; ++k) {
    int64_t n = ln.start + k;
    if (n > n_pts - 1) n = n_pts - 1;
    cd.t[k] = ln.clean ? t[n] : (double)(ln.start + k - ln.s_begin);
    if (k < R) cd.y[k] = ln.clean ? y[n] : kPoison;
  }
}
// edge_at for node start + k from the loaded times
template <int B, int R>
SPG_DEV bool edge_k(const Lane<B>& ln, const ChunkData<R>& cd, int k, double& dt, double& e, double (&A)[B][B]) {
  if (ln.start + k + 1 < ln.s_end) {
    dt = cd.t[k + 1] - cd.t[k];
    Matern<B>::transition(ln.p, dt, e, A);
    return true;
  }
  dt = 0.0;
  e = 0.0;
  mat_zero<B>(A);
  return false;
}

// Q - P0 after the non-model edge leaving a series: P0(next) - P0, or -P0 after the last series.
template <int B>
SPG_DEV void end_edge_D(const Lane<B>& ln, const double (&P0)[B][B], double (&D)[B][B]) {
  if (ln.has_next) {
    double Pn[B][B];
    Matern<B>::pinf(ln.next_clean ? load_par<B>(ln.hyper_next) : neutral_par<B>(), Pn);
    SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j) D[i][j] = Pn[i][j] - P0[i][j];
  } else {
    SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j) D[i][j] = -P0[i][j];
  }
}

// Sequential fold of the chunk's nodes into its element (rank-one observation information).
// Q of the running element is carried as D = Q - P0 so that Q_n = P0 - A_n P0 A_n^T is never
// formed: Q_new = A (Q - q q^T/s) A^T + Q_n  <=>  D_new = A (D - q q^T/s) A^T.
template <int B, int R>
SPG_DEV void fold_chunk(const Lane<B>& ln, const double (&P0)[B][B], const ChunkData<R>& cd, Elem<B>& E) {
  const SeriesPar& p = ln.p;
  const double is2 = 1.0 / p.s2;
  double D[B][B];
  {
    // first node: element (A_s, 0, Q_s, J, eta_s) with the node's constants
    double dt, e, A[B][B];
    const bool ok = edge_k<B, R>(ln, cd, 0, dt, e, A);
    mat_copy<B>(A, E.A);
    if (ok) {
      double T[B][B];
      mm<B>(A, P0, T);
      mmt_sym<B>(T, A, D);
      SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j) D[i][j] = -D[i][j];
    } else {
      end_edge_D<B>(ln, P0, D);
    }
    // a NaN observation marks a node without one (a prediction time merged into the chain):
    // no information, no likelihood term
    const double y0 = cd.y[0];
    const bool o0 = y0 == y0;
    mat_zero<B>(E.J);
    E.J[0][0] = o0 ? is2 : 0.0;
    SPG_UNROLL for (int i = 0; i < B; ++i) {
      E.b[i] = 0.0;
      E.eta[i] = 0.0;
    }
    E.eta[0] = o0 ? y0 * is2 : 0.0;
    E.cf = o0 ? -0.5 * y0 * y0 * is2 : 0.0;
  }
  // log-determinant part: the product of the innovation variances as mantissa and exponent
  // (one log for the chunk instead of one per node) and the number of observed nodes
  double ps = cd.y[0] == cd.y[0] ? p.s2 : 1.0;
  int pe = 0, nobs = cd.y[0] == cd.y[0] ? 1 : 0;
  SPG_UNROLL for (int k = 1; k < R; ++k) {
    if (k < ln.len) {
      const double yn = cd.y[k];
      const bool obs = yn == yn;
      double q[B];
      SPG_UNROLL for (int i = 0; i < B; ++i) q[i] = D[i][0] + P0[i][0];
      const double s = q[0] + p.s2;
      const double is = obs ? 1.0 / s : 0.0;        // no observation: zero gain
      double a[B];
      SPG_UNROLL for (int i = 0; i < B; ++i) a[i] = E.A[0][i];
      const double v = obs ? yn - E.b[0] : 0.0;
      const double vis = v * is;
      double Ap[B][B], bp[B], Dp[B][B];
      SPG_UNROLL for (int i = 0; i < B; ++i) {
        const double ki = q[i] * is;
        bp[i] = fma(ki, v, E.b[i]);
        SPG_UNROLL for (int j = 0; j < B; ++j) Ap[i][j] = fma(-ki, a[j], E.A[i][j]);
        SPG_UNROLL for (int j = i; j < B; ++j) Dp[i][j] = fma(-ki, q[j], D[i][j]);
        E.eta[i] = fma(a[i], vis, E.eta[i]);
        SPG_UNROLL for (int j = i; j < B; ++j) E.J[i][j] = fma(a[i] * is, a[j], E.J[i][j]);
      }
      SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < i; ++j) {
        Dp[i][j] = Dp[j][i];
        E.J[i][j] = E.J[j][i];
      }
      if (obs) {
        int e2;
        ps = frexp(ps * s, &e2);
        pe += e2;
        ++nobs;
      }
      E.cf += -0.5 * v * vis;
      double dt, e, A[B][B];
      const bool ok = edge_k<B, R>(ln, cd, k, dt, e, A);
      if (ok) {
        double T[B][B];
        mm<B>(A, Ap, E.A);
        mv<B>(A, bp, E.b);
        mm<B>(A, Dp, T);
        mmt_sym<B>(T, A, D);
      } else {
        mat_zero<B>(E.A);
        SPG_UNROLL for (int i = 0; i < B; ++i) E.b[i] = 0.0;
        end_edge_D<B>(ln, P0, D);
      }
    }
  }
  SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j) E.Q[i][j] = D[i][j] + P0[i][j];
  E.cl = -0.5 * ((double)nobs * kLog2Pi + log(ps) + (double)pe * 0.69314718055994530942);
}

// ---------------------------------------------------------------------------- LDS element pool
// Field-major: field f of slot i lives at pool[f * NS + i].
template <int B, int NS>
SPG_DEV void lds_store(double* pool, int i, const Elem<B>& E) {
  using Lay = ElemLayout<B>;
  SPG_UNROLL for (int r = 0; r < B; ++r) SPG_UNROLL for (int c = 0; c < B; ++c)
    pool[(Lay::kA + r * B + c) * NS + i] = E.A[r][c];
  SPG_UNROLL for (int r = 0; r < B; ++r) {
    pool[(Lay::kb + r) * NS + i] = E.b[r];
    pool[(Lay::keta + r) * NS + i] = E.eta[r];
  }
  int s = 0;
  SPG_UNROLL for (int r = 0; r < B; ++r) SPG_UNROLL for (int c = r; c < B; ++c) {
    pool[(Lay::kQ + s) * NS + i] = E.Q[r][c];
    pool[(Lay::kJ + s) * NS + i] = E.J[r][c];
    ++s;
  }
  pool[Lay::kcf * NS + i] = E.cf;
  pool[Lay::kcl * NS + i] = E.cl;
}
template <int B, int NS>
SPG_DEV void lds_load(const double* pool, int i, Elem<B>& E) {
  using Lay = ElemLayout<B>;
  SPG_UNROLL for (int r = 0; r < B; ++r) SPG_UNROLL for (int c = 0; c < B; ++c)
    E.A[r][c] = pool[(Lay::kA + r * B + c) * NS + i];
  SPG_UNROLL for (int r = 0; r < B; ++r) {
    E.b[r] = pool[(Lay::kb + r) * NS + i];
    E.eta[r] = pool[(Lay::keta + r) * NS + i];
  }
  int s = 0;
  SPG_UNROLL for (int r = 0; r < B; ++r) SPG_UNROLL for (int c = r; c < B; ++c) {
    const double q = pool[(Lay::kQ + s) * NS + i];
    const double j = pool[(Lay::kJ + s) * NS + i];
    E.Q[r][c] = E.Q[c][r] = q;
    E.J[r][c] = E.J[c][r] = j;
    ++s;
  }
  E.cf = pool[Lay::kcf * NS + i];
  E.cl = pool[Lay::kcl * NS + i];
}

// Messages: the predicted state (m, P) entering a node range and the information (J, eta) on the
// range's successor.  LDS layout per slot: m, P upper, J upper, eta.
template <int B>
struct Msg {
  double m[B];
  double P[B][B];
  double J[B][B];
  double eta[B];
};
template <int B>
constexpr int msg_fields() { return 2 * B + B * (B + 1); }
template <int B, int NS>
SPG_DEV void lds_load_msg(const double* pool, int i, Msg<B>& g) {
  int f = 0;
  SPG_UNROLL for (int r = 0; r < B; ++r) g.m[r] = pool[(f++) * NS + i];
  SPG_UNROLL for (int r = 0; r < B; ++r) SPG_UNROLL for (int c = r; c < B; ++c) {
    g.P[r][c] = g.P[c][r] = pool[(f++) * NS + i];
  }
  SPG_UNROLL for (int r = 0; r < B; ++r) SPG_UNROLL for (int c = r; c < B; ++c) {
    g.J[r][c] = g.J[c][r] = pool[(f++) * NS + i];
  }
  SPG_UNROLL for (int r = 0; r < B; ++r) g.eta[r] = pool[(f++) * NS + i];
}
template <int B, int NS>
SPG_DEV void lds_store_prefix(double* pool, int i, const double (&m)[B], const double (&P)[B][B]) {
  int f = 0;
  SPG_UNROLL for (int r = 0; r < B; ++r) pool[(f++) * NS + i] = m[r];
  SPG_UNROLL for (int r = 0; r < B; ++r) SPG_UNROLL for (int c = r; c < B; ++c) pool[(f++) * NS + i] = P[r][c];
}
template <int B, int NS>
SPG_DEV void lds_store_suffix(double* pool, int i, const double (&J)[B][B], const double (&eta)[B]) {
  int f = B + B * (B + 1) / 2;
  SPG_UNROLL for (int r = 0; r < B; ++r) SPG_UNROLL for (int c = r; c < B; ++c) pool[(f++) * NS + i] = J[r][c];
  SPG_UNROLL for (int r = 0; r < B; ++r) pool[(f++) * NS + i] = eta[r];
}

// ---------------------------------------------------------------------------- top-level tree
// The work-group aggregates are the leaves of a complete binary tree with Ltop = 2^n_levels
// leaves (n_levels = ceil log2 G, at least 1; identity elements pad it), reduced band by band
// by k_top_bands: every band spans 5 levels except possibly the last, which spans the rest.
// Level l of the tree starts at slot 2 Ltop - 2 (Ltop >> l); the reverse sweep walks it from
// the root to its own leaf.
struct TopTree {
  double* elems;          // field-major elements, leading dimension ld
  int64_t ld;             // at least 2 * Ltop slots
  int64_t G;              // real leaves (work-groups of the forward kernel)
  int64_t Ltop;           // 2^n_levels
  int n_levels;
  int n_bands;            // ceil(n_levels / 5)
  unsigned int* cnt;      // arrival counters; band b, group q at cnt[cnt_off[b] + q]
  int64_t cnt_off[8];
};
SPG_DEV int64_t top_level_off(const TopTree& T, int l) { return 2 * T.Ltop - 2 * (T.Ltop >> l); }

// ---------------------------------------------------------------------------- kernel: forward
// One lane per chunk; a work-group reduces its L lane elements with a balanced tree in LDS.
// Every element of the tree is also written to global memory (lane elements at slot i < L,
// internal nodes at slot L + level offset) so that the reverse kernel's down-sweep reuses it.
// Tree slots: level 0 = [0, L), level 1 = [L, L + L/2), ..., root = 2L - 2.
template <int B, int R, int L, bool BATCHED>
__global__ __launch_bounds__(L) void k_fwd(const double* __restrict__ t, const double* __restrict__ y,
                                            int64_t n_pts, const double* __restrict__ hyper, SeriesMap sm,
                                            double* __restrict__ tree_elems, int64_t tree_ld, TopTree top,
                                            unsigned long long* __restrict__ status) {
  constexpr int NF = ElemLayout<B>::kFields;
  __shared__ double pool[NF * L];
  const int tid = threadIdx.x;
  const int64_t chunk = (int64_t)blockIdx.x * L + tid;
  const int64_t gbase = (int64_t)blockIdx.x * (2 * L);
  const Lane<B> ln = lane_of<B, R, BATCHED>(chunk, n_pts, hyper, sm);
  if (ln.len > 0 && ln.start == ln.s_begin) {
    const SeriesPar& p = ln.p;
    if (!(isfinite(p.ell) && p.ell > 0.0 && isfinite(p.var) && p.var > 0.0 && isfinite(p.s2) && p.s2 > 0.0))
      atomicMin(status, 5ull);   // SPINGP_E_HYPER, no point index
  }
  double P0[B][B];
  Matern<B>::pinf(ln.p, P0);
  Elem<B> E;
  if (ln.len > 0) {
    ChunkData<R> cd;
    load_chunk<B, R>(ln, t, y, n_pts, cd);
    fold_chunk<B, R>(ln, P0, cd, E);
  } else {
    elem_identity<B>(E);
  }
  elem_store<B>(tree_elems, tree_ld, gbase + tid, E);
  lds_store<B, L>(pool, tid, E);
  lds_barrier();
  // each join of a level is split over two lanes on different wavefronts: lane j of the first
  // half of the work-group forms the new edge (A, b, Q), lane j of the second half the information
  // and normaliser (J, eta, cf, cl) of join j; both read the operands, then (after a barrier,
  // the forward half overwrites fields the backward half reads) write the result in place
  const bool fwd = tid < L / 2;
  const int jn = fwd ? tid : tid - L / 2;
  int off = L;   // slot offset of the level being produced
  SPG_UNROLL for (int stride = 1; stride < L; stride *= 2) {
    const int i = jn * 2 * stride;
    Elem<B> E1, E2, Rr;
    if (i < L) {
      lds_load<B, L>(pool, i, E1);
      lds_load<B, L>(pool, i + stride, E2);
    }
    lds_barrier();
    if (i < L) {
      if (fwd) elem_combine_fwd<B>(E1, E2, Rr);
      else elem_combine_bwd<B>(E1, E2, Rr);
      elem_store_half<B>(pool, L, i, Rr, fwd);
      elem_store_half<B>(tree_elems, tree_ld, gbase + off + jn, Rr, fwd);
    }
    off += L / (2 * stride);
    lds_barrier();
  }
  // this work-group's aggregate is leaf blockIdx.x of the top-level tree
  if (tid == 0) {
    lds_load<B, L>(pool, 0, E);
    elem_store<B>(top.elems, top.ld, blockIdx.x, E);
  }
}

// ---------------------------------------------------------------------------- kernel: top bands
// One 64-thread work-group per group of (up to) 32 leaves of band 0.  Each reduces its group in
// LDS and writes every node; then the last work-group of each group of band-0 groups (atomic
// ticket, no waiting) reduces band 1, and so on.  The work-group that completes the last band
// holds the root and, for one series, evaluates the log marginal likelihood (the prior N(0, P0)
// pushed through the whole chain).  Fences here only have to publish the few nodes this kernel
// writes.  (Splitting each join over two wavefronts, as k_fwd does, measured slower here: a
// band's work-group is small and the extra barrier per level costs more than it saves.)
constexpr int kTopThreads = 64;
template <int B, bool BATCHED>
__global__ __launch_bounds__(kTopThreads) void k_top_bands(const double* __restrict__ hyper, SeriesMap sm,
                                                            TopTree top, double* __restrict__ scal) {
  constexpr int NF = ElemLayout<B>::kFields;
  __shared__ double pool[NF * 32];
  __shared__ unsigned int s_ticket;
  const int tid = threadIdx.x;
  int64_t group = blockIdx.x, nb = top.G;   // nb: real nodes at the band's first level
  for (int band = 0; band < top.n_bands; ++band) {
    const int lev0 = 5 * band;
    const int bs = (top.n_levels - lev0) < 5 ? (top.n_levels - lev0) : 5;
    const int gsz = 1 << bs;
    const int64_t glo = group << bs;
    const int real = (int)((nb - glo) < gsz ? (nb - glo) : gsz);
    if (band > 0) {
      __threadfence();
      __syncthreads();
      if (tid == 0) s_ticket = atomicAdd(&top.cnt[top.cnt_off[band] + group], 1u);
      __syncthreads();
      if (s_ticket != (unsigned int)(real - 1)) return;     // not the last of its group
      __threadfence();
    }
    const int64_t off0 = top_level_off(top, lev0);
    if (tid < gsz) {
      Elem<B> Eg;
      if (tid < real) {
        elem_load<B>(top.elems, top.ld, off0 + glo + tid, Eg);
      } else {
        elem_identity<B>(Eg);
        elem_store<B>(top.elems, top.ld, off0 + glo + tid, Eg);
      }
      lds_store<B, 32>(pool, tid, Eg);
    }
    lds_barrier();
    for (int k = 0; k < bs; ++k) {
      const int stride = 1 << k;
      const int i = tid * 2 * stride;
      if (i < gsz) {
        Elem<B> E1, E2, Rr;
        lds_load<B, 32>(pool, i, E1);
        lds_load<B, 32>(pool, i + stride, E2);
        elem_combine<B>(E1, E2, Rr);
        lds_store<B, 32>(pool, i, Rr);
        elem_store<B>(top.elems, top.ld, top_level_off(top, lev0 + k + 1) + (glo >> (k + 1)) + tid, Rr);
      }
      lds_barrier();
    }
    if (band > 0 && tid == 0) top.cnt[top.cnt_off[band] + group] = 0u;   // ready for the next call
    nb = (nb + gsz - 1) >> bs;
    if (band + 1 < top.n_bands) {
      const int bn = (top.n_levels - lev0 - 5) < 5 ? (top.n_levels - lev0 - 5) : 5;
      group = group >> bn;
    }
  }
  if (!BATCHED && tid == 0) {
    const SeriesPar p = load_par<B>(hyper);
    double P0[B][B];
    Matern<B>::pinf(p, P0);
    Elem<B> Troot;
    lds_load<B, 32>(pool, 0, Troot);
    double m0[B], mo[B], Po[B][B], dcf, dcl;
    SPG_UNROLL for (int i = 0; i < B; ++i) m0[i] = 0.0;
    prefix_combine<B>(m0, P0, Troot, mo, Po, dcf, dcl);
    scal[0] = dcf + dcl;
    scal[1] = dcf;
    scal[2] = dcl;
  }
}

// ---------------------------------------------------------------------------- kernel: backward
// Output selection for the reverse sweep.
enum : int { kWantGrad = 1, kWantMean = 2, kWantVar = 4, kWantSub = 8, kWantLogml = 16 };

struct BwdOut {
  double* f_mean;   // [N] or null
  double* f_var;    // [N] or null
  double* z_mean;   // [B][ld] or null
  double* S_diag;   // [B(B+1)/2][ld] or null
  double* S_sub;    // [B*B][ld] or null (row n = Cov(z_{n+1}, z_n | y))
  int64_t ld;
  double* part;     // one series: [3][G] work-group gradient partials; several series: [5][slots]
                    // per-chunk (sum v^2/s, sum log s, d/dlengthscale, d/dvariance, d/dnoise)
  int64_t part_ld;
  const unsigned long long* status;   // the status word (outputs poisoned by data errors)
};

template <int B, int R, int L, int MODE, bool BATCHED>
__global__ __launch_bounds__(L, 2) void k_bwd(const double* __restrict__ t, const double* __restrict__ y,
                                               int64_t n_pts, const double* __restrict__ hyper, SeriesMap sm,
                                               const double* __restrict__ tree_elems, int64_t tree_ld,
                                               const TopTree top, BwdOut out) {
  // LDS holds messages only (the tree elements are read from global memory): message slot s
  // follows the work-group tree's level-major layout (level 0 at [0, L), ..., root 2L - 2).
  // Before the down-sweep the same space holds the top-level path siblings, field-major with
  // stride 32.
  constexpr int NS = 2 * L;
  constexpr int MF = msg_fields<B>();
  static_assert(MF * NS >= (ElemLayout<B>::kFields) * 32, "path siblings must fit in the message pool");
  constexpr bool kGrad = (MODE & kWantGrad) != 0;
  constexpr bool kCov = (MODE & (kWantVar | kWantSub)) != 0;
  constexpr bool kSub = (MODE & kWantSub) != 0;
  constexpr bool kLl = BATCHED && ((MODE & (kWantGrad | kWantLogml)) != 0);   // per-chunk logML
  constexpr bool kAdjoint = (MODE & (kWantGrad | kWantMean | kWantVar | kWantSub)) != 0;
  __shared__ double pool[MF * NS];
  const int tid = threadIdx.x;
  const int64_t chunk = (int64_t)blockIdx.x * L + tid;
  const Lane<B> ln = lane_of<B, R, BATCHED>(chunk, n_pts, hyper, sm);
  const SeriesPar p = ln.p;
  double P0[B][B];
  Matern<B>::pinf(p, P0);
  // outputs of a series whose inputs failed the device checks are NaN
  const bool poison = status_poisons_all(out.status, BATCHED) || (BATCHED && ln.len > 0 && sm.bad[ln.series] != 0);
  const int64_t wg = blockIdx.x;
  const int64_t gbase = wg * (2 * L);
  const int nlev = top.n_levels;
  {
    // ---- top-level path: child level l = tid holds sibling (wg >> l) ^ 1 of the path node
    if (tid < nlev) {
      Elem<B> E;
      elem_load<B>(top.elems, top.ld, top_level_off(top, tid) + ((wg >> tid) ^ 1), E);
      lds_store<B, 32>(pool, tid, E);
    }
    lds_barrier();
    // message entering this work-group, walked down the top-level tree: the prefix part
    // (predicted state from the first prior) on wave 0, the suffix part (information from the
    // end) on wave 1, one combine per level
    double m_[B], P_[B][B], J_[B][B], e_[B];
    if (tid == 0) {
      double Pr[B][B];
      const int32_t s0 = BATCHED ? sm.chunk_series[0] : 0;
      const bool root_clean = !BATCHED || s0 < 0 || sm.bad[s0] == 0u;
      Matern<B>::pinf(root_clean ? load_par<B>(root_hyper<BATCHED>(hyper, sm)) : neutral_par<B>(), Pr);
      SPG_UNROLL for (int i = 0; i < B; ++i) m_[i] = 0.0;
      mat_copy<B>(Pr, P_);
      for (int l = nlev - 1; l >= 0; --l) {
        if ((wg >> l) & 1) {
          Elem<B> Tl;
          lds_load<B, 32>(pool, l, Tl);
          double mo[B], Po[B][B], dcf, dcl;
          prefix_combine<B>(m_, P_, Tl, mo, Po, dcf, dcl);
          SPG_UNROLL for (int i = 0; i < B; ++i) m_[i] = mo[i];
          mat_copy<B>(Po, P_);
        }
      }
    }
    if (tid == L / 2) {
      mat_zero<B>(J_);
      SPG_UNROLL for (int i = 0; i < B; ++i) e_[i] = 0.0;
      for (int l = nlev - 1; l >= 0; --l) {
        if (!((wg >> l) & 1)) {
          Elem<B> Tr;
          lds_load<B, 32>(pool, l, Tr);
          double Jo[B][B], eo[B];
          suffix_combine<B>(Tr, J_, e_, Jo, eo);
          mat_copy<B>(Jo, J_);
          SPG_UNROLL for (int i = 0; i < B; ++i) e_[i] = eo[i];
        }
      }
    }
    lds_barrier();
    int off = 2 * L - 2;   // root slot: the message entering this work-group
    if (tid == 0) lds_store_prefix<B, NS>(pool, off, m_, P_);
    if (tid == L / 2) lds_store_suffix<B, NS>(pool, off, J_, e_);
    lds_barrier();
    // ---- work-group down-sweep: thread i < cnt carries the prefix of parent i into its right
    //      child, thread L/2 + i (another wavefront) the suffix of parent i into its left child;
    //      the children's elements come from the tree the forward kernel stored.  Each level's
    //      sibling element is loaded one level ahead (by the lanes i < 2 cnt that will use it),
    //      so its global-memory latency overlaps the current level's combine.
    const bool suf = tid >= L / 2;
    const int i = suf ? tid - L / 2 : tid;
    Elem<B> Tc;   // this lane's sibling element of the current level
    if (i < 1) elem_load<B>(tree_elems, tree_ld, gbase + (off - 2) + 2 * i + (suf ? 1 : 0), Tc);
    SPG_UNROLL for (int cnt = 1; cnt < L; cnt *= 2) {
      const int ncnt = cnt * 2, noff = off - ncnt;
      Elem<B> Tn;
      if (ncnt < L && i < ncnt)
        elem_load<B>(tree_elems, tree_ld, gbase + (noff - 2 * ncnt) + 2 * i + (suf ? 1 : 0), Tn);
      if (i < cnt) {
        Msg<B> par;
        lds_load_msg<B, NS>(pool, off + i, par);
        if (!suf) {
          double mo[B], Po[B][B], dcf, dcl;
          prefix_combine<B>(par.m, par.P, Tc, mo, Po, dcf, dcl);
          lds_store_prefix<B, NS>(pool, noff + 2 * i, par.m, par.P);
          lds_store_prefix<B, NS>(pool, noff + 2 * i + 1, mo, Po);
        } else {
          double Jo[B][B], eo[B];
          suffix_combine<B>(Tc, par.J, par.eta, Jo, eo);
          lds_store_suffix<B, NS>(pool, noff + 2 * i + 1, par.J, par.eta);
          lds_store_suffix<B, NS>(pool, noff + 2 * i, Jo, eo);
        }
      }
      lds_barrier();
      if (ncnt < L) Tc = Tn;
      off = noff;
    }
  }
  Msg<B> g;
  lds_load_msg<B, NS>(pool, tid, g);
  // the message pool is free from here on: it keeps the predicted states of the chunk's first
  // KL nodes (the rest stay in registers), field f of node k of this lane at
  // pool[(k NPS + f) L + tid]
  constexpr int NPS = B + B * (B + 1) / 2;
  constexpr int KL = R / 2 < 4 ? R / 2 : 4;
  static_assert(KL * NPS * L <= MF * NS, "predicted states must fit in the message pool");
  if (KL > 0) lds_barrier();

  // ---- chunk elimination (natural order) from the exact predicted state at its first node
  const int64_t start = ln.start;
  const int len = ln.len;
  ChunkData<R> cd;
  load_chunk<B, R>(ln, t, y, n_pts, cd);
  double sm_[R][B];                  // predicted means (nodes k >= KL)
  double sD[R][B * (B + 1) / 2];     // predicted covariances minus P0, packed upper (k >= KL)
  double m[B], D[B][B];
  double fit_chunk = 0.0;  // sum over the chunk of v_n^2 / s_n
  double ldet_chunk = 0.0; // sum over the chunk of log s_n
  SPG_UNROLL for (int i = 0; i < B; ++i) {
    m[i] = g.m[i];
    SPG_UNROLL for (int j = 0; j < B; ++j) D[i][j] = g.P[i][j] - P0[i][j];
  }
  SPG_UNROLL for (int k = 0; k < R; ++k) {
    if (k < len) {
      const int64_t n = start + k;
      if (k < KL) {
        SPG_UNROLL for (int i = 0; i < B; ++i) pool[(k * NPS + i) * L + tid] = m[i];
        int f = B;
        SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = i; j < B; ++j)
          pool[(k * NPS + f++) * L + tid] = D[i][j];
      } else {
        SPG_UNROLL for (int i = 0; i < B; ++i) {
          sm_[k][i] = m[i];
          SPG_UNROLL for (int j = i; j < B; ++j) sD[k][i * B - i * (i - 1) / 2 + (j - i)] = D[i][j];
        }
      }
      double u[B];
      SPG_UNROLL for (int i = 0; i < B; ++i) u[i] = D[i][0] + P0[i][0];
      const double yk = cd.y[k];
      const bool obs = yk == yk;                    // NaN: a node without observation
      const double s = u[0] + p.s2, is = obs ? 1.0 / s : 0.0;
      const double v = obs ? yk - m[0] : 0.0;
      if (kLl && obs) {
        fit_chunk = fma(v * v, is, fit_chunk);
        ldet_chunk += log(s);
      }
      double mp[B], Dp[B][B];
      SPG_UNROLL for (int i = 0; i < B; ++i) {
        mp[i] = fma(u[i] * is, v, m[i]);
        SPG_UNROLL for (int j = 0; j < B; ++j) Dp[i][j] = fma(-u[i] * is, u[j], D[i][j]);
      }
      double A[B][B], dt_, e_;
      const bool ok = edge_k<B, R>(ln, cd, k, dt_, e_, A);
      if (ok) {
        double T[B][B];
        mv<B>(A, mp, m);
        mm<B>(A, Dp, T);
        mmt_sym<B>(T, A, D);
      } else {
        SPG_UNROLL for (int i = 0; i < B; ++i) m[i] = 0.0;
        end_edge_D<B>(ln, P0, D);
      }
    }
  }
  double gr[3] = {0.0, 0.0, 0.0};
  if (kAdjoint) {
    // ---- adjoint seed at the successor of the chunk's last node:
    //      L_rest(m, P) = log int N(z; m, P) exp(-1/2 z^T Jb z + etab^T z) dz
    //      dL/dm = Gam^T etab - W m,  dL/dP = 1/2 (lam lam^T - W),  Gam = (I + P Jb)^-1,
    //      W = Jb Gam; the smoothing information Lhat = lam lam^T - 2 dL/dP is W itself.  (After
    //      a series' last node the edge has A = 0, so nothing of this seed reaches the series.)
    double lam[B], Lam[B][B], Lhat[B][B], Pn[B][B];
    {
      SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j) Pn[i][j] = D[i][j] + P0[i][j];
      double M[B][B], Gm[B][B], W[B][B], Gte[B], Wm[B];
      mm<B>(Pn, g.J, M);
      SPG_UNROLL for (int i = 0; i < B; ++i) M[i][i] += 1.0;
      (void)inv_logdet<B>(M, Gm);
      mm<B>(g.J, Gm, W);
      symmetrize<B>(W);
      mtv<B>(Gm, g.eta, Gte);
      mv<B>(W, m, Wm);
      SPG_UNROLL for (int i = 0; i < B; ++i) lam[i] = Gte[i] - Wm[i];
      SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j) {
        Lam[i][j] = 0.5 * (lam[i] * lam[j] - W[i][j]);
        Lhat[i][j] = W[i][j];
      }
    }
    // ---- reverse sweep.  Per node n (newest first): prediction adjoint through edge n,
    //      smoothed moments from the filtered state, then the update adjoint.  lam/Lam
    //      (gradient) follow reverse-mode differentiation of the elimination; Lhat
    //      (covariances) follows the modified Bryson-Frazier recursion
    //      Lhat_n = (I - K h^T)^T A^T Lhat_{n+1} A (I - K h^T) + h h^T / s,
    //      which avoids forming lam lam^T - 2 Lam.
    double gl_lam = 0.0, g_s2 = 0.0;   // <A_bar, dA/dlam> summed, d/d s2
    double Pb[B][B];                   // adjoint of P0
    mat_zero<B>(Pb);
    SPG_UNROLL for (int k = R - 1; k >= 0; --k) {
      if (k < len) {
        const int64_t n = start + k;
        double mk[B], Dk[B][B];
        if (k < KL) {
          SPG_UNROLL for (int i = 0; i < B; ++i) mk[i] = pool[(k * NPS + i) * L + tid];
          int f = B;
          SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = i; j < B; ++j) {
            Dk[i][j] = pool[(k * NPS + f++) * L + tid];
            Dk[j][i] = Dk[i][j];
          }
        } else {
          SPG_UNROLL for (int i = 0; i < B; ++i) {
            mk[i] = sm_[k][i];
            SPG_UNROLL for (int j = 0; j < B; ++j)
              Dk[i][j] = sD[k][i <= j ? i * B - i * (i - 1) / 2 + (j - i) : j * B - j * (j - 1) / 2 + (i - j)];
          }
        }
        double u[B];
        SPG_UNROLL for (int i = 0; i < B; ++i) u[i] = Dk[i][0] + P0[i][0];
        const double yk = ln.clean ? y[n] : kPoison;
        const bool obs = yk == yk;
        const double s = u[0] + p.s2, is = obs ? 1.0 / s : 0.0;
        // t and y re-read here (cache-resident) rather than kept live across the sweep: the
        // registers are worth more than the loads
        const double v = obs ? yk - mk[0] : 0.0;
        double mp[B], Dp[B][B];
        SPG_UNROLL for (int i = 0; i < B; ++i) {
          mp[i] = fma(u[i] * is, v, mk[i]);
          SPG_UNROLL for (int j = 0; j < B; ++j) Dp[i][j] = fma(-u[i] * is, u[j], Dk[i][j]);
        }
        // prediction adjoint through edge n (nothing flows through the edge leaving a series)
        double mbp[B], Pbp[B][B], Lhp[B][B];
        double A[B][B], dt, e;
        const bool edge_ok = edge_at<B>(ln, t, n, dt, e, A);   // recomputed: cheaper than keeping it live
        if (edge_ok) {
          mtv<B>(A, lam, mbp);            // A^T lam'
          if (kGrad) {
            double T[B][B], TD[B][B], Ab[B][B];
            mm<B>(Lam, A, T);             // Lam' A
            mtm_sym<B>(A, T, Pbp);        // A^T Lam' A
            mm<B>(T, Dp, TD);
            // A_bar = lam' m+^T + 2 Lam' A (P+ - P0): the A-dependence of Q = P0 - A P0 A^T included
            SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j)
              Ab[i][j] = fma(lam[i], mp[j], 2.0 * TD[i][j]);
            gl_lam += Matern<B>::dA_dlam_dot(p, dt, e, Ab);
            SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j)
              Pb[i][j] += Lam[i][j] - Pbp[i][j];
          }
          if (kCov) {
            double T[B][B];
            mm<B>(Lhat, A, T);
            mtm_sym<B>(A, T, Lhp);        // A^T Lhat' A
          }
        } else {
          SPG_UNROLL for (int i = 0; i < B; ++i) {
            mbp[i] = 0.0;
            SPG_UNROLL for (int j = 0; j < B; ++j) {
              Pbp[i][j] = 0.0;
              Lhp[i][j] = 0.0;
            }
          }
        }
        // smoothed moments of node n from the filtered state (m+, P+):
        //   mu = m+ + P+ A^T lam',   S = P+ - P+ (A^T Lhat' A) P+,
        //   Cov(z_{n+1}, z_n | y) = (I - P_{n+1} Lhat_{n+1}) A P+
        if (MODE & (kWantMean | kWantVar | kWantSub)) {
          double Ppl[B][B], Pl[B], mu[B];
          SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j) Ppl[i][j] = Dp[i][j] + P0[i][j];
          mv<B>(Ppl, mbp, Pl);
          SPG_UNROLL for (int i = 0; i < B; ++i) mu[i] = mp[i] + Pl[i];
          if (out.f_mean) out.f_mean[n] = poison ? kPoison : mu[0];
          if (out.z_mean)
            SPG_UNROLL for (int i = 0; i < B; ++i) out.z_mean[(int64_t)i * out.ld + n] = poison ? kPoison : mu[i];
          if (kCov) {
            double X[B][B], S[B][B];
            mm<B>(Ppl, Lhp, X);
            mmt_sym<B>(X, Ppl, S);
            SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j) S[i][j] = Ppl[i][j] - S[i][j];
            if (out.f_var) out.f_var[n] = poison ? kPoison : S[0][0];
            if (out.S_diag) {
              int s_ = 0;
              SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = i; j < B; ++j)
                out.S_diag[(int64_t)(s_++) * out.ld + n] = poison ? kPoison : S[i][j];
            }
            if (kSub && edge_ok && out.S_sub) {
              double Y[B][B], AP[B][B], Ssub[B][B];
              mm<B>(Pn, Lhat, Y);
              SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j)
                Y[i][j] = (i == j ? 1.0 : 0.0) - Y[i][j];
              mm<B>(A, Ppl, AP);
              mm<B>(Y, AP, Ssub);
              SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j)
                out.S_sub[(int64_t)(i * B + j) * out.ld + n] = poison ? kPoison : Ssub[i][j];
            }
          }
        }
        // update adjoint at node n (h = e_0): adjoints of the predicted state (m_n, P_n)
        const double kl = dot<B>(u, mbp) * is;      // K^T lam+
        const double vbar = kl - v * is;
        if (kGrad) {
          double w[B];
          mv<B>(Pbp, u, w);
          const double uw = dot<B>(u, w);
          const double sbar = (uw - kl * s * v) * is * is - 0.5 * is + 0.5 * v * v * is * is;
          SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j) Lam[i][j] = Pbp[i][j];
          Lam[0][0] += sbar;
          SPG_UNROLL for (int i = 0; i < B; ++i) {
            const double ub = (mbp[i] * v - 2.0 * w[i]) * is;
            Lam[0][i] += 0.5 * ub;
            Lam[i][0] += 0.5 * ub;
          }
          g_s2 += sbar;
        }
        if (kCov) {
          // Lhat = (I - K e0^T)^T Lhp (I - K e0^T) + e0 e0^T / s,  K = u / s
          double Lk[B], Y[B][B];
          SPG_UNROLL for (int i = 0; i < B; ++i) {
            double t_ = 0.0;
            SPG_UNROLL for (int j = 0; j < B; ++j) t_ = fma(Lhp[i][j], u[j], t_);
            Lk[i] = t_ * is;                         // Lhp K
          }
          SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j) Y[i][j] = Lhp[i][j];
          SPG_UNROLL for (int i = 0; i < B; ++i) Y[i][0] -= Lk[i];          // Lhp (I - K e0^T)
          double KY[B];
          SPG_UNROLL for (int j = 0; j < B; ++j) {
            double t_ = 0.0;
            SPG_UNROLL for (int i = 0; i < B; ++i) t_ = fma(u[i], Y[i][j], t_);
            KY[j] = t_ * is;                         // K^T Y
          }
          SPG_UNROLL for (int j = 0; j < B; ++j) Y[0][j] -= KY[j];
          Y[0][0] += is;
          SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = i; j < B; ++j) {
            Lhat[i][j] = 0.5 * (Y[i][j] + Y[j][i]);
            Lhat[j][i] = Lhat[i][j];
          }
          if (kSub) SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j) Pn[i][j] = Dk[i][j] + P0[i][j];
        }
        SPG_UNROLL for (int i = 0; i < B; ++i) lam[i] = mbp[i];
        lam[0] -= vbar;
        // the first node of the series is drawn from the prior N(0, P0)
        if (kGrad && n == ln.s_begin) {
          SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j) Pb[i][j] += Lam[i][j];
        }
      }
    }
    if (kGrad) {
      double dP[B][B];
      Matern<B>::dpinf_dlam(p, dP);
      const double dlam_dell = -p.lam / p.ell;
      gr[0] = (gl_lam + frob<B>(Pb, dP)) * dlam_dell;
      gr[1] = frob<B>(Pb, P0) / p.var;
      gr[2] = g_s2;
    }
  }
  if (BATCHED) {
    // ---- per-chunk partials; k_series_reduce sums them per series in a fixed order
    if (kLl) {
      out.part[chunk] = fit_chunk;
      out.part[out.part_ld + chunk] = ldet_chunk;
    }
    if (kGrad) SPG_UNROLL for (int c = 0; c < 3; ++c) out.part[(int64_t)(c + 2) * out.part_ld + chunk] = gr[c];
  } else if (kGrad) {
    // ---- one series: fixed-order work-group reduction of the gradient partials (reuses the
    //      pool); k_grad_finish sums the work-group partials in a fixed order.  No cross-work-
    //      group signalling here: an agent-scope fence per work-group (an L2 write-back on this
    //      GPU) measured 2 to 14 us slower than the separate launch.
    lds_barrier();
    SPG_UNROLL for (int c = 0; c < 3; ++c) pool[c * L + tid] = gr[c];
    lds_barrier();
    SPG_UNROLL for (int stride = L / 2; stride > 0; stride /= 2) {
      if (tid < stride) {
        SPG_UNROLL for (int c = 0; c < 3; ++c) pool[c * L + tid] += pool[c * L + tid + stride];
      }
      lds_barrier();
    }
    if (tid == 0) SPG_UNROLL for (int c = 0; c < 3; ++c) out.part[c * out.part_ld + blockIdx.x] = pool[c * L];
  }
}

// ---------------------------------------------------------------------------- diagnostics
// Materialised blocks (not used by the hot path, which never forms them).  Per node n of a
// series [s, e):  A_n = expm(F dt_n) and Q_n = P0 - A_n P0 A_n^T for the edge n -> n+1 (zero at
// the series' last node), and the multiplied-out blocks of the posterior precision (Theorem 1)
//   D_n = J + [n = s] P0^-1 + [n > s] Q_{n-1}^-1 + [n < e-1] A_n^T Q_n^-1 A_n,
//   B_n = K_{n+1,n} = -Q_n^-1 A_n            (zero at the series' last node).
// They need Q^-1, so they are only meaningful where every Q_n is well conditioned (no
// duplicate or near-duplicate times).  One lane per chunk, its R nodes in turn.  Layout: A and
// B_n row-major [B*B][ld], Q and D packed upper [B(B+1)/2][ld]; any output may be null.
template <int B, int R, bool BATCHED>
__global__ __launch_bounds__(128) void k_blocks(const double* __restrict__ t, int64_t n_pts,
                                                const double* __restrict__ hyper, SeriesMap sm, int64_t slots,
                                                double* __restrict__ Ao, double* __restrict__ Qo,
                                                double* __restrict__ Do, double* __restrict__ Bo, int64_t ld) {
  const int64_t chunk = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (chunk >= slots) return;
  const Lane<B> ln = lane_of<B, R, BATCHED>(chunk, n_pts, hyper, sm);
  if (ln.len == 0) return;
  double P0[B][B], Pi[B][B];
  Matern<B>::pinf(ln.p, P0);
  (void)inv_logdet<B>(P0, Pi);
  const double is2 = 1.0 / ln.p.s2;
  // Q^-1 of the edge entering the chunk's first node (if it is not the series' first node)
  double Qprev_i[B][B];
  mat_zero<B>(Qprev_i);
  if (ln.start > ln.s_begin) {
    double dt, e, A[B][B], T[B][B], Q[B][B];
    dt = t[ln.start] - t[ln.start - 1];
    Matern<B>::transition(ln.p, dt, e, A);
    mm<B>(A, P0, T);
    mmt_sym<B>(T, A, Q);
    SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j) Q[i][j] = P0[i][j] - Q[i][j];
    (void)inv_logdet<B>(Q, Qprev_i);
  }
  SPG_UNROLL for (int k = 0; k < R; ++k) {
    if (k < ln.len) {
      const int64_t n = ln.start + k;
      double A[B][B], Q[B][B], Qi[B][B], D[B][B], Bn[B][B];
      double dt, e;
      const bool edge = edge_at<B>(ln, t, n, dt, e, A);
      if (edge) {
        double T[B][B];
        mm<B>(A, P0, T);
        mmt_sym<B>(T, A, Q);
        SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j) Q[i][j] = P0[i][j] - Q[i][j];
        (void)inv_logdet<B>(Q, Qi);
        symmetrize<B>(Qi);
        mm<B>(Qi, A, T);
        SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j) Bn[i][j] = -T[i][j];
        mtm_sym<B>(A, T, D);                  // A^T Q^-1 A
      } else {
        mat_zero<B>(Q);
        mat_zero<B>(Qi);
        mat_zero<B>(Bn);
        mat_zero<B>(D);
      }
      const bool first = n == ln.s_begin;
      SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j)
        D[i][j] += first ? Pi[i][j] : Qprev_i[i][j];
      D[0][0] += is2;
      int pk = 0;
      SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = i; j < B; ++j) {
        if (Qo) Qo[(int64_t)pk * ld + n] = Q[i][j];
        if (Do) Do[(int64_t)pk * ld + n] = 0.5 * (D[i][j] + D[j][i]);
        ++pk;
      }
      SPG_UNROLL for (int i = 0; i < B; ++i) SPG_UNROLL for (int j = 0; j < B; ++j) {
        if (Ao) Ao[(int64_t)(i * B + j) * ld + n] = A[i][j];
        if (Bo) Bo[(int64_t)(i * B + j) * ld + n] = Bn[i][j];
      }
      mat_copy<B>(Qi, Qprev_i);
    }
  }
}

// ---------------------------------------------------------------------------- several series
// Device-side validation of several series, one thread per chunk slot: finite t and y, t
// non-decreasing inside each series.  key = (index << 4) | code, minimised over offending points.
template <int R>
__global__ void k_validate_chunks(const double* __restrict__ t, const double* __restrict__ y, int64_t n_pts,
                                  const double* __restrict__ hyper, SeriesMap sm,
                                  unsigned long long* __restrict__ key) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < sm.n_series) {
    for (int k = 0; k < 3; ++k) {
      const double h = hyper[3 * c + k];
      if (!(isfinite(h) && h > 0.0)) {
        atomicMin(key, 5ull);                                              // SPINGP_E_HYPER
        sm.bad[c] = 1u;
      }
    }
  }
  if (c >= sm.slots) return;
  const Lane<2> ln = lane_of<2, R, true>(c, n_pts, hyper, sm);
  for (int k = 0; k < ln.len; ++k) {
    const int64_t n = ln.start + k;
    unsigned long long code = 0;
    if (!isfinite(t[n]) || !isfinite(y[n])) code = 4;                      // SPINGP_E_NONFINITE
    else if (n + 1 < ln.s_end && t[n + 1] < t[n]) code = 3;               // SPINGP_E_UNSORTED
    if (code) {
      atomicMin(key, ((unsigned long long)(n + 1) << 4) | code);
      sm.bad[ln.series] = 1u;
      return;
    }
  }
}

}  // namespace spg
