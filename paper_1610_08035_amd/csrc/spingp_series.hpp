// Kernels that do not depend on the tile shape: the chunk map of several series built at
// assemble time, and the fixed-order sums of the reverse kernel's partials (per series, or over
// the work-groups of one series).  Included by the C-ABI translation unit only.
#pragma once

#include "spingp_kernels.hpp"

namespace spg {

// One series: sum of the G work-group gradient partials in a fixed order (lane-strided, then a
// fixed tree), and the log likelihood from the root of the reduction.  Gradient components
// outside gmask are 0; after a data error (status word set) both outputs are NaN.
__global__ __launch_bounds__(256) void k_grad_finish(const double* __restrict__ part, int64_t part_ld, int64_t G,
                                                      const double* __restrict__ scal, double* __restrict__ logml,
                                                      double* __restrict__ grad,
                                                      const unsigned long long* __restrict__ status, uint32_t gmask) {
  __shared__ double red[3][256];
  const int tid = threadIdx.x;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t i = tid; i < G; i += 256) {
    SPG_UNROLL for (int c = 0; c < 3; ++c) acc[c] += part[c * part_ld + i];
  }
  SPG_UNROLL for (int c = 0; c < 3; ++c) red[c][tid] = acc[c];
  __syncthreads();
  for (int stride = 128; stride > 0; stride /= 2) {
    if (tid < stride) SPG_UNROLL for (int c = 0; c < 3; ++c) red[c][tid] += red[c][tid + stride];
    __syncthreads();
  }
  if (tid == 0) {
    const bool poison = *status != ~0ull;
    if (grad) SPG_UNROLL for (int c = 0; c < 3; ++c) grad[c] = poison ? kPoison : (((gmask >> c) & 1u) ? red[c][0] : 0.0);
    if (logml) logml[0] = poison ? kPoison : scal[0];
  }
}

// Fixed-order per-series sum of the per-chunk partials: one 64-lane work-group per series; lane i
// adds chunks first + i, first + i + 64, ... in order, then a fixed tree over the lanes.  Writes
// logml[s] (eq. ml2), and datafit[s] = y^T K_y^-1 y, logdet[s] = log det K_y, grad[s][0..2] where
// not null.  An empty series gets logml 0 and a zero gradient.  Gradient components outside gmask
// are 0; the outputs of a series whose inputs failed the device checks are NaN.
__global__ __launch_bounds__(64) void k_series_reduce(SeriesMap sm, const double* __restrict__ part,
                                                       int64_t part_ld, int64_t n_pts, double* __restrict__ logml,
                                                       double* __restrict__ datafit, double* __restrict__ logdet,
                                                       double* __restrict__ grad,
                                                       const unsigned long long* __restrict__ status, uint32_t gmask) {
  __shared__ double red[5][64];
  const int tid = threadIdx.x;
  const int64_t s = blockIdx.x;
  const int64_t c0 = sm.chunk_first[s];
  const int64_t c1 = sm.chunk_first[s + 1] < sm.slots ? sm.chunk_first[s + 1] : sm.slots;
  const int nf = grad ? 5 : 2;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t c = c0 + tid; c < c1; c += 64) {
    for (int f = 0; f < nf; ++f) acc[f] += part[f * part_ld + c];
  }
  for (int f = 0; f < 5; ++f) red[f][tid] = acc[f];
  __syncthreads();
  for (int stride = 32; stride > 0; stride /= 2) {
    if (tid < stride) for (int f = 0; f < 5; ++f) red[f][tid] += red[f][tid + stride];
    __syncthreads();
  }
  if (tid == 0) {
    const int64_t ob = sm.offsets[s], oe = sm.offsets[s + 1];
    const double ns = (oe > ob && ob >= 0 && oe <= n_pts) ? (double)(oe - ob) : 0.0;
    const double fit = red[0][0], ld = red[1][0];
    const bool bad = status_poisons_all(status, true) || sm.bad[s] != 0;
    if (logml) logml[s] = bad ? kPoison : -0.5 * fit - 0.5 * ld - 0.5 * ns * kLog2Pi;
    if (datafit) datafit[s] = bad ? kPoison : fit;
    if (logdet) logdet[s] = bad ? kPoison : ld;
    if (grad)
      for (int f = 0; f < 3; ++f) grad[s * 3 + f] = bad ? kPoison : (((gmask >> f) & 1u) ? red[f + 2][0] : 0.0);
  }
}

// Chunk map of several series (built once per assemble).  Chunks per series c_s = ceil(len_s / R);
// chunk_first is their exclusive prefix sum (one work-group, carried across blocks of 256).
__global__ __launch_bounds__(256) void k_chunk_first(const int64_t* __restrict__ offsets, int32_t n_series,
                                                      int64_t n_pts, int R, int64_t* __restrict__ chunk_first,
                                                      unsigned long long* __restrict__ status) {
  __shared__ int64_t sc[256];
  __shared__ int64_t carry;
  const int tid = threadIdx.x;
  if (tid == 0) {
    carry = 0;
    if (offsets[0] != 0 || offsets[n_series] != n_pts) atomicMin(status, 1ull);   // SPINGP_E_INVALID
  }
  __syncthreads();
  for (int64_t base = 0; base < n_series; base += 256) {
    const int64_t s = base + tid;
    int64_t c = 0;
    if (s < n_series) {
      const int64_t len = offsets[s + 1] - offsets[s];
      if (len < 0) atomicMin(status, 1ull);            // decreasing offsets
      c = len > 0 ? (len + R - 1) / R : 0;
    }
    sc[tid] = c;
    __syncthreads();
    for (int d = 1; d < 256; d *= 2) {                 // inclusive scan
      const int64_t v = tid >= d ? sc[tid - d] : 0;
      __syncthreads();
      sc[tid] += v;
      __syncthreads();
    }
    if (s < n_series) chunk_first[s] = carry + sc[tid] - c;
    __syncthreads();
    if (tid == 255) carry += sc[255];
    __syncthreads();
  }
  if (tid == 0) chunk_first[n_series] = carry;
}

// chunk_series: -1 everywhere, then the series of every chunk.
__global__ void k_chunk_fill(int32_t* __restrict__ chunk_series, int64_t slots) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < slots) chunk_series[i] = -1;
}
__global__ void k_chunk_map(const int64_t* __restrict__ chunk_first, int32_t n_series, int64_t slots,
                            int32_t* __restrict__ chunk_series) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_series) return;
  const int64_t c1 = chunk_first[s + 1] < slots ? chunk_first[s + 1] : slots;
  for (int64_t c = chunk_first[s]; c < c1; ++c) chunk_series[c] = (int32_t)s;
}

// ---------------------------------------------------------------------------- prediction
// Prediction times t* are merged into the chain as nodes without an observation (NaN in the
// merged y).  Order: a training point precedes a prediction time equal to it.  With both
// arrays sorted the merged positions are a permutation of [0, n + m); with t* unsorted (an
// error reported through the status word) they stay inside [0, n + m).
SPG_DEV int64_t count_less(const double* __restrict__ a, int64_t n, double x) {
  int64_t lo = 0, hi = n;           // first index with a[i] >= x
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}
SPG_DEV int64_t count_not_greater(const double* __restrict__ a, int64_t n, double x) {
  int64_t lo = 0, hi = n;           // first index with a[i] > x
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] <= x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ void k_merge(const double* __restrict__ t, const double* __restrict__ y, int64_t n,
                        const double* __restrict__ ts, int64_t m, double* __restrict__ tm,
                        double* __restrict__ ym) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n) {
    const int64_t pos = idx + count_less(ts, m, t[idx]);
    tm[pos] = t[idx];
    ym[pos] = y[idx];
  } else if (idx < n + m) {
    const int64_t j = idx - n;
    const int64_t pos = j + count_not_greater(t, n, ts[j]);
    tm[pos] = ts[j];
    ym[pos] = __builtin_nan("");
  }
}

// Prediction times must be finite and non-decreasing: key = (index << 4) | code as elsewhere,
// the index counted in t*.
__global__ void k_validate_star(const double* __restrict__ ts, int64_t m, unsigned long long* __restrict__ key) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  unsigned long long code = 0;
  if (!isfinite(ts[j])) code = 4;                       // SPINGP_E_NONFINITE
  else if (j + 1 < m && ts[j + 1] < ts[j]) code = 3;    // SPINGP_E_UNSORTED
  if (code) atomicMin(key, ((unsigned long long)(j + 1) << 4) | code);
}

// Several series: series s holds training points [off[s], off[s+1]) and prediction times
// [os[s], os[s+1]); both merge into [mo[s], mo[s+1]) with mo = off + os.  Indices are clamped so
// that offsets reported invalid by the status word never reach outside the arrays.
SPG_DEV int32_t series_of(const int64_t* __restrict__ off, int32_t S, int64_t i) {
  int32_t lo = 0, hi = S - 1;       // the last s with off[s] <= i
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}
SPG_DEV void clamp_range(const int64_t* __restrict__ off, int32_t s, int64_t n, int64_t& a, int64_t& e) {
  a = off[s];
  e = off[s + 1];
  a = a < 0 ? 0 : (a > n ? n : a);
  e = e < a ? a : (e > n ? n : e);
}

__global__ void k_merged_offsets(const int64_t* __restrict__ off, const int64_t* __restrict__ os, int32_t S,
                                 int64_t* __restrict__ mo) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s <= S) mo[s] = off[s] + os[s];
}

SPG_DEV int64_t merged_pos_train(const double* __restrict__ t, const int64_t* __restrict__ off,
                                 const double* __restrict__ ts, const int64_t* __restrict__ os, int32_t S,
                                 int64_t n, int64_t m, int64_t i) {
  const int32_t s = series_of(off, S, i);
  int64_t a, e, as, es;
  clamp_range(off, s, n, a, e);
  clamp_range(os, s, m, as, es);
  int64_t pos = a + as + (i - a) + count_less(ts + as, es - as, t[i]);
  return pos < 0 ? 0 : (pos > n + m - 1 ? n + m - 1 : pos);
}
SPG_DEV int64_t merged_pos_star(const double* __restrict__ t, const int64_t* __restrict__ off,
                                const double* __restrict__ ts, const int64_t* __restrict__ os, int32_t S,
                                int64_t n, int64_t m, int64_t j) {
  const int32_t s = series_of(os, S, j);
  int64_t a, e, as, es;
  clamp_range(off, s, n, a, e);
  clamp_range(os, s, m, as, es);
  int64_t pos = a + as + (j - as) + count_not_greater(t + a, e - a, ts[j]);
  return pos < 0 ? 0 : (pos > n + m - 1 ? n + m - 1 : pos);
}

__global__ void k_merge_batch(const double* __restrict__ t, const double* __restrict__ y,
                              const int64_t* __restrict__ off, int32_t S, int64_t n, const double* __restrict__ ts,
                              const int64_t* __restrict__ os, int64_t m, double* __restrict__ tm,
                              double* __restrict__ ym) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n) {
    const int64_t pos = merged_pos_train(t, off, ts, os, S, n, m, idx);
    tm[pos] = t[idx];
    ym[pos] = y[idx];
  } else if (idx < n + m) {
    const int64_t j = idx - n;
    const int64_t pos = merged_pos_star(t, off, ts, os, S, n, m, j);
    tm[pos] = ts[j];
    ym[pos] = __builtin_nan("");
  }
}

// Prediction times of several series: finite, non-decreasing inside each series (they may
// restart between series); offsets_star[0] = 0, non-decreasing, offsets_star[S] = m.
__global__ void k_validate_star_batch(const double* __restrict__ ts, const int64_t* __restrict__ os, int32_t S,
                                      int64_t m, unsigned long long* __restrict__ key, uint32_t* __restrict__ bad) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0 && (os[0] != 0 || os[S] != m)) atomicMin(key, 1ull);           // SPINGP_E_INVALID
  if (j < S && os[j + 1] < os[j]) atomicMin(key, 1ull);
  if (j >= m) return;
  const int32_t s = series_of(os, S, j);
  unsigned long long code = 0;
  if (!isfinite(ts[j])) code = 4;                                          // SPINGP_E_NONFINITE
  else if (j + 1 < m && j + 1 < os[s + 1] && ts[j + 1] < ts[j]) code = 3;   // SPINGP_E_UNSORTED
  if (code) {
    atomicMin(key, ((unsigned long long)(j + 1) << 4) | code);
    bad[s] = 1u;
  }
}

__global__ void k_gather_batch(const double* __restrict__ t, const int64_t* __restrict__ off, int32_t S, int64_t n,
                               const double* __restrict__ ts, const int64_t* __restrict__ os, int64_t m,
                               const double* __restrict__ fm, const double* __restrict__ fv,
                               double* __restrict__ f_mean, double* __restrict__ f_var,
                               const unsigned long long* __restrict__ status, const uint32_t* __restrict__ bad) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const int64_t pos = merged_pos_star(t, off, ts, os, S, n, m, j);
  // a failed check of the bound inputs or of t* poisons the series (all of them for bad offsets)
  const bool poison = status_poisons_all(status, true) || bad[series_of(os, S, j)] != 0;
  if (f_mean) f_mean[j] = poison ? kPoison : fm[pos];
  if (f_var) f_var[j] = poison ? kPoison : fv[pos];
}

__global__ void k_gather(const double* __restrict__ t, int64_t n, const double* __restrict__ ts, int64_t m,
                         const double* __restrict__ fm, const double* __restrict__ fv, double* __restrict__ f_mean,
                         double* __restrict__ f_var, const unsigned long long* __restrict__ status) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const int64_t pos = j + count_not_greater(t, n, ts[j]);
  const bool poison = *status != ~0ull;
  if (f_mean) f_mean[j] = poison ? kPoison : fm[pos];
  if (f_var) f_var[j] = poison ? kPoison : fv[pos];
}

}  // namespace spg
