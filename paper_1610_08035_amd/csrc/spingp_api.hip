// Host side of the C ABI declared in include/spingp.h: handle, workspace, validation and the
// launch sequence of the hot path.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <new>

#include "../../include/spingp.h"
#include "spingp_kernels.hpp"

namespace {

constexpr int kR = 8;        // points folded sequentially per lane
constexpr int kL = 128;      // lanes (chunks) per work-group
constexpr int kT = 256;      // threads of the element-wise helper kernels

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
int64_t next_pow2(int64_t x) {
  int64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Device-side validation: key = (index << 4) | code, minimised over offending points.
__global__ void k_validate(const double* __restrict__ t, const double* __restrict__ y, int64_t n,
                           const double* __restrict__ hyper, int n_hyper, unsigned long long* key) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    for (int k = 0; k < n_hyper; ++k) {
      const double h = hyper[k];
      if (!(isfinite(h) && h > 0.0)) atomicMin(key, (unsigned long long)SPINGP_E_HYPER);
    }
  }
  if (i >= n) return;
  const double ti = t[i], yi = y[i];
  unsigned long long code = 0;
  if (!isfinite(ti) || !isfinite(yi)) code = SPINGP_E_NONFINITE;
  else if (i + 1 < n && t[i + 1] < ti) code = SPINGP_E_UNSORTED;
  if (code) atomicMin(key, ((unsigned long long)(i + 1) << 4) | code);
}

__global__ void k_fill_key(unsigned long long* key) { *key = ~0ull; }

__global__ void k_copy_scalars(const double* __restrict__ scal, int64_t n_pts, double* logml, double* datafit,
                               double* logdet) {
  if (threadIdx.x == 0) {
    if (logml) logml[0] = scal[0];
    if (datafit) datafit[0] = -2.0 * scal[1];
    if (logdet) logdet[0] = -2.0 * scal[2] - (double)n_pts * spg::kLog2Pi;
  }
}

}  // namespace

struct spingp_ctx {
  int b = 0;
  int n_hyper = 0;
  int64_t max_points = 0;
  int32_t max_series = 0;
  hipStream_t stream = nullptr;
  // workspace
  double* lane = nullptr;          // work-group trees of the forward kernel (2L slots each)
  double* top = nullptr;           // top-level tree over the work-group aggregates
  unsigned int* top_cnt = nullptr; // arrival counters of the top-level bands
  int64_t top_ld = 0, top_cnt_n = 0;
  unsigned int* done = nullptr;    // finished work-groups of the backward kernel
  double* scal = nullptr;          // one series: log-likelihood terms at the root
  double* part = nullptr;          // gradient / log-likelihood partials
  int64_t part_ld = 0;
  int32_t* chunk_series = nullptr; // several series: series of every chunk slot
  int64_t* chunk_first = nullptr;  // several series: first chunk of every series
  unsigned long long* key = nullptr;
  int64_t lane_ld = 0, G_max = 0, slots_max = 0;
  // bound inputs
  const double* t = nullptr;
  const double* y = nullptr;
  const double* hyper = nullptr;
  const int64_t* offsets = nullptr;
  int64_t n_points = 0;
  int32_t n_series = 0;
  bool batched = false;
  int64_t G = 0;
  bool assembled = false;
  bool factored = false;
  // profiling (optional)
  static constexpr int kPool = 64;
  bool prof = false;
  int prof_n = 0;
  int prof_kid[kPool];
  hipEvent_t prof_ev[2 * kPool];
  double prof_ms[SPINGP_N_KERNELS];
  int64_t prof_cnt[SPINGP_N_KERNELS];
};

static void prof_flush(spingp_ctx* h) {
  if (!h->prof || h->prof_n == 0) return;
  (void)hipEventSynchronize(h->prof_ev[2 * h->prof_n - 1]);
  for (int i = 0; i < h->prof_n; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->prof_ev[2 * i], h->prof_ev[2 * i + 1]) == hipSuccess) {
      h->prof_ms[h->prof_kid[i]] += ms;
      h->prof_cnt[h->prof_kid[i]] += 1;
    }
  }
  h->prof_n = 0;
}
static void prof_begin(spingp_ctx* h) {
  if (!h->prof) return;
  if (h->prof_n == spingp_ctx::kPool) prof_flush(h);
  (void)hipEventRecord(h->prof_ev[2 * h->prof_n], h->stream);
}
static void prof_end(spingp_ctx* h, int kid) {
  if (!h->prof) return;
  (void)hipEventRecord(h->prof_ev[2 * h->prof_n + 1], h->stream);
  h->prof_kid[h->prof_n] = kid;
  h->prof_n += 1;
}

static int hip_ok(hipError_t e) { return e == hipSuccess ? SPINGP_OK : SPINGP_E_HIP; }

// Work-groups of the forward and reverse kernels for n points in s series: one lane per chunk
// of R consecutive nodes of one series; with several series every series starts a new chunk,
// so there are at most ceil(n / R) + s chunks (the unused slots at the end are padding).
static int64_t groups_for(int64_t n, int64_t s, bool batched) {
  const int64_t chunks = ceil_div(n, kR) + (batched ? s : 0);
  return ceil_div(chunks, kL);
}

extern "C" int spingp_create(spingp_handle* out, const spingp_term* terms, int32_t n_terms, int64_t max_points,
                             int32_t max_series, void* stream) {
  if (!out || !terms || n_terms < 1 || max_points < 1 || max_series < 1) return SPINGP_E_INVALID;
  *out = nullptr;
  if (n_terms != 1) return SPINGP_E_UNSUPPORTED;
  int b;
  if (terms[0].kind == SPINGP_MATERN32) b = 2;
  else if (terms[0].kind == SPINGP_MATERN52) b = 3;
  else return SPINGP_E_UNSUPPORTED;
  // grid sizes are 32-bit: at most 2^31 - 1 work-groups of the largest launch
  if (max_points > (int64_t(1) << 40) || groups_for(max_points, max_series, max_series > 1) >= (int64_t(1) << 31))
    return SPINGP_E_UNSUPPORTED;
  spingp_ctx* h = new (std::nothrow) spingp_ctx();
  if (!h) return SPINGP_E_NOMEM;
  h->b = b;
  h->n_hyper = 3;
  h->max_points = max_points;
  h->max_series = max_series;
  h->stream = (hipStream_t)stream;
  const int NF = (b == 2) ? spg::ElemLayout<2>::kFields : spg::ElemLayout<3>::kFields;
  h->G_max = groups_for(max_points, max_series, max_series > 1);
  h->slots_max = h->G_max * kL;
  h->lane_ld = h->G_max * 2 * kL;
  int64_t ltop = 32;
  while (ltop < h->G_max) ltop *= 32;
  h->top_ld = 2 * ltop;
  h->top_cnt_n = 0;
  for (int64_t n = h->G_max; ; n = ceil_div(n, 32)) {
    h->top_cnt_n += ceil_div(n, 32);
    if (n <= 32) break;
  }
  h->part_ld = max_series > 1 ? h->slots_max : h->G_max;
  const int64_t part_n = max_series > 1 ? 5 * h->slots_max : 3 * h->G_max;
  bool ok = true;
  ok = ok && hipMalloc(&h->lane, sizeof(double) * NF * h->lane_ld) == hipSuccess;
  ok = ok && hipMalloc(&h->top, sizeof(double) * NF * h->top_ld) == hipSuccess;
  ok = ok && hipMalloc(&h->top_cnt, sizeof(unsigned int) * h->top_cnt_n) == hipSuccess;
  ok = ok && hipMemset(h->top_cnt, 0, sizeof(unsigned int) * h->top_cnt_n) == hipSuccess;
  ok = ok && hipMalloc(&h->scal, sizeof(double) * 8) == hipSuccess;
  ok = ok && hipMalloc(&h->part, sizeof(double) * part_n) == hipSuccess;
  ok = ok && hipMalloc(&h->key, sizeof(unsigned long long)) == hipSuccess;
  ok = ok && hipMalloc(&h->done, sizeof(unsigned int)) == hipSuccess;
  ok = ok && hipMemset(h->done, 0, sizeof(unsigned int)) == hipSuccess;
  ok = ok && hipMemset(h->key, 0xff, sizeof(unsigned long long)) == hipSuccess;
  if (max_series > 1) {
    ok = ok && hipMalloc(&h->chunk_series, sizeof(int32_t) * h->slots_max) == hipSuccess;
    ok = ok && hipMalloc(&h->chunk_first, sizeof(int64_t) * ((int64_t)max_series + 1)) == hipSuccess;
  }
  ok = ok && hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    spingp_destroy(h);
    return SPINGP_E_NOMEM;
  }
  *out = h;
  return SPINGP_OK;
}

extern "C" int spingp_profile(spingp_handle h, int enable) {
  if (!h) return SPINGP_E_INVALID;
  if (enable && !h->prof) {
    for (int i = 0; i < 2 * spingp_ctx::kPool; ++i)
      if (hipEventCreate(&h->prof_ev[i]) != hipSuccess) return SPINGP_E_HIP;
    for (int k = 0; k < SPINGP_N_KERNELS; ++k) {
      h->prof_ms[k] = 0.0;
      h->prof_cnt[k] = 0;
    }
    h->prof_n = 0;
    h->prof = true;
  } else if (!enable && h->prof) {
    prof_flush(h);
    for (int i = 0; i < 2 * spingp_ctx::kPool; ++i) (void)hipEventDestroy(h->prof_ev[i]);
    h->prof = false;
  }
  return SPINGP_OK;
}

extern "C" int spingp_profile_read(spingp_handle h, double* total_ms, int64_t* launches) {
  if (!h || !total_ms || !launches) return SPINGP_E_INVALID;
  if (!h->prof) return SPINGP_E_ORDER;
  prof_flush(h);
  for (int k = 0; k < SPINGP_N_KERNELS; ++k) {
    total_ms[k] = h->prof_ms[k];
    launches[k] = h->prof_cnt[k];
    h->prof_ms[k] = 0.0;
    h->prof_cnt[k] = 0;
  }
  return SPINGP_OK;
}

extern "C" int spingp_destroy(spingp_handle h) {
  if (!h) return SPINGP_E_INVALID;
  (void)spingp_profile(h, 0);
  if (h->stream || h->lane) (void)hipStreamSynchronize(h->stream);
  (void)hipFree(h->lane);
  (void)hipFree(h->top);
  (void)hipFree(h->top_cnt);
  (void)hipFree(h->scal);
  (void)hipFree(h->part);
  (void)hipFree(h->key);
  (void)hipFree(h->done);
  (void)hipFree(h->chunk_series);
  (void)hipFree(h->chunk_first);
  delete h;
  return SPINGP_OK;
}

extern "C" int spingp_state_dim(spingp_handle h) { return h ? h->b : -1; }
extern "C" int spingp_n_hyper(spingp_handle h) { return h ? h->n_hyper : -1; }

static spg::SeriesMap make_map(const spingp_ctx* h) {
  spg::SeriesMap sm;
  memset(&sm, 0, sizeof(sm));
  sm.n_series = h->n_series;
  if (h->batched) {
    sm.offsets = h->offsets;
    sm.chunk_series = h->chunk_series;
    sm.chunk_first = h->chunk_first;
    sm.slots = h->G * kL;
  }
  return sm;
}

extern "C" int spingp_assemble(spingp_handle h, const double* t, const double* y, const int64_t* offsets,
                               int32_t n_series, int64_t n_points, const double* hyper, uint32_t flags) {
  if (!h || !t || !y || !hyper || flags != 0) return SPINGP_E_INVALID;
  if (n_series < 1 || n_series > h->max_series) return SPINGP_E_INVALID;
  if (n_points < 1 || n_points > h->max_points) return SPINGP_E_INVALID;
  if (n_series > 1 && !offsets) return SPINGP_E_INVALID;
  h->assembled = false;
  h->factored = false;
  h->t = t;
  h->y = y;
  h->hyper = hyper;
  h->offsets = offsets;
  h->n_points = n_points;
  h->n_series = n_series;
  // one series is the whole array (offsets, if given, are not read)
  h->batched = n_series > 1;
  h->G = groups_for(n_points, n_series, h->batched);
  hipLaunchKernelGGL(k_fill_key, dim3(1), dim3(1), 0, h->stream, h->key);
  prof_begin(h);
  if (!h->batched) {
    hipLaunchKernelGGL(k_validate, dim3((unsigned)ceil_div(n_points, kT)), dim3(kT), 0, h->stream, t, y, n_points,
                       hyper, h->n_hyper, h->key);
  } else {
    const int64_t slots = h->G * kL;
    hipLaunchKernelGGL(spg::k_chunk_first, dim3(1), dim3(256), 0, h->stream, offsets, n_series, n_points, kR,
                       h->chunk_first, h->key);
    hipLaunchKernelGGL(spg::k_chunk_fill, dim3((unsigned)ceil_div(slots, kT)), dim3(kT), 0, h->stream,
                       h->chunk_series, slots);
    hipLaunchKernelGGL(spg::k_chunk_map, dim3((unsigned)ceil_div(n_series, kT)), dim3(kT), 0, h->stream,
                       h->chunk_first, n_series, slots, h->chunk_series);
    hipLaunchKernelGGL(spg::k_validate_chunks<kR>, dim3((unsigned)ceil_div(slots, kT)), dim3(kT), 0, h->stream, t,
                       y, n_points, hyper, make_map(h), h->key);
  }
  prof_end(h, 0);
  const int rc = hip_ok(hipGetLastError());
  h->assembled = rc == SPINGP_OK;
  return rc;
}

static spg::TopTree make_top(spingp_ctx* h) {
  spg::TopTree T;
  memset(&T, 0, sizeof(T));
  T.elems = h->top;
  T.ld = h->top_ld;
  T.G = h->G;
  T.cnt = h->top_cnt;
  int nb = 1;
  int64_t ltop = 32;
  while (ltop < h->G) {
    ltop *= 32;
    ++nb;
  }
  T.Ltop = ltop;
  T.n_bands = nb;
  int64_t off = 0, n = h->G;
  for (int b = 0; b < nb; ++b) {
    T.cnt_off[b] = off;
    off += ceil_div(n, 32);
    n = ceil_div(n, 32);
  }
  return T;
}

template <int B, bool BATCHED>
static int launch_factor(spingp_ctx* h) {
  const spg::TopTree top = make_top(h);
  const spg::SeriesMap sm = make_map(h);
  prof_begin(h);
  hipLaunchKernelGGL((spg::k_fwd<B, kR, kL, BATCHED>), dim3((unsigned)h->G), dim3(kL), 0, h->stream, h->t, h->y,
                     h->n_points, h->hyper, sm, h->lane, h->lane_ld, top, h->key);
  prof_end(h, 1);
  prof_begin(h);
  hipLaunchKernelGGL((spg::k_top_bands<B, BATCHED>), dim3((unsigned)ceil_div(h->G, 32)), dim3(64), 0, h->stream,
                     h->hyper, sm, top, h->scal);
  prof_end(h, 2);
  return hip_ok(hipGetLastError());
}

static int do_factor(spingp_ctx* h) {
  if (h->b == 2) return h->batched ? launch_factor<2, true>(h) : launch_factor<2, false>(h);
  return h->batched ? launch_factor<3, true>(h) : launch_factor<3, false>(h);
}

extern "C" int spingp_factor(spingp_handle h) {
  if (!h) return SPINGP_E_INVALID;
  if (!h->assembled) return SPINGP_E_ORDER;
  const int rc = do_factor(h);
  h->factored = rc == SPINGP_OK;
  return rc;
}

template <int B, int MODE, bool BATCHED>
static int launch_bwd(spingp_ctx* h, const spg::BwdOut& o) {
  prof_begin(h);
  hipLaunchKernelGGL((spg::k_bwd<B, kR, kL, MODE, BATCHED>), dim3((unsigned)h->G), dim3(kL), 0, h->stream, h->t,
                     h->y, h->n_points, h->hyper, make_map(h), h->lane, h->lane_ld, make_top(h), o);
  prof_end(h, 3);
  return hip_ok(hipGetLastError());
}

template <int MODE>
static int run_bwd(spingp_ctx* h, const spg::BwdOut& o) {
  if (h->b == 2) return h->batched ? launch_bwd<2, MODE, true>(h, o) : launch_bwd<2, MODE, false>(h, o);
  return h->batched ? launch_bwd<3, MODE, true>(h, o) : launch_bwd<3, MODE, false>(h, o);
}

// several series: per-series fixed-order sums of the reverse kernel's per-chunk partials
static int series_reduce(spingp_ctx* h, double* logml, double* datafit, double* logdet, double* grad) {
  prof_begin(h);
  hipLaunchKernelGGL(spg::k_series_reduce, dim3((unsigned)h->n_series), dim3(64), 0, h->stream, make_map(h),
                     h->part, h->part_ld, h->n_points, logml, datafit, logdet, grad);
  prof_end(h, 4);
  return hip_ok(hipGetLastError());
}

static spg::BwdOut make_out(spingp_ctx* h) {
  spg::BwdOut o;
  memset(&o, 0, sizeof(o));
  o.ld = h->n_points;
  o.part = h->part;
  o.part_ld = h->part_ld;
  o.done = h->done;
  o.scal = h->scal;
  return o;
}

extern "C" int spingp_logml(spingp_handle h, double* logml, double* datafit, double* logdet) {
  if (!h || !logml) return SPINGP_E_INVALID;
  if (!h->factored) return SPINGP_E_ORDER;
  if (!h->batched) {
    hipLaunchKernelGGL(k_copy_scalars, dim3(1), dim3(64), 0, h->stream, h->scal, h->n_points, logml, datafit,
                       logdet);
    return hip_ok(hipGetLastError());
  }
  // several series: the per-series terms come from an elimination sweep over every chunk
  const int rc = run_bwd<spg::kWantLogml>(h, make_out(h));
  if (rc) return rc;
  return series_reduce(h, logml, datafit, logdet, nullptr);
}

extern "C" int spingp_solve(spingp_handle h, double* f_mean, double* z_mean) {
  if (!h) return SPINGP_E_INVALID;
  if (!h->factored) return SPINGP_E_ORDER;
  if (!f_mean && !z_mean) return SPINGP_OK;
  spg::BwdOut o = make_out(h);
  o.f_mean = f_mean;
  o.z_mean = z_mean;
  return run_bwd<spg::kWantMean>(h, o);
}

extern "C" int spingp_selinv(spingp_handle h, double* f_var, double* S_diag, double* S_sub) {
  if (!h) return SPINGP_E_INVALID;
  if (!h->factored) return SPINGP_E_ORDER;
  if (!f_var && !S_diag && !S_sub) return SPINGP_OK;
  spg::BwdOut o = make_out(h);
  o.f_var = f_var;
  o.S_diag = S_diag;
  o.S_sub = S_sub;
  if (S_sub) return run_bwd<spg::kWantVar | spg::kWantSub>(h, o);
  return run_bwd<spg::kWantVar>(h, o);
}

extern "C" int spingp_logml_grad(spingp_handle h, double* logml, double* grad) {
  if (!h || !logml || !grad) return SPINGP_E_INVALID;
  if (!h->assembled) return SPINGP_E_ORDER;
  // the forward pass always runs: hyperparameters live in device memory and may have changed
  int rc = spingp_factor(h);
  if (rc) return rc;
  spg::BwdOut o = make_out(h);
  if (!h->batched) {
    o.logml = logml;
    o.grad = grad;
  }
  rc = run_bwd<spg::kWantGrad>(h, o);
  if (rc || !h->batched) return rc;
  return series_reduce(h, logml, nullptr, nullptr, grad);
}

extern "C" int spingp_status(spingp_handle h, int64_t* first_bad) {
  if (!h) return SPINGP_E_INVALID;
  if (first_bad) *first_bad = -1;
  if (hipStreamSynchronize(h->stream) != hipSuccess) return SPINGP_E_HIP;
  if (!h->assembled) return SPINGP_OK;
  unsigned long long key = 0;
  if (hipMemcpy(&key, h->key, sizeof(key), hipMemcpyDeviceToHost) != hipSuccess) return SPINGP_E_HIP;
  if (key == ~0ull) return SPINGP_OK;
  const int code = (int)(key & 15ull);
  const int64_t idx = (int64_t)(key >> 4) - 1;
  if (first_bad) *first_bad = idx;
  return code;
}

extern "C" const char* spingp_strerror(int code) {
  switch (code) {
    case SPINGP_OK: return "ok";
    case SPINGP_E_INVALID: return "invalid argument";
    case SPINGP_E_ORDER: return "call made before the calls it depends on";
    case SPINGP_E_UNSORTED: return "time points decrease inside a series";
    case SPINGP_E_NONFINITE: return "non-finite time or observation";
    case SPINGP_E_HYPER: return "hyperparameter not finite or not positive";
    case SPINGP_E_NOMEM: return "device workspace allocation failed";
    case SPINGP_E_HIP: return "HIP runtime error";
    case SPINGP_E_UNSUPPORTED: return "model or size not supported";
    default: return "unknown status";
  }
}
