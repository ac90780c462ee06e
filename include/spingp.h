/*
 * spingp.h - C ABI of the MI355X (gfx950) library for temporal Gaussian-process inference
 * in sparse-precision form (SpInGP, Grigorievskiy, Lawrence & Sarkka, arXiv:1610.08035).
 *
 * Model (paper Sec. 2.1, eq. ss1): a GP with a Matern covariance is the output y_n = h^T z_n
 * + eps_n of a linear state-space chain z_{n+1} = A_n z_n + q_n, q_n ~ N(0, Q_n),
 * z_0 ~ N(0, P0), eps_n ~ N(0, s2), with A_n = expm(F (t_{n+1} - t_n)) and
 * Q_n = P0 - A_n P0 A_n^T (eq. ss_matern).  The posterior precision of the stacked states is
 * block tridiagonal with b x b blocks (Theorem 1): Kinv + I (x) h h^T / s2.
 *
 * Conventions shared by every call
 *   - Every array argument is a DEVICE pointer (e.g. torch tensor data) owned by the caller,
 *     float64, contiguous, and must stay valid until the handle's stream has executed the
 *     work.  All calls enqueue on the handle's stream and return without synchronising,
 *     except spingp_create, spingp_destroy and spingp_status.
 *   - The library owns its workspace; it is allocated once in spingp_create, so the other
 *     calls never allocate device memory, with one exception: the first spingp_predict on a
 *     handle allocates the merged chain's buffers (4 doubles per point of max_points), which
 *     the handle then keeps (call it once before a capture or a loop that must not allocate).
 *   - Host-detectable errors (null handle or pointer, sizes above the handle's maximum,
 *     unsupported model, call order) are returned synchronously as a spingp_status_t.
 *     Data errors (decreasing or non-finite t, non-finite y, non-positive or non-finite
 *     hyperparameters) are detected on the device, recorded in a status word and reported
 *     by spingp_status.  Until the next spingp_assemble the outputs they affect are NaN: every
 *     output of a one-series handle; with several series, the outputs of the failing series
 *     (all series when the offsets themselves are invalid).
 *   - There is no numerical-failure code: the reduction never inverts Q_n or a covariance, its
 *     pivots are I + Q J with eigenvalues >= 1 and innovation variances >= s2 > 0, so valid
 *     inputs cannot make it break down.
 *   - Nothing is printed, thrown across the ABI or exits the process.
 *   - One handle per host thread and stream.
 *
 * Layouts
 *   - Series are concatenated (t, y have n_points entries).
 *   - State-level outputs are structure-of-arrays with leading dimension ld = n_points:
 *     component c of node n is at base[c * ld + n].  Symmetric b x b blocks are packed upper
 *     triangle, row-major (for b = 3: 00 01 02 11 12 22); general blocks row-major.
 *   - Hyperparameter row (one per series, device memory): per term, in order,
 *     Matern: (lengthscale, signal variance); then the noise variance s2.
 */
#ifndef SPINGP_H
#define SPINGP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spingp_ctx* spingp_handle;

typedef enum {
  SPINGP_OK = 0,
  SPINGP_E_INVALID = 1,     /* bad argument (null pointer, size, value) */
  SPINGP_E_ORDER = 2,       /* call made before the calls it depends on */
  SPINGP_E_UNSORTED = 3,    /* t decreases inside a series (device-detected) */
  SPINGP_E_NONFINITE = 4,   /* NaN/Inf in t or y (device-detected) */
  SPINGP_E_HYPER = 5,       /* hyperparameter not finite or not > 0 (device-detected) */
  SPINGP_E_NOMEM = 6,       /* workspace allocation failed (spingp_create, first spingp_predict) */
  SPINGP_E_HIP = 7,         /* a HIP runtime call failed */
  SPINGP_E_UNSUPPORTED = 8  /* model or size the library does not implement */
} spingp_status_t;

typedef enum {
  SPINGP_MATERN32 = 1,  /* Matern nu = 3/2, state (f, f'), b = 2 */
  SPINGP_MATERN52 = 2,  /* Matern nu = 5/2, b = 3 */
  SPINGP_PERIODIC = 3,  /* periodic, cosine terms 0..harmonics, b = 2 (harmonics + 1) */
  SPINGP_MATERN12 = 4,  /* Matern nu = 1/2 (exponential kernel), b = 1 */
  SPINGP_MATERN72 = 5,  /* Matern nu = 7/2, b = 4 */
  SPINGP_QUASIPERIODIC = 6, /* periodic times exp(-|tau| / decay), b = 2 (harmonics + 1) */
  SPINGP_SQEXP = 7          /* squared exponential by a spectral approximation of order
                               `harmonics` (a state-space form that approximates the kernel,
                               Sec. 2.2: 1 / S truncated after order + 1 terms of its series;
                               even orders 2..10), b = harmonics */
} spingp_kind_t;

/* One additive covariance term; `harmonics` is the number of harmonics of periodic terms and
 * the approximation order of the squared exponential, unused otherwise. */
typedef struct {
  int32_t kind;
  int32_t harmonics;
} spingp_term;

/*
 * Create a handle for a model given as a sum of terms (host array of n_terms entries) and the
 * largest problem it will see.  `stream` is a hipStream_t (NULL = the default stream).
 * Supported models: a single Matern term, nu = 1/2, 3/2, 5/2 or 7/2 (b = 1 to 4; hyperparameter
 * row (lengthscale, signal variance, noise variance), lam = sqrt(2 nu) / lengthscale), any
 * number of series up to max_series; and, for one series, any other sum of up to 8 terms of
 * these kinds with state dimension b = sum of the blocks <= 16 (Sec. 2.1: the sum of
 * independent processes, block-diagonal state), among them the paper's Matern-3/2 + 10th-order
 * squared exponential (b = 12, Sec. 4.2) and the three-term CO2 kernel Matern-3/2 +
 * quasi-periodic (3 harmonics) + squared exponential of order 6 (b = 16, Sec. 4.3).  Blocks:
 * Matern 1..4, periodic and quasi-periodic 2 (harmonics + 1) with harmonics 0..7, squared
 * exponential its order (even, 2..10).  The hyperparameter row of a sum lists each term's in
 * order, then the noise variance: Matern (lengthscale, variance), periodic (lengthscale,
 * variance, period), quasi-periodic (lengthscale, variance, period, decay lengthscale),
 * squared exponential (lengthscale, variance).  Allocates all device workspace (sized for every
 * compiled tile shape, see spingp_tile_shape); returns SPINGP_E_UNSUPPORTED for other models.
 */
int spingp_create(spingp_handle* out, const spingp_term* terms, int32_t n_terms, int64_t max_points,
                  int32_t max_series, void* stream);

/* Release the handle and its workspace (synchronises the stream first). */
int spingp_destroy(spingp_handle h);

/* State dimension b and hyperparameters per series of the handle's model. */
int spingp_state_dim(spingp_handle h);
int spingp_n_hyper(spingp_handle h);

/* Device bytes of workspace the handle holds (spingp_create's, plus the prediction buffers
 * once spingp_predict has run), -1 for NULL. */
int64_t spingp_workspace_bytes(spingp_handle h);

/* Flags of spingp_assemble. */
#define SPINGP_FLAG_GRAPH 1u     /* spingp_logml_grad replays a HIP graph of its launches */
#define SPINGP_FLAG_AUTOTUNE 2u  /* choose the tile shape from the process-wide tuning cache */

/*
 * Assemble: bind the inputs and build the factored block-tridiagonal precision (Theorem 1
 * with G^T Sigma^-1 G = I (x) h h^T / s2, Sec. 2.2).  t, y: [n_points] (n_points >= 1);
 * offsets: [n_series + 1] int64 device array with offsets[0] = 0, non-decreasing,
 * offsets[n_series] = n_points (required when n_series > 1, ignored for one series; empty
 * series are allowed); hyper: [n_series x n_hyper].  Time must be non-decreasing inside each
 * series and may restart between series.  The blocks (A_n, Q_n, J, eta_n) are recomputed from
 * t, y and hyper inside the kernels that use them, so this call only validates the inputs and,
 * for several series, builds the map from chunks of R nodes to series; device-side validation
 * results (bad offsets report SPINGP_E_INVALID) are read with spingp_status.
 * flags: 0 or a combination of
 *   SPINGP_FLAG_GRAPH: the first spingp_logml_grad call, and any call with other output
 *     pointers, captures its launch sequence into a HIP graph on a private non-blocking stream
 *     (created at the first capture) and instantiates it; calls replay it on the handle's
 *     stream (hyperparameters are read from device memory, so new values need no new capture).
 *   SPINGP_FLAG_AUTOTUNE: use the tile shape the process-wide cache holds for this problem
 *     class (b, one or several series, ceil log2 n_points, ceil log2 n_series); on a miss run
 *     spingp_tune(h, 3) here, which synchronises the stream.
 * Invalidates any earlier factorisation and captured graph.
 */
int spingp_assemble(spingp_handle h, const double* t, const double* y, const int64_t* offsets, int32_t n_series,
                    int64_t n_points, const double* hyper, uint32_t flags);

/*
 * Factor: odd-even block cyclic reduction of the precision (Sec. 3.1, subproblems 1 and 3).
 * Folds each chunk of consecutive nodes, reduces the chunk elements with a balanced tree and
 * runs the down-sweeps that hand every chunk its exact boundary state.  Needs assemble.
 */
int spingp_factor(spingp_handle h);

/*
 * Log marginal likelihood (eq. ml2 via the determinant lemma eq. det_1) of the factored
 * problem.  logml: [n_series]; datafit: NULL or [n_series] = y^T K_y^-1 y; logdet: NULL or
 * [n_series] = log det K_y.  An empty series has all three 0.  Needs factor.  One series reads
 * the root of the reduction; several series run an elimination sweep over every chunk.
 */
int spingp_logml(spingp_handle h, double* logml, double* datafit, double* logdet);

/*
 * Posterior mean (subproblem 1, eq. mean3/mean6 at the training times): f_mean: NULL or
 * [n_points] = E[f(t_n) | y]; z_mean: NULL or [b x n_points] SoA = E[z_n | y].  Needs factor.
 */
int spingp_solve(spingp_handle h, double* f_mean, double* z_mean);

/*
 * Selected inverse (subproblems 2 and 4: the block-tridiagonal part of the inverse precision,
 * Sec. 3.1): f_var: NULL or [n_points] = Var[f(t_n) | y] (latent, eq. k3, no noise);
 * S_diag: NULL or [b(b+1)/2 x n_points] = Cov(z_n | y); S_sub: NULL or [b*b x n_points], entry n
 * = Cov(z_{n+1}, z_n | y) for n < n_points - 1 inside one series (the entry at the last node of
 * every series is left untouched).  Needs factor.
 */
int spingp_selinv(spingp_handle h, double* f_var, double* S_diag, double* S_sub);

/*
 * Log marginal likelihood and its gradient (Sec. 2.4) with respect to the raw hyperparameters
 * of the hyperparameter row: grad: [n_series x n_hyper], logml: [n_series] (an empty series
 * gets 0 and a zero gradient).  mask: NULL (every component) or a HOST array of n_hyper bytes;
 * components whose byte is 0 are written as 0 (for hyperparameters an optimiser holds fixed;
 * a HIP graph is captured again when the mask changes).  Always runs the forward reduction
 * itself (it reads the hyperparameters from device memory, so an optimiser may update them
 * between calls without a new assemble), then the adjoint sweep; leaves the handle factored.
 * Replays a HIP graph when assembled with SPINGP_FLAG_GRAPH.  Needs assemble.
 */
int spingp_logml_grad(spingp_handle h, double* logml, double* grad, const uint8_t* mask);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): spingp_logml_grad for one series of a single Matern
 * term without a handle.  terms: host array, n_terms = 1, kind SPINGP_MATERN12/32/52/72; t, y:
 * [n_points] device arrays (t non-decreasing, finite); hyper: [3] device array (lengthscale,
 * signal variance, noise variance, all > 0); logml: [1], grad: [3] device outputs; stream: a
 * hipStream_t (NULL = the default stream).  The inputs are not checked on the device: invalid
 * data gives unspecified values, without accesses outside the arguments and the workspace.
 * Workspace: a fixed device array of SPINGP_NOALLOC_SCRATCH_BYTES inside the library, one copy
 * per GPU, kept until the process ends; the call allocates and frees nothing.  It runs the same
 * kernels as spingp_logml_grad with tile shape 0 (so the results are identical to a handle's on
 * that shape).  Sizes whose workspace exceeds the array return SPINGP_E_UNSUPPORTED: n_points up
 * to 2^16 fit for every b (at most 90 112 at b = 4, 142 336 at b = 3, 259 072 at b = 2, 523 264
 * at b = 1).  All calls on one GPU share its array: calls
 * that overlap in time on one GPU (several streams or host threads) race and must be ordered by
 * the caller.  Enqueues on `stream` and returns without synchronising.
 */
#define SPINGP_NOALLOC_SCRATCH_BYTES (8 << 20)
int spingp_logml_grad_noalloc(const spingp_term* terms, int32_t n_terms, const double* t, const double* y,
                              int64_t n_points, const double* hyper, double* logml, double* grad, void* stream);

/*
 * Tile shapes (R nodes folded per lane, L lanes per work-group) compiled into the library;
 * shape 0 is the default.  Results agree across shapes up to rounding.
 */
int spingp_tile_count(void);
int spingp_tile_shape(int32_t index, int32_t* R, int32_t* L);
/*
 * Current shape of the handle; selecting one re-validates and re-maps the bound inputs.
 * Shapes with R < 8 are available only on handles created with max_points <= 2^20 (their
 * workspace is twice as large); elsewhere spingp_set_tile returns SPINGP_E_UNSUPPORTED and
 * the autotuner skips them.
 */
int spingp_get_tile(spingp_handle h, int32_t* index);
int spingp_set_tile(spingp_handle h, int32_t index);
/*
 * Autotuner: time spingp_logml_grad `reps` times on the assembled problem for every tile shape,
 * in two passes over the shapes (HIP events on the handle's stream; synchronises), keep the
 * shape with the best of its two timings for this handle and record it in the process-wide
 * cache used by SPINGP_FLAG_AUTOTUNE.  Needs assemble.
 */
int spingp_tune(spingp_handle h, int32_t reps);

/*
 * Prediction at new times (eq. mean4-mean6 and the variance of eq. k3 at t*): the latent
 * predictive mean f_mean[j] = E[f(t*_j) | y] and variance f_var[j] = Var[f(t*_j) | y] (no noise
 * term).  t_star: [n_star] device array, finite; f_mean, f_var: NULL or [n_star].
 * One series (offsets_star NULL): t_star non-decreasing.  Several series: offsets_star is an
 * [n_series + 1] device int64 array, offsets_star[0] = 0, non-decreasing, offsets_star[n_series]
 * = n_star; times [offsets_star[s], offsets_star[s+1]) belong to series s, with its
 * hyperparameters, and are non-decreasing within it; a series may get none.  The call re-runs
 * the assemble-time checks of the bound inputs and checks t_star: spingp_status then reports
 * these (for t_star: code 1 for the offsets, 3 or 4 with the index in t_star); results are then
 * unspecified.  The prediction times are merged into the chain as nodes without an
 * observation (after training points at equal times) and the whole reduction runs on the merged
 * chain, so n_points + n_star must not exceed the handle's max_points (SPINGP_E_INVALID).  Uses
 * the hyperparameters in device memory at the time of the call.  Overwrites the handle's
 * factorisation: call spingp_factor again before spingp_logml, spingp_solve or spingp_selinv
 * (spingp_logml_grad refactors by itself).  Needs assemble; a batched handle needs offsets_star
 * (SPINGP_E_INVALID without).  The first call allocates the prediction buffers (32 bytes per
 * point of max_points; SPINGP_E_NOMEM if that fails), later calls reuse them.
 */
int spingp_predict(spingp_handle h, const double* t_star, const int64_t* offsets_star, int64_t n_star,
                   double* f_mean, double* f_var);

/*
 * Diagnostics (not part of the hot path, which never forms these blocks): the edge blocks and
 * the multiplied-out blocks of the posterior precision of every series (Theorem 1, Sec. 2.2):
 *   A: NULL or [b*b x n_points], entry n = A_n = expm(F (t_{n+1} - t_n)) (row-major; zero at
 *      the last node of a series);
 *   Q: NULL or [b(b+1)/2 x n_points] packed upper, Q_n = P0 - A_n P0 A_n^T (zero there too);
 *   D: NULL or [b(b+1)/2 x n_points] packed upper, diagonal block D_n = J + (P0^-1 at a
 *      series' first node, else Q_{n-1}^-1) + A_n^T Q_n^-1 A_n (the last term absent at its
 *      last node), J = h h^T / s2;
 *   Bsub: NULL or [b*b x n_points], entry n = the block (n+1, n) = -Q_n^-1 A_n.
 * D and Bsub need Q_n^-1 and lose accuracy as Q_n approaches singularity (near-duplicate
 * times); Q_n = 0 (duplicate times) gives non-finite values.  Needs assemble.  Matern models
 * only (SPINGP_E_UNSUPPORTED for the sum kernel).
 */
int spingp_blocks(spingp_handle h, double* A, double* Q, double* D, double* Bsub);

/*
 * Synchronise the handle's stream and report the first device-detected data error since the
 * last assemble: returns SPINGP_OK or the error code; *first_bad (host, may be NULL) receives
 * the offending point index (or -1 for a hyperparameter error / no error).
 */
int spingp_status(spingp_handle h, int64_t* first_bad);

/*
 * Diagnostics: per-kernel timing with HIP events recorded on the handle's stream around every
 * launch the library makes.  spingp_profile(h, 1) creates the events and starts recording,
 * spingp_profile(h, 0) stops and releases them.  spingp_profile_read synchronises and returns,
 * per kernel id (0 validation and chunk map, 1 forward fold + work-group tree, 2 top-level
 * tree, 3 top-level path walk + work-group down-sweep + chunk elimination + adjoint, 4 sums of
 * the reverse kernel's partials (per series, or over work-groups for one series), 5 a whole
 * graph replay of spingp_logml_grad), the total
 * milliseconds and launch counts since the last read (host arrays of SPINGP_N_KERNELS).
 */
#define SPINGP_N_KERNELS 6
int spingp_profile(spingp_handle h, int enable);
int spingp_profile_read(spingp_handle h, double* total_ms, int64_t* launches);

/* Static description of a status code. */
const char* spingp_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* SPINGP_H */
