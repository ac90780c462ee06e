// Internal host interface between the C ABI (spingp_api.hip) and the tile translation units
// (spingp_tile.hip, compiled once per tile shape).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spingp_kernels.hpp"

namespace spg {

// Everything a launch sequence needs: bound inputs, workspace and the stream.
struct LaunchCtx {
  int b;
  hipStream_t stream;
  const double* t;
  const double* y;
  const double* hyper;
  const int64_t* offsets;
  int64_t n_points;
  int32_t n_series;
  bool batched;
  double* lane;                  // work-group trees, leading dimension lane_ld
  int64_t lane_ld;
  double* top;                   // top-level tree, leading dimension top_ld
  int64_t top_ld;
  unsigned int* top_cnt;
  double* scal;
  double* part;
  int64_t part_ld;
  int32_t* chunk_series;
  int64_t* chunk_first;
  uint32_t* bad;                 // several series: per-series failed-check flags
  unsigned long long* key;
  // optional timing hook around every launch: mark(arg, kernel id, 0 = before, 1 = after)
  void (*mark)(void* arg, int kid, int end);
  void* mark_arg;
};

// Kernel ids of the timing hook.
enum : int { kKidValidate = 0, kKidFwd = 1, kKidTop = 2, kKidBwd = 3, kKidReduce = 4, kKidGraph = 5 };

// One tile shape: R points folded per lane, L lanes per work-group.
struct TileOps {
  int R;
  int L;
  // work-groups for n points in s series (every series starts a new chunk when batched)
  int64_t (*groups)(int64_t n, int64_t s, bool batched);
  // several series: chunk map and per-series validation of the bound inputs
  hipError_t (*map)(const LaunchCtx& c);
  // forward fold + work-group trees, then the top-level tree
  hipError_t (*factor)(const LaunchCtx& c);
  // reverse sweep with the given output selection (kWant* bits)
  hipError_t (*bwd)(const LaunchCtx& c, int mode, const BwdOut& o);
  // materialised edge and precision blocks (diagnostics)
  hipError_t (*blocks)(const LaunchCtx& c, double* A, double* Q, double* D, double* Bsub);
};

// Shape of the top-level tree over G leaves: n_levels = ceil log2 G (at least 1), bands of 5
// levels (the last one may be shorter).
inline int top_levels(int64_t G) {
  int k = 1;
  while (((int64_t)1 << k) < G) ++k;
  return k;
}
inline int top_band_levels(int n_levels, int band) {
  const int r = n_levels - 5 * band;
  return r < 5 ? r : 5;
}

// Sizes of the top-level tree over G leaves: slots (2 * Ltop) and arrival counters.
inline void top_sizes(int64_t G, int64_t& slots, int64_t& counters) {
  const int K = top_levels(G);
  slots = (int64_t)2 << K;
  counters = 0;
  int64_t n = G;
  for (int b = 0; 5 * b < K; ++b) {
    const int bs = top_band_levels(K, b);
    n = (n + ((int64_t)1 << bs) - 1) >> bs;
    counters += n;
  }
}

inline TopTree make_top(const LaunchCtx& c, int64_t G) {
  TopTree T;
  T.elems = c.top;
  T.ld = c.top_ld;
  T.G = G;
  T.cnt = c.top_cnt;
  T.n_levels = top_levels(G);
  T.Ltop = (int64_t)1 << T.n_levels;
  T.n_bands = (T.n_levels + 4) / 5;
  for (int b = 0; b < 8; ++b) T.cnt_off[b] = 0;
  int64_t off = 0, n = G;
  for (int b = 0; b < T.n_bands; ++b) {
    const int bs = top_band_levels(T.n_levels, b);
    T.cnt_off[b] = off;
    n = (n + ((int64_t)1 << bs) - 1) >> bs;   // groups of this band
    off += n;
  }
  return T;
}

inline SeriesMap make_map(const LaunchCtx& c, int64_t slots) {
  SeriesMap sm;
  sm.offsets = nullptr;
  sm.chunk_series = nullptr;
  sm.chunk_first = nullptr;
  sm.slots = 0;
  sm.n_series = c.n_series;
  sm.bad = nullptr;
  if (c.batched) {
    sm.offsets = c.offsets;
    sm.chunk_series = c.chunk_series;
    sm.chunk_first = c.chunk_first;
    sm.slots = slots;
    sm.bad = c.bad;
  }
  return sm;
}

// Tile shapes compiled into the library, in order of preference when untuned.
constexpr int kNumTiles = 6;
const TileOps* tile_ops(int i);

}  // namespace spg
