// Launch sequences of one tile shape (R points folded per lane, L lanes per work-group).
// Compiled once per shape with -DSPG_TILE_R=<R> -DSPG_TILE_L=<L>; each object exports
// spg::tile_ops_R<R>_L<L>().
#include "spingp_host.hpp"

#ifndef SPG_TILE_R
#error "SPG_TILE_R must be defined"
#endif
#ifndef SPG_TILE_L
#error "SPG_TILE_L must be defined"
#endif

#define SPG_CAT2(a, b, c, d) a##b##c##d
#define SPG_CAT(a, b, c, d) SPG_CAT2(a, b, c, d)
#define SPG_TILE_FN SPG_CAT(tile_ops_R, SPG_TILE_R, _L, SPG_TILE_L)

namespace spg {
namespace {

constexpr int R = SPG_TILE_R;
constexpr int L = SPG_TILE_L;

int64_t groups(int64_t n, int64_t s, bool batched) {
  const int64_t chunks = (n + R - 1) / R + (batched ? s : 0);
  return (chunks + L - 1) / L;
}

inline void mark(const LaunchCtx& c, int kid, int end) {
  if (c.mark) c.mark(c.mark_arg, kid, end);
}

hipError_t map(const LaunchCtx& c) {
  const int64_t slots = groups(c.n_points, c.n_series, true) * L;
  const SeriesMap sm = make_map(c, slots);
  constexpr int T = 256;
  hipLaunchKernelGGL(k_validate_chunks<R>, dim3((unsigned)((slots + T - 1) / T)), dim3(T), 0, c.stream, c.t, c.y,
                     c.n_points, c.hyper, sm, c.key);
  return hipGetLastError();
}

template <int B, bool BATCHED>
hipError_t factor_b(const LaunchCtx& c) {
  const int64_t G = groups(c.n_points, c.n_series, BATCHED);
  const TopTree top = make_top(c, G);
  const SeriesMap sm = make_map(c, G * L);
  mark(c, kKidFwd, 0);
  hipLaunchKernelGGL((k_fwd<B, R, L, BATCHED>), dim3((unsigned)G), dim3(L), 0, c.stream, c.t, c.y, c.n_points,
                     c.hyper, sm, c.lane, c.lane_ld, top, c.key);
  mark(c, kKidFwd, 1);
  mark(c, kKidTop, 0);
  hipLaunchKernelGGL((k_top_bands<B, BATCHED>), dim3((unsigned)((G + 31) / 32)), dim3(kTopThreads), 0, c.stream,
                     c.hyper, sm, top, c.scal);
  mark(c, kKidTop, 1);
  return hipGetLastError();
}

hipError_t factor(const LaunchCtx& c) {
  switch (c.b) {
    case 1: return c.batched ? factor_b<1, true>(c) : factor_b<1, false>(c);
    case 2: return c.batched ? factor_b<2, true>(c) : factor_b<2, false>(c);
    case 3: return c.batched ? factor_b<3, true>(c) : factor_b<3, false>(c);
    case 4: return c.batched ? factor_b<4, true>(c) : factor_b<4, false>(c);
    default: return hipErrorInvalidValue;
  }
}

template <int B, int MODE, bool BATCHED>
hipError_t bwd_b(const LaunchCtx& c, const BwdOut& o) {
  const int64_t G = groups(c.n_points, c.n_series, BATCHED);
  mark(c, kKidBwd, 0);
  hipLaunchKernelGGL((k_bwd<B, R, L, MODE, BATCHED>), dim3((unsigned)G), dim3(L), 0, c.stream, c.t, c.y,
                     c.n_points, c.hyper, make_map(c, G * L), c.lane, c.lane_ld, make_top(c, G), o);
  mark(c, kKidBwd, 1);
  return hipGetLastError();
}

template <int MODE>
hipError_t bwd_m(const LaunchCtx& c, const BwdOut& o) {
  switch (c.b) {
    case 1: return c.batched ? bwd_b<1, MODE, true>(c, o) : bwd_b<1, MODE, false>(c, o);
    case 2: return c.batched ? bwd_b<2, MODE, true>(c, o) : bwd_b<2, MODE, false>(c, o);
    case 3: return c.batched ? bwd_b<3, MODE, true>(c, o) : bwd_b<3, MODE, false>(c, o);
    case 4: return c.batched ? bwd_b<4, MODE, true>(c, o) : bwd_b<4, MODE, false>(c, o);
    default: return hipErrorInvalidValue;
  }
}

hipError_t bwd(const LaunchCtx& c, int mode, const BwdOut& o) {
  switch (mode) {
    case kWantGrad: return bwd_m<kWantGrad>(c, o);
    case kWantMean: return bwd_m<kWantMean>(c, o);
    case kWantVar: return bwd_m<kWantVar>(c, o);
    case kWantVar | kWantSub: return bwd_m<kWantVar | kWantSub>(c, o);
    case kWantLogml:
      // the per-chunk log-likelihood partials exist for several series only
      if (!c.batched) return hipErrorInvalidValue;
      switch (c.b) {
        case 1: return bwd_b<1, kWantLogml, true>(c, o);
        case 2: return bwd_b<2, kWantLogml, true>(c, o);
        case 3: return bwd_b<3, kWantLogml, true>(c, o);
        case 4: return bwd_b<4, kWantLogml, true>(c, o);
        default: return hipErrorInvalidValue;
      }
    default: return hipErrorInvalidValue;
  }
}

template <int B, bool BATCHED>
hipError_t blocks_b(const LaunchCtx& c, double* A, double* Q, double* D, double* Bs) {
  const int64_t slots = groups(c.n_points, c.n_series, BATCHED) * L;
  constexpr int T = 128;
  hipLaunchKernelGGL((k_blocks<B, R, BATCHED>), dim3((unsigned)((slots + T - 1) / T)), dim3(T), 0, c.stream, c.t,
                     c.n_points, c.hyper, make_map(c, slots), slots, A, Q, D, Bs, c.n_points);
  return hipGetLastError();
}

hipError_t blocks(const LaunchCtx& c, double* A, double* Q, double* D, double* Bs) {
  switch (c.b) {
    case 1: return c.batched ? blocks_b<1, true>(c, A, Q, D, Bs) : blocks_b<1, false>(c, A, Q, D, Bs);
    case 2: return c.batched ? blocks_b<2, true>(c, A, Q, D, Bs) : blocks_b<2, false>(c, A, Q, D, Bs);
    case 3: return c.batched ? blocks_b<3, true>(c, A, Q, D, Bs) : blocks_b<3, false>(c, A, Q, D, Bs);
    case 4: return c.batched ? blocks_b<4, true>(c, A, Q, D, Bs) : blocks_b<4, false>(c, A, Q, D, Bs);
    default: return hipErrorInvalidValue;
  }
}

const TileOps kOps = {R, L, groups, map, factor, bwd, blocks};

}  // namespace

const TileOps* SPG_TILE_FN() { return &kOps; }

}  // namespace spg
