// Launch sequence of the wide-state path (see spingp_wide.hpp).
#include "spingp_host.hpp"
#include "spingp_wide.hpp"

namespace spg {
namespace wide {
namespace {

using ModelP = SumM32Periodic<3, false>;               // Matern-3/2 + periodic
using ModelQ = SumM32Periodic<3, true>;                // Matern-3/2 + quasi-periodic
using ModelS = SumM32Periodic<3, true, kSqExpOrder>;   // ... + squared exponential
static_assert(ModelP::B == ModelQ::B, "one state dimension for the two b = 10 models");
// Work-group caps: what fits on the 256 CUs at once for each kernel's LDS and registers, so
// that every team stays resident and loops over its items instead of a launch ending with a
// second, partly empty round.  b = 10: up 11 KB and 148 VGPRs (12 per CU; level 1 98 VGPRs,
// 14), down 10 KB and 128 VGPRs (16), node 14 KB and 213 VGPRs (8), leaf 16 per CU.  b = 16: up
// 28 KB and 256 VGPRs (4 per CU; level 1 210 VGPRs, 5), down 24 KB (6), node 39 KB and 256
// VGPRs (4), leaf 15 KB (10).
struct Caps {
  int up, up1, down, leaf, node;   // up1: the up-sweep's first level
};
constexpr Caps kCaps10 = {3072, 3584, 4096, 4096, 2048};
constexpr Caps kCaps16 = {1024, 1280, 1536, 2560, 1024};
inline const Caps& caps(int model) { return model == kModelQuasiSqExp ? kCaps16 : kCaps10; }

inline void mark(const WideCtx& c, int kid, int end) {
  if (c.mark) c.mark(c.mark_arg, kid, end);
}
inline unsigned grid_for(int64_t items, int cap) { return (unsigned)(items < cap ? items : cap); }

}  // namespace

// Calls f with a value of the model's type.
template <class F>
auto with_model(int model, F&& f) {
  if (model == kModelQuasiSqExp) return f(ModelS());
  if (model == kModelQuasi) return f(ModelQ());
  return f(ModelP());
}

int state_dim(int model) {
  return with_model(model, [](auto m) { return decltype(m)::B; });
}
int n_hyper(int model) {
  return with_model(model, [](auto m) { return decltype(m)::NH; });
}
int64_t elem_stride(int model) {
  return with_model(model, [](auto m) { return (int64_t)Lay<decltype(m)::B>::kEs; });
}
int64_t msg_stride(int model) {
  return with_model(model, [](auto m) { return (int64_t)Lay<decltype(m)::B>::kMs; });
}
int64_t const_size(int model) {
  return with_model(model, [](auto m) { return (int64_t)decltype(m)::kConst; });
}
int64_t part_stride(int model) {
  return with_model(model, [](auto m) { return (int64_t)decltype(m)::kPart; });
}

void plan_levels(int64_t n, WideCtx& c) {
  int k = 0;
  int64_t off = 0;
  for (int64_t m = n;; m = (m + 1) / 2) {
    c.n[k] = m;
    c.off[k] = off;
    off += m;
    ++k;
    if (m == 1 || k == kMaxLevels) break;
  }
  c.n_levels = k;
  const int cap = caps(c.model).node;
  c.node_grid = (int)(n < cap ? n : cap);
}

template <class Model>
hipError_t factor_m(const WideCtx& c) {
  constexpr int B = Model::B;
  mark(c, kKidFwd, 0);
  hipLaunchKernelGGL(k_wide_setup<Model>, dim3(1), dim3(kW), 0, c.stream, c.hyper, c.cst);
  const Caps& cp = caps(c.model);
  hipLaunchKernelGGL(k_wide_leaf<Model>, dim3(grid_for(c.n_points, cp.leaf)), dim3(kW), 0, c.stream, c.t, c.y, c.n_points,
                     c.cst, c.elems);
  // level 1 joins leaves (rank-one node information: closed-form inverse)
  for (int k = 1; k < c.n_levels; ++k) {
    if (k == 1)
      hipLaunchKernelGGL((k_wide_up<B, true>), dim3(grid_for(c.n[k], cp.up1)), dim3(kW), 0, c.stream, c.elems,
                         c.off[k - 1], c.n[k - 1], c.off[k], c.n[k]);
    else
      hipLaunchKernelGGL((k_wide_up<B, false>), dim3(grid_for(c.n[k], cp.up)), dim3(kW), 0, c.stream, c.elems,
                         c.off[k - 1], c.n[k - 1], c.off[k], c.n[k]);
  }
  mark(c, kKidFwd, 1);
  mark(c, kKidTop, 0);
  hipLaunchKernelGGL(k_wide_root<Model>, dim3(1), dim3(kW), 0, c.stream, c.cst, c.elems, c.off[c.n_levels - 1],
                     c.msgs, c.scal);
  mark(c, kKidTop, 1);
  return hipGetLastError();
}

hipError_t factor(const WideCtx& c) {
  return with_model(c.model, [&](auto m) { return factor_m<decltype(m)>(c); });
}

template <int B>
static void down_b(const WideCtx& c) {
  const int cap = caps(c.model).down;
  // the last level's children are leaves (rank-one node information: closed-form inverse)
  for (int k = c.n_levels - 1; k >= 1; --k) {
    if (k == 1 && c.model == kModelPeriodic)   // leaf edges: Q only in the Matern block
      hipLaunchKernelGGL((k_wide_down<B, true, true>), dim3(grid_for(c.n[k - 1], cap)), dim3(kW), 0, c.stream,
                         c.elems, c.msgs, c.off[k], c.off[k - 1], c.n[k - 1]);
    else if (k == 1)
      hipLaunchKernelGGL((k_wide_down<B, true>), dim3(grid_for(c.n[k - 1], cap)), dim3(kW), 0, c.stream, c.elems,
                         c.msgs, c.off[k], c.off[k - 1], c.n[k - 1]);
    else
      hipLaunchKernelGGL((k_wide_down<B, false>), dim3(grid_for(c.n[k - 1], cap)), dim3(kW), 0, c.stream, c.elems,
                         c.msgs, c.off[k], c.off[k - 1], c.n[k - 1]);
  }
}

hipError_t down(const WideCtx& c) {
  mark(c, kKidBwd, 0);
  if (c.model == kModelQuasiSqExp)
    down_b<ModelS::B>(c);
  else
    down_b<ModelP::B>(c);
  mark(c, kKidBwd, 1);
  return hipGetLastError();
}

template <int MODE>
static void launch_node(const WideCtx& c, const WideOut& o) {
  with_model(c.model, [&](auto m) {
    hipLaunchKernelGGL((k_wide_node<decltype(m), MODE>), dim3((unsigned)c.node_grid), dim3(kW), 0, c.stream, c.t,
                       c.y, c.n_points, c.cst, c.elems, c.msgs, o);
    return 0;
  });
}

hipError_t node(const WideCtx& c, int mode, double* f_mean, double* f_var, double* z_mean, double* S_diag,
                double* S_sub) {
  WideOut o;
  o.f_mean = f_mean;
  o.f_var = f_var;
  o.z_mean = z_mean;
  o.S_diag = S_diag;
  o.S_sub = S_sub;
  o.ld = c.n_points;
  o.part = c.part;
  o.status = c.status;
  mark(c, kKidBwd, 0);
  switch (mode) {
    case kWantGrad: launch_node<kWantGrad>(c, o); break;
    case kWantMean: launch_node<kWantMean>(c, o); break;
    case kWantVar: launch_node<kWantVar>(c, o); break;
    case kWantVar | kWantSub: launch_node<kWantVar | kWantSub>(c, o); break;
    default: return hipErrorInvalidValue;
  }
  mark(c, kKidBwd, 1);
  return hipGetLastError();
}

template <class Model>
hipError_t finish_m(const WideCtx& c, double* logml, double* grad) {
  mark(c, kKidReduce, 0);
  // the totals follow the rows of all node work-groups
  double* tot = c.part + (int64_t)c.node_grid * Model::kPart;
  hipLaunchKernelGGL(k_wide_sum<Model>, dim3((unsigned)Model::kPart), dim3(kW), 0, c.stream, c.part, c.node_grid,
                     tot);
  hipLaunchKernelGGL(k_wide_final<Model>, dim3(1), dim3(kW), 0, c.stream, c.cst, tot, c.scal, logml, grad, c.status,
                     c.gmask);
  mark(c, kKidReduce, 1);
  return hipGetLastError();
}

hipError_t finish(const WideCtx& c, double* logml, double* grad) {
  return with_model(c.model, [&](auto m) { return finish_m<decltype(m)>(c, logml, grad); });
}

}  // namespace wide
}  // namespace spg
