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
// Work-group caps: every team stays resident and loops over its items, so that a launch does
// not end with a second, partly empty round.  The cap is what fits on the device at once for
// the kernel's registers and LDS (the occupancy query, once per kernel and process).
template <auto K>
int resident_groups() {
  static int cached = 0;   // one instance per kernel
  if (cached == 0) {
    int dev = 0, per_cu = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, K, kW, 0) != hipSuccess || per_cu < 1 || cus < 1)
      return 1024;
    cached = per_cu * cus;
  }
  return cached;
}

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
  const int cap = with_model(c.model, [](auto m) {
    return resident_groups<k_wide_node<decltype(m), kWantGrad>>();
  });
  c.node_grid = (int)(n < cap ? n : cap);
}

template <class Model>
hipError_t factor_m(const WideCtx& c) {
  constexpr int B = Model::B;
  mark(c, kKidFwd, 0);
  hipLaunchKernelGGL(k_wide_setup<Model>, dim3(1), dim3(kW), 0, c.stream, c.hyper, c.cst);
  hipLaunchKernelGGL(k_wide_leaf<Model>, dim3(grid_for(c.n_points, resident_groups<k_wide_leaf<Model>>())), dim3(kW), 0,
                     c.stream, c.t, c.y, c.n_points, c.cst, c.elems);
  // level 1 joins leaves (rank-one node information: closed-form inverse)
  for (int k = 1; k < c.n_levels; ++k) {
    if (k == 1)
      hipLaunchKernelGGL((k_wide_up<B, true>), dim3(grid_for(c.n[k], resident_groups<k_wide_up<B, true>>())), dim3(kW),
                         0, c.stream, c.elems, c.off[k - 1], c.n[k - 1], c.off[k], c.n[k]);
    else
      hipLaunchKernelGGL((k_wide_up<B, false>), dim3(grid_for(c.n[k], resident_groups<k_wide_up<B, false>>())), dim3(kW),
                         0, c.stream, c.elems, c.off[k - 1], c.n[k - 1], c.off[k], c.n[k]);
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
  // the last level's children are leaves (rank-one node information: closed-form inverse)
  for (int k = c.n_levels - 1; k >= 1; --k) {
    if (k == 1 && c.model == kModelPeriodic)   // leaf edges: Q only in the Matern block
      hipLaunchKernelGGL((k_wide_down<B, true, true>),
                         dim3(grid_for(c.n[k - 1], resident_groups<k_wide_down<B, true, true>>())), dim3(kW), 0,
                         c.stream, c.elems, c.msgs, c.off[k], c.off[k - 1], c.n[k - 1]);
    else if (k == 1)
      hipLaunchKernelGGL((k_wide_down<B, true>), dim3(grid_for(c.n[k - 1], resident_groups<k_wide_down<B, true>>())),
                         dim3(kW), 0, c.stream, c.elems, c.msgs, c.off[k], c.off[k - 1], c.n[k - 1]);
    else
      hipLaunchKernelGGL((k_wide_down<B, false>), dim3(grid_for(c.n[k - 1], resident_groups<k_wide_down<B, false>>())),
                         dim3(kW), 0, c.stream, c.elems, c.msgs, c.off[k], c.off[k - 1], c.n[k - 1]);
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
