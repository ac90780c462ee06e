// Launch sequence of the wide-state path for one state dimension (see spingp_wide.hpp).
// Compiled once per b with -DSPG_WIDE_B=<b>; each object exports spg::wide::ops_b<b>().
#include "spingp_wide_host.hpp"
#include "spingp_wide.hpp"

#ifndef SPG_WIDE_B
#error "SPG_WIDE_B must be defined"
#endif

#define SPG_WCAT2(a, b) a##b
#define SPG_WCAT(a, b) SPG_WCAT2(a, b)
#define SPG_WIDE_FN SPG_WCAT(ops_b, SPG_WIDE_B)

namespace spg {
namespace wide {
namespace {

constexpr int B = SPG_WIDE_B;

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

int node_cap() { return resident_groups<k_wide_node<B, kWantGrad>>(); }

hipError_t factor(const WideCtx& c) {
  const SumDesc& d = c.desc;
  mark(c, kKidFwd, 0);
  hipLaunchKernelGGL(k_wide_setup<B>, dim3(1), dim3(kW), 0, c.stream, d, c.hyper, c.cst);
  hipLaunchKernelGGL(k_wide_edges<B>, dim3((unsigned)((c.n_points + kEdgeThreads - 1) / kEdgeThreads)),
                     dim3(kEdgeThreads), 0, c.stream, d, c.t, c.n_points, c.cst, c.edges);
  hipLaunchKernelGGL(k_wide_leaf<B>, dim3(grid_for(c.n_points, resident_groups<k_wide_leaf<B>>())), dim3(kW), 0,
                     c.stream, d, c.t, c.y, c.n_points, c.cst, c.edges, c.elems, c.deriv);
  // level 1 joins leaves (rank-one node information: closed-form inverse)
  for (int k = 1; k < c.n_levels; ++k) {
    if (k == 1)
      hipLaunchKernelGGL((k_wide_up<B, true>), dim3(grid_for(c.n[k], resident_groups<k_wide_up<B, true>>())), dim3(kW),
                         0, c.stream, c.elems, c.off[k - 1], c.n[k - 1], c.off[k], c.n[k]);
    else
      hipLaunchKernelGGL((k_wide_up<B, false>), dim3(grid_for(c.n[k], resident_groups<k_wide_up<B, false>>())),
                         dim3(kW), 0, c.stream, c.elems, c.off[k - 1], c.n[k - 1], c.off[k], c.n[k]);
  }
  mark(c, kKidFwd, 1);
  mark(c, kKidTop, 0);
  hipLaunchKernelGGL(k_wide_root<B>, dim3(1), dim3(kW), 0, c.stream, d, c.cst, c.elems, c.off[c.n_levels - 1],
                     c.msgs, c.scal);
  mark(c, kKidTop, 1);
  return hipGetLastError();
}

hipError_t down(const WideCtx& c) {
  mark(c, kKidBwd, 0);
  // the last level's children are leaves (rank-one node information: closed-form inverse)
  for (int k = c.n_levels - 1; k >= 1; --k) {
    if (k == 1 && c.desc.q2)   // leaf edges: Q only in the leading 2 x 2 block
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
  mark(c, kKidBwd, 1);
  return hipGetLastError();
}

template <int MODE>
void launch_node(const WideCtx& c, const WideOut& o) {
  hipLaunchKernelGGL((k_wide_node<B, MODE>), dim3((unsigned)c.node_grid), dim3(kW), 0, c.stream, c.desc, c.t, c.y,
                     c.n_points, c.cst, c.elems, c.msgs, c.deriv, o);
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

hipError_t finish(const WideCtx& c, double* logml, double* grad) {
  mark(c, kKidReduce, 0);
  // the totals follow the rows of all node work-groups
  const int kPart = B * B + c.desc.na + 1;
  double* tot = c.part + (int64_t)c.node_grid * kPart;
  hipLaunchKernelGGL(k_wide_sum<B>, dim3((unsigned)kPart), dim3(kW), 0, c.stream, c.part, c.node_grid, kPart, tot);
  hipLaunchKernelGGL(k_wide_final<B>, dim3(1), dim3(kW), 0, c.stream, c.desc, c.cst, tot, c.scal, logml, grad,
                     c.status, c.gmask);
  mark(c, kKidReduce, 1);
  return hipGetLastError();
}

const Ops kOps = {B, node_cap, factor, down, node, finish};

}  // namespace

const Ops* SPG_WIDE_FN() { return &kOps; }

}  // namespace wide
}  // namespace spg
