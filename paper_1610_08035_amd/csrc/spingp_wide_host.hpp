// Internal host interface of the wide-state path between the C ABI (spingp_api.hip) and the
// per-state-dimension launch units (spingp_wide.hip, compiled once per b).  Not part of the
// public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spingp_host.hpp"      // launch-mark ids and the node step's kWant* bits
#include "spingp_sumdesc.hpp"

namespace spg {

// Wide-state path (a sum of terms, b <= 16, one series): level-by-level reduction with one
// wavefront per element operation (spingp_wide.hpp); one launch unit per state dimension.
namespace wide {
constexpr int kMaxLevels = 64;
struct WideCtx {
  hipStream_t stream;
  const double* t;
  const double* y;
  const double* hyper;
  int64_t n_points;
  double* elems;      // all tree levels, item-major
  double* msgs;       // messages of all levels, item-major
  double* cst;        // model constants of the current hyperparameters
  double* part;       // per-work-group gradient partials of the node step
  double* deriv;      // per node: the edge's transition derivatives on the support (the term's
                      // channels per entry, SumDesc::ndv doubles)
  double* edges;      // per node: the transcendental part of its edge (scalars, Matern blocks)
  double* scal;       // log-likelihood terms at the root
  int n_levels;       // level 0 = the N leaves, level n_levels - 1 = the root
  int64_t n[kMaxLevels];
  int64_t off[kMaxLevels];
  int node_grid;      // work-groups of the node step (rows of part)
  SumDesc desc;       // the model
  const unsigned long long* status;   // the status word (data errors poison the outputs)
  uint32_t gmask;     // gradient components written by finish (bit k), the others are 0
  void (*mark)(void* arg, int kid, int end);
  void* mark_arg;
};
// Launch sequences of one state dimension.
struct Ops {
  int b;
  int (*node_cap)();                                        // resident node-step work-groups
  hipError_t (*factor)(const WideCtx& c);                   // setup, leaves, up-sweep, root
  hipError_t (*down)(const WideCtx& c);                     // down-sweep of all levels
  hipError_t (*node)(const WideCtx& c, int mode, double* f_mean, double* f_var, double* z_mean, double* S_diag,
                     double* S_sub);                        // node step (kWant* bits)
  hipError_t (*finish)(const WideCtx& c, double* logml, double* grad);   // gradient sum
};
const Ops* ops(int b);   // nullptr outside 2..kMaxB
// Element and message strides (doubles per stored item) and the node step's partial row.
inline int64_t elem_stride(int b) { return (3 * b * b + 2 * b + 2 + 7) / 8 * 8; }
inline int64_t msg_stride(int b) { return (2 * b * b + 2 * b + 7) / 8 * 8; }
inline int64_t part_stride(const SumDesc& d) { return (int64_t)d.b * d.b + d.na + 1; }
void plan_levels(int64_t n, WideCtx& c);
}  // namespace wide

}  // namespace spg
