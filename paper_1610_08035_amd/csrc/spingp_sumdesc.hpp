// Runtime description of a sum of covariance terms for the wide-state path (shared by the host
// code that builds it and the kernels that read it).  The state is block diagonal, one block
// per term, in the order of the term list (Sec. 2.1: a sum of independent processes).
#pragma once
#include <stdint.h>

namespace spg {
namespace wide {

constexpr int kMaxTerms = 8;
constexpr int kMaxB = 16;         // one 16 x 16 matrix-core tile per product
constexpr int kMaxJobs = 32;      // transcendental scalars of one edge
constexpr int kMaxBlk = 192;      // Matern edge blocks (3 m^2 per term, sum of m^2 <= 4 b)
constexpr int kMaxSupport = 128;  // two per lane of a 64-lane team
constexpr int kMaxChannels = 16;  // derivative channels (at most two per term)
constexpr int kMaxSqExpOrder = 10;  // squared exponential: even orders 2..10

enum : int { kTermMatern = 0, kTermPeriodic = 1, kTermQuasi = 2, kTermSqExp = 3 };

struct TermInfo {
  int type;    // kTerm*
  int order;   // Matern: block size m (nu = m - 1/2); periodic and quasi-periodic: harmonics J
               // (block 2 (J + 1)); squared exponential: approximation order n (block n)
  int s0;      // first state of the block
  int n;       // block size
  int h0;      // first hyperparameter of the term in the row
  int ch0;     // first derivative channel: Matern lam, periodic period, quasi-periodic period
               // and decay (two), squared exponential lam
  int nch;     // channels of the term (1 or 2)
  int c0;      // first model constant of the term
  int sup0;    // first support entry (transition entries with a derivative)
  int nsup;    // support entries: the whole block (Matern, squared exponential) or the 2 x 2
               // harmonic blocks (periodic, quasi-periodic)
  int job0;    // first edge scalar: cos and sin of each harmonic's angle and exp(-dt / l_D)
               // (quasi-periodic), e^{r_k lam dt} of each root (squared exp.); a Matern term's one
               // job forms its whole block
  int njob;
  int blk0;    // Matern: its edge block (A, Q, dA/dlam, m^2 each) in the edge scratch
  int dv0;     // first stored transition derivative: the term's support entries, nch values each
};

struct SumDesc {
  int nt;           // terms
  int b;            // state dimension
  int nh;           // hyperparameters per series (the terms', then the noise variance)
  int na;           // derivative channels
  int ns;           // support entries
  int ndv;          // stored transition derivatives per node (support entries x their channels)
  int njob;         // edge scalars
  int nblk;         // doubles of the Matern edge blocks
  uint32_t obs;     // bit k: state k is observed (h_k = 1)
  int has_se;       // some term is a squared exponential (its Q is formed as P0 - A P0 A^T)
  int q2;           // every leaf Q lies in the leading 2 x 2 block (Matern-1/2 or -3/2 first,
                    // periodic terms after): closed-form inverses on the leaf edges
  // constants block: s2, the terms' constants, per-state output scale, P0' (working basis),
  // P0 (original basis)
  int kS2, kScale, kP0, kP0o, kConst;
  TermInfo t[kMaxTerms];
};

}  // namespace wide
}  // namespace spg
