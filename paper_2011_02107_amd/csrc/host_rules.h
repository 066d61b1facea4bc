// Host-only rules of the DACP path: parameter selection, the acceptance rule and the
// bookkeeping of the divide-and-conquer merge.  No HIP types: this part is compiled with the
// host compiler, both into the library and into the sanitizer harness of the test suite.
#pragma once

#include <cstdint>
#include <vector>

#include "../../include/dacp.h"

namespace dacp {
namespace rules {

// Estimated number of levels in [-a_r E_b, a_r E_b] from Jackson-damped Chebyshev moments of the
// density (kernel polynomial method; closed-form integral of every term).
double kpm_count(const std::vector<double> &mu, int64_t D, double a_r);
// Smallest a_r in (0, 1) whose estimated count reaches `count` (bisection).
double window_for_count(const std::vector<double> &mu, int64_t D, double count);
// Sampled evolution orders k_j = 2 floor(j pi / (2 a_r)), j = 1..n (App. B, App. C: even orders).
std::vector<int64_t> sample_orders(double a_r, int n);

// Window, filter order and basis size of one attempt (Sec. II.A, II.B, III).
struct Plan {
  double n_w, a_r, a;
  int K, b, n, m;
};
Plan make_plan(const dacp_opts &o, int64_t D, int N, double e_b, const std::vector<double> &mu, double window_ratio,
               int attempt);

// Positions of theta sorted by (|theta|, theta).
std::vector<int> central_order(const std::vector<double> &theta);

// Result of the acceptance rule (accept_rule).
struct AcceptResult {
  std::vector<char> ok, ghost;  // per Ritz value (index into theta)
  std::vector<double> est;      // per candidate position q < n_sel (INFINITY for a ghost)
  std::vector<int> core_idx;    // candidate positions of the contiguous core, walking outward
  double max_est = 0.0;
  int n_ghost = 0;
};

// Largest number of neighbouring Ritz values grouped into one cluster by accept_rule.
constexpr int kAcceptMaxCluster = 8;

// The acceptance rule (Sec. II.C residual check with a quadratic residual bound).
//   theta[r]      Ritz values, ascending
//   order         central_order(theta)
//   rnorm[n_sel]  residual norms ||H phi - theta phi|| of the unit Ritz vectors of the first n_sel
//                 positions of `order` (the candidates)
//   a, tol        window half-width and accepted error
// Rule:
//   * A candidate is a ghost when rnorm >= a - |theta|: a unit vector made only of eigenvectors
//     outside the window [-a, a] has exactly that residual or more, so such a Ritz value may
//     approximate no level at all.  Below it, Weyl's bound puts a level of H within rnorm of theta,
//     inside the window.
//   * Estimate (block quadratic residual bound): for a cluster C of consecutive non-ghost Ritz
//     values with orthonormal Ritz vectors X_C and residual block R_C, the |C| eigenvalues of H
//     paired with them lie within ||R_C||^2 / delta_C, delta_C being the distance from C to the rest
//     of the spectrum.  Here ||R_C||^2 <= sum of rnorm^2 over C, and the rest of the spectrum is
//     represented by the non-ghost Ritz values outside C (each moved towards C by its own residual,
//     zero where it is not a candidate) and by the window edges (levels beyond +-a are not
//     resolved).  The estimate of a candidate is the smallest of rnorm and this bound over every
//     run C of at most kAcceptMaxCluster candidates that contains it.  Accepted: estimate <= tol.
//   * Core: walk the candidates outward in |theta| while |theta| <= a; the first candidate that is
//     a ghost or not accepted ends it.
AcceptResult accept_rule(const std::vector<double> &theta, const std::vector<int> &order, int n_sel,
                         const std::vector<double> &rnorm, double a, double tol);

// Number of runs of at least b consecutive values of the ascending list eigs[n] in which each
// value lies within 2 tol of the next (levels of multiplicity b at the accepted accuracy).
int clusters_at_width(const double *eigs, int n, double tol, int b);

// Divide-and-conquer merge bookkeeping (host side of the rank-one update): sort the two halves'
// eigenvalues, deflate tiny z components and close pairs (Givens rotations that zero one z of
// the pair), and list the non-deflated problem.
//   dv[n]       eigenvalues of the two solved halves in block order
//   z[n]        the update vector, normalised; rho > 0 the update weight
//   lo          absolute row of the block's first eigenvector
// Outputs: sorted values ds/zs with their absolute rows rowid; defl[j] = 1 for a deflated
// sorted entry; rotations as row pairs (rot_pq) and (c, s) (rot_cs), applied in order; nd = the
// sorted positions that stay in the secular problem.
struct DcDeflation {
  std::vector<double> ds, zs;
  std::vector<int> rowid;
  std::vector<char> defl;
  std::vector<int> rot_pq;
  std::vector<double> rot_cs;
  std::vector<int> nd;
};
DcDeflation dc_deflate(const std::vector<double> &dv, const std::vector<double> &z, double rho, int lo);

// Final placement after a merge: entries (value, kind, index) with kind 0 = deflated (index = an
// absolute row) and kind 1 = secular root (index = position in the non-deflated list), sorted by
// value (stable).  Gives, per output row t of the block, where it comes from.
struct DcEntry {
  double v;
  int kind, idx;
};
struct DcPlacement {
  std::vector<int> src_defl, dst_defl;  // deflated: source absolute row -> block row
  std::vector<int> dst_of_root;         // root q -> block row
  std::vector<double> w;                // eigenvalue of block row t
};
DcPlacement dc_place(std::vector<DcEntry> ents, int k);

// Moment projection from a stored basis (App. C, Eq. shift): with T_A T_x = (T_{A+x} + T_{|A-x|}) / 2,
// the Gram block of an anchor panel of order A with a stored panel of order x gives the moment at
// one of A + x, |A - x| once the moment at the other is known (both at once when A or x is 0).
// Anchor orders for the uniform grid whose last sample is kn: 0, 1, 2, kn - 2 .. kn + 1, ascending
// and distinct.
std::vector<int64_t> anchor_orders(int64_t kn);
// The derivation chain for panel orders `orders` (orders[0] = 0, last = kn): sweeping the (anchor,
// panel) pairs until nothing new follows, each moment is derived once, from the first pair that
// reaches it; only the rules that the orders x + y, |x - y| of two panel orders need (and those
// they are derived from) are kept, in the order found, so a rule's other moment comes before it.
struct MomentChain {
  std::vector<int> table;           // per kept rule: anchor index, panel index, earlier rule or -1
  std::vector<int64_t> order;       // per kept rule: the order of the moment it gives
  std::vector<int> block_of;        // order k = 0 .. 2 kn: the kept rule giving moment k, or -1
  int64_t missing = -1;             // an order the assembly needs that the anchors do not reach
};
MomentChain moment_chain(const std::vector<int64_t> &orders, const std::vector<int64_t> &anchors);

}  // namespace rules
}  // namespace dacp
