// The sequence of fused Taylor-term sweeps that evaluates
// x = tau phi1(tau A) b (section 2.2).
//
// exp(tau B) applied to the augmented unit vector, B = [[A, b], [0, 0]], is
// evaluated as s factors of the degree-m Taylor polynomial T_m(h B),
// h = tau / s.  One factor maps [x; 1] to [x + y_1 + ... + y_m; 1] with
//   y_1 = h (A x + b),   y_j = (h / j) A y_{j-1},
// starting from x = 0.  Each y_j costs one application of A, fused with the
// running sum in a single sweep (TermOp).  Two algebraic shortcuts remove the
// sweeps that would apply A to the zero vector:
//   - sub-step 1, term 1: y_1 = h b, so term 2 is (h^2/2) A b with the sum
//     started at h b;
//   - if m == 1, sub-step 1 leaves x = h b and sub-step 2 computes
//     y_1 = h^2 A b + h b with the sum started at h b.
// The last sweep either adds the sum into u (the step u + x) or stores it.
//
// With a second vector d the same sweeps evaluate
// x = tau phi1(tau A) b + tau phi2(tau A) d: the augmented matrix then fills
// both columns of its omega block, [d / tau, b], next to the nilpotent block
// J = [[0, 1], [0, 0]], and the augmented unit vector starts at eta = (0, 1).
// eta after k sub-steps is (k h, 1), so one sub-step's terms become
//   y_1 = h (A x + b + (k h / tau) d),   y_2 = (h/2) A y_1 + (h^2 / (2 tau)) d,
//   y_j = (h / j) A y_{j-1} (j >= 3);
// d enters two sweeps per sub-step as a second source (TermOp::bsrc2).  With
// m = 1 the phi2 part is truncated away entirely.
#pragma once

#include <vector>

#include "internal.hpp"

namespace expint {

struct StepBuffers {
  void* b = nullptr;
  void* y[2] = {nullptr, nullptr};
  void* acc[2] = {nullptr, nullptr};
};

// b: the vector phi1 acts on; d (may be NULL): the vector phi2 acts on.
// Exactly one of x_out (store the result) and u (add the result into u) is
// non-NULL.
std::vector<TermOp> phi1_schedule(const StepBuffers& ws, int s, int m, double tau, const void* b, void* x_out,
                                  void* u, const void* d = nullptr);

// The same polynomial with the terms of every sub-step taken two at a time
// by pair sweeps (TermOp::pair; label form, m >= 2): sub-step terms
// (1, 2), (3, 4), ... (terms (2, 3), (4, 5), ... in sub-step 1, whose term 1
// is h b), and a single-term sweep for a term left over at the end.  The
// running sum gains two terms per sweep.
std::vector<TermOp> phi1_schedule_pairs(const StepBuffers& ws, int s, int m, double tau, const void* b,
                                        void* x_out, void* u);

// Turns every sweep of a schedule into a sweep of the linearised operator
// J = A + rho diag(1 - 2 u_n) (TermOp::ju), so the schedule evaluates
// x = tau phi1(tau J) b.  un is read at each voxel by the sweep that writes
// that voxel only, so it may be the u the last sweep adds into.
void set_linearised(std::vector<TermOp>& ops, const void* un, double rho);

}  // namespace expint
