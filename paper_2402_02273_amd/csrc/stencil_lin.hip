// Taylor-term sweeps of the linearised operator J = A + rho diag(1 - 2 u_n)
// (section 2.1 moves the part of the reaction that is linear in the new state
// into the matrix; the step of section 2.2 then applies phi1 to J).  Same
// kernels as the Taylor terms of A with one more field read per sweep, u_n,
// at the voxel being written.

#include "internal.hpp"
#include "sweep_launch.hpp"

namespace expint {

hipError_t launch_term_lin(expint_dtype dt, expint_bc bc, const Geom& g, const Tiling& tl, const Coef& cf,
                           const TermOp& op, hipStream_t st) {
  if (!op.ju || op.pair) return hipErrorInvalidValue;
  SweepArgs a{};
  a.op = op;
  return sweep<kTermJ>(dt, bc, g, tl, cf, a, st);
}

}  // namespace expint
