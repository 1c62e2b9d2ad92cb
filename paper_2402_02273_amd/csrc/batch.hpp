// Descriptors of the batched sweeps (host and device).
#pragma once

#include "internal.hpp"

namespace expint {

// One instance of a batch, as the batched kernel sees it.
struct BatchInst {
  Geom g;
  int bx, by, lp;  // tile: bx (z) x by (y) threads, lp x-planes per thread
  int gx, gy;      // tiles along z and y
  int nblocks;     // tiles of one sweep
  Coef coef;       // label form
  double rho;
};

// One sweep of one instance inside a launch.  For a right-hand-side launch,
// op.src is u and op.y_out is b.
struct BatchOp {
  int inst;
  int block_start;  // offset of this instance's tiles in the launch's work list
  TermOp op;
};

hipError_t launch_batch(expint_dtype dt, expint_bc bc, bool rhs, const BatchInst* insts, const BatchOp* ops, int nops,
                        int total_blocks, int grid, hipStream_t st);

}  // namespace expint
