// Descriptors of the batched sweeps (host and device).
#pragma once

#include "internal.hpp"

namespace expint {

constexpr int kBatchMaxOps = 64;  // ops per batched launch (the host splits larger ones)

// One sweep of one instance inside a launch, with everything the kernel
// needs about that instance.  For a right-hand-side launch, op.src is u and
// op.y_out is b.
struct BatchItem {
  int block_start;      // offset of this instance's tiles in the launch's work list
  int nx, ny, nz;
  FastDiv gx, gy;       // tiles along z and y (divisors of the tile index)
  int by;               // rows (y) per tile
  int bx, bx_log2;      // threads along z (16, 32 or 64); vec: lanes per z-segment
  int vec;              // vec: z-vectorised sweep (gx = z-segments)
  const uint8_t* labels;
  double rho;
  TermOp op;
};

// One launch over items[0 .. nitems) (nitems <= kBatchMaxOps): all of them
// right-hand sides (rhs) or all Taylor terms of the given flavour (lin: of
// the linearised operator, TermOp::ju set in every item); every instance
// involved uses lp planes per thread.  tables: per item the class table (64
// values) followed by the wall table (8 values), in the dtype.
hipError_t launch_batch(expint_dtype dt, expint_bc bc, bool rhs, bool lin, int flavor, int lp,
                        const BatchItem* items, const void* tables, int nitems, int total_blocks, int grid,
                        hipStream_t st);

}  // namespace expint
