// Tile-shape selection for the stencil sweeps.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace expint {

// Times every valid (bx, lp) tiling of the Taylor-term sweep for this grid,
// dtype, boundary and coefficient form on `st`, using the three scratch fields
// (each g.n values of dtype; their contents are overwritten), and returns the
// fastest.  Results are cached per (grid, dtype, bc, form) for the process.
// EXPINT_AUTOTUNE=0 in the environment skips the search (default_tiling).
hipError_t autotune_sweep(expint_dtype dt, expint_bc bc, const Geom& g, const Coef& cf, void* f0, void* f1, void* f2,
                          hipStream_t st, Tiling* out);

}  // namespace expint
