// Tile-shape selection for the stencil sweeps.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace expint {

// Times every valid tiling of the Taylor-term sweep for this grid, dtype,
// boundary and coefficient form on `st` -- (bx, lp) of the scalar sweep and,
// if allow_vec and the grid qualifies, (rw, lp) of the z-vectorised sweep --
// using the three scratch fields (each g.n values of dtype; their contents are
// overwritten), and returns the fastest.  For a z-vectorised winner the final
// choice is made on a dependent pair as in a step (a skip sweep writes a term,
// a flush sweep reads it back): every vector shape within 10% of the best,
// with plain and with non-temporal output stores of the Taylor terms (best of
// three alternating rounds); non-temporal stores must be at least 2% faster
// (Tiling::nt).
// Results are cached per (grid, dtype, bc, form, candidate set) for the
// process.  EXPINT_AUTOTUNE=0 in the
// environment skips the search (default_tiling); EXPINT_TILE=scalar or vec
// restricts the candidates to one sweep shape; EXPINT_TUNE_FILE=path keeps
// the choices in a text file that later processes read instead of timing.
// ju (n values of dtype, overwritten) selects the Taylor sweeps of the
// linearised operator J = A + jrho diag(1 - 2 ju) instead, which a linearised
// step runs: those read u_n as well and keep plain stores, so they are tuned
// apart (their own cache and tuning-file key: flags bit 8).
// vec_only: where the grid allows the z-vectorised shape, time only those
// shapes (the batch: its batched scalar sweeps lose more against the vector
// ones than single-grid timings show).
hipError_t autotune_sweep(expint_dtype dt, expint_bc bc, const Geom& g, const Coef& cf, void* f0, void* f1, void* f2,
                          hipStream_t st, bool allow_vec, Tiling* out, void* ju = nullptr, double jrho = 0.0,
                          bool vec_only = false);

// The flags of the key autotune_sweep files its choice for this grid under
// (bit 1 label form, 2 z-vectorised shapes timed, 4 scalar shapes timed,
// 8 linearised operator); they follow EXPINT_TILE as the search does.
int autotune_key_flags(const Geom& g, const Coef& cf, bool allow_vec, bool ju, bool vec_only);

// A tiling chosen in a wider context than one grid's sweeps (a batch times
// whole steps of all its grids), kept in the same process cache and tuning
// file under (grid, dtype, bc, flags); the caller sets a flags bit of its own
// (16 for the batch) on top of autotune_key_flags.  autotune_find reads the
// tuning file first, as autotune_sweep does, and returns false if there is
// no entry; autotune_keep stores and appends one.
bool autotune_find(expint_dtype dt, expint_bc bc, const Geom& g, int flags, Tiling* out);
void autotune_keep(expint_dtype dt, expint_bc bc, const Geom& g, int flags, const Tiling& t);

// Decides whether the step takes its Taylor terms two at a time (pair
// sweeps, label form only) and with which tiling.  mode SINGLE: never (ty = 0
// in *out).  PAIRS: always, in the fastest pair tiling.  AUTO: times every
// pair tiling against a single-term skip sweep plus a flush sweep in the
// tiling `single` and keeps the pair sweeps if the fastest is quicker than
// those two.  Dense-form coefficients always get ty = 0.  Cached per (grid,
// dtype, bc, mode) for the process.  EXPINT_AUTOTUNE=0 in the environment
// skips the timing: pairs (ty = 8, lp = 8) unless mode is SINGLE.
hipError_t autotune_pairs(expint_dtype dt, expint_bc bc, const Geom& g, const Coef& cf, void* f0, void* f1, void* f2,
                          hipStream_t st, const Tiling& single, expint_sweeps mode, PairTiling* out);

}  // namespace expint
