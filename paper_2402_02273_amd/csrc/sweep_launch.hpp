// Launch side of the stencil sweeps: the sweep kernels over a tiling and the
// host dispatch on dtype, boundary, term flavour and planes per thread.
// stencil.hip instantiates it for the operator, the right-hand side and the
// Taylor terms of A; stencil_lin.hip for the Taylor terms of the linearised
// operator, so the two sets of kernels compile in parallel.
#pragma once

#include "internal.hpp"
#include "sweep_device.hpp"

namespace expint {

// One sweep over a bx x by patch of lp consecutive x-planes (see
// sweep_column for the per-thread work).
template <typename T, int BC, int LP, int KIND, int FL>
__global__ __launch_bounds__(kBlock) void k_sweep(Geom g, FastDiv gx, FastDiv gy, Coef cf, SweepArgs a) {
  __shared__ LdsCoef<T> s;
  load_tables(s, cf, threadIdx.y * blockDim.x + threadIdx.x, kBlock);
  __syncthreads();
  const int L = xcd_remap(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
  const int t = static_cast<int>(gx.div(static_cast<uint32_t>(L)));
  const int bxi = L - t * static_cast<int>(gx.d);
  const int xg = static_cast<int>(gy.div(static_cast<uint32_t>(t)));
  const int byi = t - xg * static_cast<int>(gy.d);
  const int i0 = xg * LP;
  const int j = byi * static_cast<int>(blockDim.y) + static_cast<int>(threadIdx.y);
  const int k = bxi * static_cast<int>(blockDim.x) + static_cast<int>(threadIdx.x);
  if (j >= g.ny || k >= g.nz) return;
  sweep_column<T, BC, LP, KIND, FL>(g, cf, s, a, i0, j, k, LP);
}

// The z-vectorised sweep (sweep_column4): workgroup = 256 / rw rows of one
// z-segment of rw lanes, lp planes; NT: Taylor-term outputs by non-temporal
// stores.
template <typename T, int BC, int LP, int KIND, int FL, bool NT>
__global__ __launch_bounds__(kBlock) void k_sweep4(Geom g, ColumnGrid cg, Coef cf, SweepArgs a) {
  __shared__ LdsCoef<T> s;
  const int L = xcd_remap(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
  const int tid = static_cast<int>(threadIdx.x);
  const ColumnTile c = column_tile(cg, L, LP, tid);
  const int i0 = c.i0, kq = c.kq, j = c.j, k4 = c.k4, rw = cg.rw;
  // the class table is staged after the first field loads are in flight
  auto ready = [&]() {
    load_tables(s, cf, tid, kBlock);
    __syncthreads();
  };
  const bool live = j < g.ny && k4 < (g.nz >> 2);
  sweep_column4<T, BC, LP, KIND, FL, NT>(g, cf.labels, s, a, i0, j, k4, kq, rw, live, ready);
}

template <typename T, int BC, int KIND, int FL>
static void sweep_lp(const Geom& g, const Tiling& tl, const Coef& cf, const SweepArgs& a, hipStream_t st) {
  if (tl.vec) {
    const int rows = kBlock / tl.rw;
    const ColumnGrid cg(((g.nz >> 2) + tl.rw - 1) / tl.rw, (g.ny + rows - 1) / rows, tl.rw);
    const dim3 grid(static_cast<unsigned>(sweep_blocks(g, tl))), block(kBlock);
    // the store policy applies to the Taylor terms of A; those of the
    // linearised operator were measured slower with non-temporal stores
    if constexpr (KIND == kTerm) {
      if (tl.nt) {
        switch (tl.lp) {
          case 1: k_sweep4<T, BC, 1, KIND, FL, true><<<grid, block, 0, st>>>(g, cg, cf, a); break;
          case 2: k_sweep4<T, BC, 2, KIND, FL, true><<<grid, block, 0, st>>>(g, cg, cf, a); break;
          default: k_sweep4<T, BC, 4, KIND, FL, true><<<grid, block, 0, st>>>(g, cg, cf, a); break;
        }
        return;
      }
    }
    switch (tl.lp) {
      case 1: k_sweep4<T, BC, 1, KIND, FL, false><<<grid, block, 0, st>>>(g, cg, cf, a); break;
      case 2: k_sweep4<T, BC, 2, KIND, FL, false><<<grid, block, 0, st>>>(g, cg, cf, a); break;
      default: k_sweep4<T, BC, 4, KIND, FL, false><<<grid, block, 0, st>>>(g, cg, cf, a); break;
    }
    return;
  }
  const FastDiv gx(static_cast<uint32_t>((g.nz + tl.bx - 1) / tl.bx)), gy(static_cast<uint32_t>((g.ny + tl.by - 1) / tl.by));
  const dim3 grid(static_cast<unsigned>(sweep_blocks(g, tl))), block(tl.bx, tl.by);
  switch (tl.lp) {
    case 1: k_sweep<T, BC, 1, KIND, FL><<<grid, block, 0, st>>>(g, gx, gy, cf, a); break;
    case 2: k_sweep<T, BC, 2, KIND, FL><<<grid, block, 0, st>>>(g, gx, gy, cf, a); break;
    default: k_sweep<T, BC, 4, KIND, FL><<<grid, block, 0, st>>>(g, gx, gy, cf, a); break;
  }
}

template <typename T, int BC, int KIND>
static void sweep_typed(const Geom& g, const Tiling& tl, const Coef& cf, const SweepArgs& a, hipStream_t st) {
  if (!is_term(KIND)) {
    sweep_lp<T, BC, KIND, kGeneric>(g, tl, cf, a, st);
    return;
  }
  switch (a.op.flavor) {
    case kSkip: sweep_lp<T, BC, KIND, kSkip>(g, tl, cf, a, st); break;
    case kFlushY: sweep_lp<T, BC, KIND, kFlushY>(g, tl, cf, a, st); break;
    case kFlushNoY: sweep_lp<T, BC, KIND, kFlushNoY>(g, tl, cf, a, st); break;
    case kFirst: sweep_lp<T, BC, KIND, kFirst>(g, tl, cf, a, st); break;
    default: sweep_lp<T, BC, KIND, kGeneric>(g, tl, cf, a, st); break;
  }
}

// Whether every field the sweep touches starts on a 4-value boundary (the
// z-vectorised sweep moves 4-value vectors; caller buffers may be views).
inline bool vec_aligned(int kind, const SweepArgs& a, const Coef& cf, expint_dtype dt) {
  const uintptr_t m = 4 * dtype_bytes(dt) - 1;
  auto ok = [m](const void* p) { return (reinterpret_cast<uintptr_t>(p) & m) == 0; };
  if ((reinterpret_cast<uintptr_t>(cf.labels) & 3) != 0) return false;
  if (is_term(kind))
    return ok(a.op.src) && ok(a.op.bsrc) && ok(a.op.acc_in) && ok(a.op.y_out) && ok(a.op.acc_out) && ok(a.op.u) &&
           ok(a.op.ju) && ok(a.op.bsrc2);
  return ok(a.x) && ok(a.out) && ok(a.aux0) && ok(a.aux1);
}

template <int KIND>
static hipError_t sweep(expint_dtype dt, expint_bc bc, const Geom& g, const Tiling& tl_in, const Coef& cf,
                        const SweepArgs& a, hipStream_t st) {
  if (!tiling_valid(tl_in) || (tl_in.vec && !vec_sweep_ok(g, cf.labels_form))) return hipErrorInvalidValue;
  // a misaligned field takes the scalar sweep for this launch
  const Tiling tl = tl_in.vec && !vec_aligned(KIND, a, cf, dt) ? default_tiling(g) : tl_in;
  if (dt == EXPINT_F64) {
    if (bc == EXPINT_NOFLUX) sweep_typed<double, 0, KIND>(g, tl, cf, a, st);
    else sweep_typed<double, 1, KIND>(g, tl, cf, a, st);
  } else {
    if (bc == EXPINT_NOFLUX) sweep_typed<float, 0, KIND>(g, tl, cf, a, st);
    else sweep_typed<float, 1, KIND>(g, tl, cf, a, st);
  }
  return hipGetLastError();
}

}  // namespace expint
