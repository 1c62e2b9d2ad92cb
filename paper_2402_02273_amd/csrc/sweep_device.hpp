// Device-side building blocks of the stencil sweeps, shared by the
// single-grid kernels (stencil.hip) and the batched kernel (batch.hip).
//
// A sweep thread owns one (j, k) column of a tile and marches through lp
// consecutive x-planes, keeping the x-1 / x / x+1 values (and labels) of the
// source field in registers; the four lateral neighbours are plain loads
// served by L1/L2.  Neighbour indices outside the box are clamped to the voxel
// itself, so the difference x_q - x_p of a wall face is exactly 0 (zero flux,
// the paper's no-flux boundary) and every load is unconditional; zero-
// Dirichlet walls add -D_p/h^2 x_p per wall face instead.  The operator is the
// conservative 7-point form of div(D grad u) (section 2.1) with harmonic face
// means from the class-pair table.
#pragma once

#include "internal.hpp"

namespace expint {

template <typename T>
struct LdsCoef {
  T tab[kTab];
  T wall[kMaxClasses];
};

// Copies the class-pair table into LDS (label form); thread t of nthreads.
// The caller synchronises afterwards.
template <typename T>
__device__ __forceinline__ void load_tables(LdsCoef<T>& s, const Coef& cf, int t, int nthreads) {
  if (cf.labels_form) {
    for (int i = t; i < kTab; i += nthreads) s.tab[i] = static_cast<const T*>(cf.tab)[i];
    if (t < kMaxClasses) s.wall[t] = static_cast<const T*>(cf.wallc)[t];
  }
}

enum SweepKind { kTerm = 0, kRhs = 1, kApply = 2, kAdjRhs = 3 };
constexpr int kRuntimeFlavor = -1;

struct SweepArgs {
  TermOp op;          // kTerm
  const void* x;      // kRhs / kApply / kAdjRhs stencil input
  void* out;          // kRhs / kApply / kAdjRhs output
  const void* aux0;   // kAdjRhs: lambda in
  const void* aux1;   // kAdjRhs: u
  double rho;         // kRhs / kAdjRhs
};

// Outputs of one Taylor-term sweep at voxel q (see TermOp).
template <typename T, int FL>
__device__ __forceinline__ void term_store(const TermOp& op, int q, T ax, T xc) {
  const T c = static_cast<T>(op.c);
  if (FL == kSkip) {
    static_cast<T*>(op.y_out)[q] = c * ax;
  } else if (FL == kFlushY || FL == kFlushNoY) {
    const T y = c * ax;
    static_cast<T*>(op.acc_out)[q] = static_cast<const T*>(op.acc_in)[q] + static_cast<T>(op.cs) * xc + y;
    if (FL == kFlushY) static_cast<T*>(op.y_out)[q] = y;
  } else if (FL == kFirst) {
    const T y = c * ax + static_cast<T>(op.cb) * static_cast<const T*>(op.bsrc)[q];
    static_cast<T*>(op.acc_out)[q] = static_cast<T>(op.cs) * xc + y;
    static_cast<T*>(op.y_out)[q] = y;
  } else {
    T y = c * ax;
    if (op.bsrc) y += static_cast<T>(op.cb) * static_cast<const T*>(op.bsrc)[q];
    T v = static_cast<T>(op.cs) * xc + y;
    if (op.acc_in) v += static_cast<T>(op.ca) * static_cast<const T*>(op.acc_in)[q];
    if (op.u) {
      T* u = static_cast<T*>(op.u);
      u[q] = u[q] + v;
    } else {
      if (op.y_out) static_cast<T*>(op.y_out)[q] = y;
      if (op.acc_out) static_cast<T*>(op.acc_out)[q] = v;
    }
  }
}

template <typename T>
__device__ __forceinline__ void term_store_runtime(const TermOp& op, int q, T ax, T xc) {
  switch (op.flavor) {
    case kSkip: term_store<T, kSkip>(op, q, ax, xc); break;
    case kFlushY: term_store<T, kFlushY>(op, q, ax, xc); break;
    case kFlushNoY: term_store<T, kFlushNoY>(op, q, ax, xc); break;
    case kFirst: term_store<T, kFirst>(op, q, ax, xc); break;
    default: term_store<T, kGeneric>(op, q, ax, xc); break;
  }
}

// The sweep of one thread: column (j, k), planes i0 .. i0 + lp - 1 (clipped
// to the grid).  LP > 0 fixes the plane count at compile time; LP == 0 takes
// the runtime lp.  FL == kRuntimeFlavor dispatches on op.flavor.
template <typename T, int BC, int LP, int KIND, int FL>
__device__ __forceinline__ void sweep_column(const Geom& g, const Coef& cf, const LdsCoef<T>& s, const SweepArgs& a,
                                             int i0, int j, int k, int lp) {
  const int sx = g.ny * g.nz;
  const int dym = j > 0 ? -g.nz : 0, dyp = j < g.ny - 1 ? g.nz : 0;
  const int dzm = k > 0 ? -1 : 0, dzp = k < g.nz - 1 ? 1 : 0;
  const int wall_yz = BC ? (j == 0) + (j == g.ny - 1) + (k == 0) + (k == g.nz - 1) : 0;
  const T* __restrict__ x = static_cast<const T*>(KIND == kTerm ? a.op.src : a.x);
  const uint8_t* __restrict__ lab = cf.labels;
  const T* __restrict__ fx = static_cast<const T*>(cf.fx);
  const T* __restrict__ fy = static_cast<const T*>(cf.fy);
  const T* __restrict__ fz = static_cast<const T*>(cf.fz);
  int q = (i0 * g.ny + j) * g.nz + k;
  const int qm0 = i0 > 0 ? q - sx : q;
  T xm = x[qm0], xc = x[q];
  int lm = 0, lc = 0;
  T km = T(0);  // dense form: coefficient of the -x face
  if (cf.labels_form) {
    lm = lab[qm0];
    lc = lab[q];
  } else {
    km = fx[qm0];
  }
  const int np = LP > 0 ? LP : lp;
#pragma unroll 4
  for (int sp = 0; sp < np; ++sp) {
    const int i = i0 + sp;
    if (i >= g.nx) break;
    const int qn = i < g.nx - 1 ? q + sx : q;
    const T xn = x[qn];
    const T x2 = x[q + dym], x3 = x[q + dyp], x4 = x[q + dzm], x5 = x[q + dzp];
    T ax;
    int ln = 0;
    if (cf.labels_form) {
      ln = lab[qn];
      const int l2 = lab[q + dym], l3 = lab[q + dyp], l4 = lab[q + dzm], l5 = lab[q + dzp];
      const T* row = s.tab + lc * kMaxClasses;
      ax = row[lm] * (xm - xc) + row[ln] * (xn - xc) + row[l2] * (x2 - xc) + row[l3] * (x3 - xc) +
           row[l4] * (x4 - xc) + row[l5] * (x5 - xc);
      if (BC) ax -= s.wall[lc] * xc * T(wall_yz + (i == 0) + (i == g.nx - 1));
    } else {
      const T kp = fx[q];
      ax = km * (xm - xc) + kp * (xn - xc) + fy[q + dym] * (x2 - xc) + fy[q] * (x3 - xc) + fz[q + dzm] * (x4 - xc) +
           fz[q] * (x5 - xc);
      if (BC) ax -= static_cast<const T*>(cf.wallv)[q] * xc * T(wall_yz + (i == 0) + (i == g.nx - 1));
      km = kp;
    }
    if (KIND == kTerm) {
      if (FL == kRuntimeFlavor) term_store_runtime<T>(a.op, q, ax, xc);
      else term_store<T, FL>(a.op, q, ax, xc);
    } else if (KIND == kRhs) {
      static_cast<T*>(a.out)[q] = ax + static_cast<T>(a.rho) * xc * (T(1) - xc);
    } else if (KIND == kAdjRhs) {
      // lambda + A g + rho (1 - 2 u) g: the transpose of the step's Jacobian
      // applied to g (A is symmetric)
      const T uq = static_cast<const T*>(a.aux1)[q];
      static_cast<T*>(a.out)[q] =
          static_cast<const T*>(a.aux0)[q] + ax + static_cast<T>(a.rho) * (T(1) - T(2) * uq) * xc;
    } else {
      static_cast<T*>(a.out)[q] = ax;
    }
    xm = xc;
    xc = xn;
    lm = lc;
    lc = ln;
    q += sx;
  }
}

}  // namespace expint
