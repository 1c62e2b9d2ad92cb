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

// Workgroups are dealt to the 8 XCDs round-robin; map workgroup L of nb to a
// tile so that each XCD takes a contiguous run of tiles (neighbouring planes
// then share that XCD's L2).
__device__ __forceinline__ int xcd_remap(int L, int nb) {
  if ((nb & 7) == 0) {
    const int per = nb >> 3;
    return (L & 7) * per + (L >> 3);
  }
  return L;
}

// The tile of workgroup L (after xcd_remap) in the z-vectorised sweeps'
// decomposition (ColumnGrid), with lp planes per lane, and thread tid's place
// in it: z-segment zs, row block yb, first plane i0, lane index kq in the
// segment, row j and 4-voxel vector k4.  The divisions by the tile counts
// are multiplies by host-computed constants, on the scalar unit.
struct ColumnTile {
  int zs, yb, i0, kq, j, k4;
};
__device__ __forceinline__ ColumnTile column_tile(const ColumnGrid& cg, int L, int lp, int tid) {
  ColumnTile c;
  const int t = static_cast<int>(cg.zs.div(static_cast<uint32_t>(L)));
  c.zs = L - t * static_cast<int>(cg.zs.d);
  const int xg = static_cast<int>(cg.y.div(static_cast<uint32_t>(t)));
  c.yb = t - xg * static_cast<int>(cg.y.d);
  c.i0 = xg * lp;
  c.kq = tid & (cg.rw - 1);
  c.j = c.yb * (kBlock >> cg.rw_log2) + (tid >> cg.rw_log2);
  c.k4 = c.zs * cg.rw + c.kq;
  return c;
}

// kTermJ is a Taylor-term sweep of the linearised operator
// J = A + rho diag(1 - 2 u_n) (TermOp::ju, TermOp::jrho): the diagonal term is
// added to the stencil result before the term's outputs are formed.
enum SweepKind { kTerm = 0, kRhs = 1, kApply = 2, kAdjRhs = 3, kTermJ = 4 };
constexpr int kRuntimeFlavor = -1;
__host__ __device__ constexpr bool is_term(int kind) { return kind == kTerm || kind == kTermJ; }

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
    if (op.bsrc2) y += static_cast<T>(op.cb2) * static_cast<const T*>(op.bsrc2)[q];
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
  const T* __restrict__ x = static_cast<const T*>(is_term(KIND) ? a.op.src : a.x);
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
    if (KIND == kTermJ) {
      // u_n at this voxel only; a last sweep that adds into u_n reads it first
      const T d = static_cast<T>(a.op.jrho) * (T(1) - T(2) * static_cast<const T*>(a.op.ju)[q]);
      ax += d * xc;
    }
    if (is_term(KIND)) {
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

// ---------------------------------------------------------------------------
// z-vectorised sweep: a lane owns four consecutive z voxels (one 4-value
// vector of each field and one 32-bit word of labels), so every load and
// store of a wavefront is a run of 16-byte (FP32) or 32-byte (FP64) vectors.
// Lanes are grouped in z-segments of rw lanes (4 rw voxels); the z
// neighbours of a lane's first and last voxel come from the adjacent lanes of
// the segment by shuffles, at a segment edge inside the row by one scalar
// load, at a wall from the voxel itself (zero flux).  Needs nz % 4 == 0 and
// the label form.  Same arithmetic per voxel as sweep_column.
// ---------------------------------------------------------------------------

template <typename T>
struct alignas(4 * sizeof(T)) Vec4 {
  T v[4];
};

template <typename T>
__device__ __forceinline__ Vec4<T> ld4(const void* p, int q4) {
  return static_cast<const Vec4<T>*>(p)[q4];
}
template <typename T>
struct NtVec {
  typedef T type __attribute__((ext_vector_type(4)));
};
// NT: a non-temporal store, which streams the vector out during the sweep
// instead of leaving it dirty in L2 (Tiling::nt).
template <typename T, bool NT = false>
__device__ __forceinline__ void st4(void* p, int q4, const Vec4<T>& v) {
  if (NT) {
    const typename NtVec<T>::type w = {v.v[0], v.v[1], v.v[2], v.v[3]};
    __builtin_nontemporal_store(w, static_cast<typename NtVec<T>::type*>(p) + q4);
  } else {
    static_cast<Vec4<T>*>(p)[q4] = v;
  }
}

__device__ __forceinline__ int label_byte(uint32_t w, int e) { return static_cast<int>((w >> (8 * e)) & 255u); }

// Outputs of one Taylor-term sweep on the four voxels of vector q4 (see
// TermOp); NT: by non-temporal stores.
template <typename T, int FL, bool NT = false>
__device__ __forceinline__ void term_store4(const TermOp& op, int q4, const T (&ax)[4], const Vec4<T>& xc) {
  const T c = static_cast<T>(op.c), cs = static_cast<T>(op.cs);
  Vec4<T> y;
  if (FL == kSkip) {
#pragma unroll
    for (int e = 0; e < 4; ++e) y.v[e] = c * ax[e];
    st4<T, NT>(op.y_out, q4, y);
  } else if (FL == kFlushY || FL == kFlushNoY) {
    const Vec4<T> ai = ld4<T>(op.acc_in, q4);
    Vec4<T> v;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      y.v[e] = c * ax[e];
      v.v[e] = ai.v[e] + cs * xc.v[e] + y.v[e];
    }
    st4<T, NT>(op.acc_out, q4, v);
    if (FL == kFlushY) st4<T, NT>(op.y_out, q4, y);
  } else if (FL == kFirst) {
    const Vec4<T> b = ld4<T>(op.bsrc, q4);
    const T cb = static_cast<T>(op.cb);
    Vec4<T> v;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      y.v[e] = c * ax[e] + cb * b.v[e];
      v.v[e] = cs * xc.v[e] + y.v[e];
    }
    st4<T, NT>(op.acc_out, q4, v);
    st4<T, NT>(op.y_out, q4, y);
  } else {
    Vec4<T> v;
#pragma unroll
    for (int e = 0; e < 4; ++e) y.v[e] = c * ax[e];
    if (op.bsrc) {
      const Vec4<T> b = ld4<T>(op.bsrc, q4);
      const T cb = static_cast<T>(op.cb);
#pragma unroll
      for (int e = 0; e < 4; ++e) y.v[e] += cb * b.v[e];
    }
    if (op.bsrc2) {
      const Vec4<T> b2 = ld4<T>(op.bsrc2, q4);
      const T cb2 = static_cast<T>(op.cb2);
#pragma unroll
      for (int e = 0; e < 4; ++e) y.v[e] += cb2 * b2.v[e];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) v.v[e] = cs * xc.v[e] + y.v[e];
    if (op.acc_in) {
      const Vec4<T> ai = ld4<T>(op.acc_in, q4);
      const T ca = static_cast<T>(op.ca);
#pragma unroll
      for (int e = 0; e < 4; ++e) v.v[e] += ca * ai.v[e];
    }
    if (op.u) {
      Vec4<T> uu = ld4<T>(op.u, q4);
#pragma unroll
      for (int e = 0; e < 4; ++e) uu.v[e] = uu.v[e] + v.v[e];
      st4<T, NT>(op.u, q4, uu);
    } else {
      if (op.y_out) st4<T, NT>(op.y_out, q4, y);
      if (op.acc_out) st4<T, NT>(op.acc_out, q4, v);
    }
  }
}

// No-op for callers whose class tables are already in LDS.
struct TablesReady {
  __device__ __forceinline__ void operator()() const {}
};

// Per-plane hook of sweep_column4 that does nothing (see there).
struct NoFace {
  template <typename... Args>
  __device__ __forceinline__ void operator()(Args&&...) const {}
};

// The sweep of one lane: vector k4 (voxels 4 k4 .. 4 k4 + 3) of row j,
// planes i0 .. i0 + LP - 1 (clipped to the grid); kq is the lane's index in
// its z-segment of rw lanes.  live: the lane's vector is inside the grid.
// Every lane of the workgroup calls this; a lane that is not live issues no
// loads or stores and returns after ready(), and a live lane only uses a
// neighbour's shuffled values when that neighbour is in the same row and
// inside the grid (else the wall or segment-edge value).
// ready() runs after the first plane's loads are issued and before the class
// table is read, in control flow that every lane of the workgroup reaches: a
// caller that stages the table there with a workgroup barrier overlaps the
// two (a barrier reached on two divergent paths of one wave would be passed
// twice by that wave and pair with a later barrier of the others).
// face(i, q, xc, xn, xy, xz, lc, ln, ly, lz) runs once per plane with the
// source values the stencil holds: the lane's four voxels, their +x and +y
// neighbours, the +z neighbour of the last voxel, and the matching labels
// (each neighbour is the voxel itself at a wall).
template <typename T, int BC, int LP, int KIND, int FL, bool NT = false, typename Ready = TablesReady,
          typename Face = NoFace>
__device__ __forceinline__ void sweep_column4(const Geom& g, const uint8_t* lab, const LdsCoef<T>& s,
                                              const SweepArgs& a, int i0, int j, int k4, int kq, int rw,
                                              bool live, Ready&& ready = Ready{}, Face&& face = Face{}) {
  const int nz4 = g.nz >> 2;
  const int sx4 = g.ny * nz4;
  const int dym = j > 0 ? -nz4 : 0, dyp = j < g.ny - 1 ? nz4 : 0;
  const bool wall_lo = k4 == 0, wall_hi = k4 == nz4 - 1;          // z walls
  const bool edge_lo = !wall_lo && kq == 0, edge_hi = !wall_hi && kq == rw - 1;  // segment edges in the row
  const int wall_y = BC ? (j == 0) + (j == g.ny - 1) : 0;
  const T* __restrict__ x = static_cast<const T*>(is_term(KIND) ? a.op.src : a.x);
  const uint32_t* __restrict__ l4 = reinterpret_cast<const uint32_t*>(lab);
  int q = (i0 * g.ny + j) * nz4 + k4;
  Vec4<T> xm, xc;
  uint32_t lm = 0, lc = 0;
  // loads of the plane computed next: +x neighbour, lateral neighbours
  // (kTermJ: and u_n of the plane itself)
  Vec4<T> fxn, fya, fyb, fun;
  uint32_t fln = 0, fla = 0, flb = 0;
  auto fetch = [&](int i, int qq) {
    const int qn = i < g.nx - 1 ? qq + sx4 : qq;
    fxn = ld4<T>(x, qn);
    fln = l4[qn];
    fya = ld4<T>(x, qq + dym);
    fyb = ld4<T>(x, qq + dyp);
    fla = l4[qq + dym];
    flb = l4[qq + dyp];
    if (KIND == kTermJ) fun = ld4<T>(a.op.ju, qq);
  };
  if (live) {
    const int qm0 = i0 > 0 ? q - sx4 : q;
    xm = ld4<T>(x, qm0);
    xc = ld4<T>(x, q);
    lm = l4[qm0];
    lc = l4[q];
    fetch(i0, q);
  }
  ready();
  if (!live) return;
#pragma unroll
  for (int sp = 0; sp < LP; ++sp) {
    const int i = i0 + sp;
    if (i >= g.nx) break;
    const Vec4<T> xn = fxn, ya = fya, yb = fyb, un = fun;
    const uint32_t ln = fln, la = fla, lb = flb;
    if (sp + 1 < LP && i + 1 < g.nx) fetch(i + 1, q + sx4);
    // z neighbours of voxels 0 and 3
    T zl = __shfl_up(xc.v[3], 1, rw), zr = __shfl_down(xc.v[0], 1, rw);
    int lzl = label_byte(__shfl_up(lc, 1, rw), 3), lzr = label_byte(__shfl_down(lc, 1, rw), 0);
    if (wall_lo) {
      zl = xc.v[0];
      lzl = label_byte(lc, 0);
    } else if (edge_lo) {
      zl = x[4 * q - 1];
      lzl = lab[4 * q - 1];
    }
    if (wall_hi) {
      zr = xc.v[3];
      lzr = label_byte(lc, 3);
    } else if (edge_hi) {
      zr = x[4 * q + 4];
      lzr = lab[4 * q + 4];
    }
    const int wall_x = BC ? wall_y + (i == 0) + (i == g.nx - 1) : 0;
    // class pairs le * 8 + l of the four voxels with each neighbour, one per
    // byte (labels are below 8, so the bytes do not carry): one table index
    // per face from a byte extract
    const uint32_t pc = lc << 3;
    const uint32_t pm = pc + lm, pn = pc + ln, pa = pc + la, pb = pc + lb;
    const uint32_t pzm = pc + ((lc << 8) | static_cast<uint32_t>(lzl));
    const uint32_t pzp = pc + ((lc >> 8) | (static_cast<uint32_t>(lzr) << 24));
    T ax[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const T v = xc.v[e];
      const int le = label_byte(lc, e);
      const T vzm = e > 0 ? xc.v[e - 1] : zl;
      const T vzp = e < 3 ? xc.v[e + 1] : zr;
      ax[e] = s.tab[label_byte(pm, e)] * (xm.v[e] - v) + s.tab[label_byte(pn, e)] * (xn.v[e] - v) +
              s.tab[label_byte(pa, e)] * (ya.v[e] - v) + s.tab[label_byte(pb, e)] * (yb.v[e] - v) +
              s.tab[label_byte(pzm, e)] * (vzm - v) + s.tab[label_byte(pzp, e)] * (vzp - v);
      if (BC) {
        const int nw = wall_x + (e == 0 && wall_lo) + (e == 3 && wall_hi);
        ax[e] -= s.wall[le] * v * T(nw);
      }
      if (KIND == kTermJ) {
        const T d = static_cast<T>(a.op.jrho) * (T(1) - T(2) * un.v[e]);
        ax[e] += d * v;
      }
    }
    if (is_term(KIND)) {
      term_store4<T, FL, NT>(a.op, q, ax, xc);
    } else if (KIND == kRhs) {
      Vec4<T> o;
      const T rho = static_cast<T>(a.rho);
#pragma unroll
      for (int e = 0; e < 4; ++e) o.v[e] = ax[e] + rho * xc.v[e] * (T(1) - xc.v[e]);
      st4<T>(a.out, q, o);
    } else if (KIND == kAdjRhs) {
      const Vec4<T> lam = ld4<T>(a.aux0, q), uq = ld4<T>(a.aux1, q);
      const T rho = static_cast<T>(a.rho);
      Vec4<T> o;
#pragma unroll
      for (int e = 0; e < 4; ++e) o.v[e] = lam.v[e] + ax[e] + rho * (T(1) - T(2) * uq.v[e]) * xc.v[e];
      st4<T>(a.out, q, o);
    } else {
      Vec4<T> o;
#pragma unroll
      for (int e = 0; e < 4; ++e) o.v[e] = ax[e];
      st4<T>(a.out, q, o);
    }
    face(i, q, xc, xn, yb, zr, lc, ln, lb, lzr);
    xm = xc;
    xc = xn;
    lm = lc;
    lc = ln;
    q += sx4;
  }
}

}  // namespace expint
