// Class-diffusivity derivatives of the bilinear form <ybar, A y> for the
// discrete adjoint of the exponential Euler step (label form).
//
// With the conservative operator (A y)_p = sum_q K_pq (y_q - y_p) / h^2,
//   <ybar, A y> = - sum over faces p|q of K_pq (ybar_p - ybar_q)(y_p - y_q) / h^2
//                 - sum over zero-Dirichlet wall faces of D_p ybar_p y_p / h^2,
// so its derivative with respect to the diffusivity D_c of tissue class c is
// a weighted sum of face products: the weights -dK(D_a, D_b)/dD_c / h^2 (and
// -[a == c] / h^2 at walls) come precomputed per class pair in FP64.  Every
// face is visited once (the +x, +y, +z faces of each voxel).
//
// A gradient evaluates thousands of such forms (one per Taylor term of the
// reverse pass), so they are not reduced one by one: workgroup b adds
// weight * (its FP64 partial sums) into slot b of a partial buffer that stays
// on the device, and one fixed-order reduction at the end turns the slots into
// the class gradients.  Each slot is updated by one workgroup per launch and
// launches are stream-ordered, so results are bit-reproducible.

#include <algorithm>
#include <cstdint>
#include <initializer_list>

#include "internal.hpp"
#include "sweep_device.hpp"

namespace expint {

namespace {

constexpr int kFaceLP = 4;  // x-planes per lane of the vectorised face products

// x plus its value at the lane the DPP pattern CTRL names (a permutation
// within each row of 16 lanes), moved as two 32-bit halves.  Every lane has
// a source, so bound control is set and the moves need no old value.
template <int CTRL>
__device__ __forceinline__ double dpp_add(double x) {
  const unsigned long long bits = static_cast<unsigned long long>(__double_as_longlong(x));
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(bits & 0xffffffffull), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(bits >> 32), CTRL, 0xf, 0xf, true);
  const unsigned long long p = (static_cast<unsigned long long>(static_cast<unsigned int>(hi)) << 32) |
                               static_cast<unsigned int>(lo);
  return x + __longlong_as_double(static_cast<long long>(p));
}

// The sum over each row of 16 lanes, in every lane of the row: pairs
// (quad_perm 1,0,3,2), quads (quad_perm 2,3,0,1), half rows (half mirror),
// rows (mirror); register moves only, no LDS.
__device__ __forceinline__ double row_sum(double v) {
  v = dpp_add<0xb1>(v);
  v = dpp_add<0x4e>(v);
  v = dpp_add<0x141>(v);
  return dpp_add<0x140>(v);
}

// The value of the workgroup's partial slot for class c, read at the start
// of a kernel by lane 16 c so that its latency overlaps the sweep (each slot
// is written by one workgroup per launch, and launches are stream-ordered).
template <int NC>
__device__ __forceinline__ double slot_prefetch(const double* partial) {
  const int tid = static_cast<int>(threadIdx.x);
  return (tid & 15) == 0 && (tid >> 4) < NC ? partial[static_cast<size_t>(blockIdx.x) * kMaxClasses + (tid >> 4)]
                                            : 0.0;
}

// Sums acc over the workgroup in a fixed order (rows of 16 lanes; then the
// workgroup's 16 row sums of class c, as row c of 16 lanes) and writes
// prev + weight * sum into partial[blockIdx.x * 8 + c] for the NC classes of
// the grid (the slots of the other classes stay as filled, zero); prev is
// what slot_prefetch read.  Every thread of the workgroup must call it, in
// converged control flow.
template <int NC>
__device__ __forceinline__ void block_accumulate(double (&acc)[kMaxClasses], double weight, double* partial,
                                                 double prev) {
  static_assert(kBlock == 256 && 16 * NC <= kBlock, "16 rows of 16 lanes; one row per class for the second level");
  __shared__ double red[kBlock / 16][kMaxClasses];
  const int tid = static_cast<int>(threadIdx.x);
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double v = row_sum(acc[c]);
    if ((tid & 15) == 0) red[tid >> 4][c] = v;
  }
  __syncthreads();
  if (tid < 16 * NC) {  // whole rows, so every lane a DPP move reads is active
    const int c = tid >> 4;
    const double v = row_sum(red[tid & 15][c]);
    if ((tid & 15) == 0) partial[static_cast<size_t>(blockIdx.x) * kMaxClasses + c] = prev + weight * v;
  }
}

// Class weights of the faces in LDS with the class index fastest, so that
// one face's NC weights are adjacent: tab[(a * 8 + b) * face_stride<NC>() + c].
template <int NC>
constexpr int face_stride() {
  return NC <= 2 ? 2 : (NC <= 4 ? 4 : 8);
}

struct FaceTables {
  alignas(16) double tab[kMaxClasses * kTab];  // [a][b][c], see face_stride
  double wall[kMaxClasses * kMaxClasses];      // [c][a]
};

// Stages the entries a grid of NC classes can reach (class c, labels a, b
// below NC) from the device tables ([c][a][b] and [c][a]).
template <int NC>
__device__ __forceinline__ void load_face_tables(FaceTables& ft, const double* dtab, const double* dwall) {
  for (int t = threadIdx.x; t < NC * NC * NC; t += kBlock) {
    const int c = t / (NC * NC), a = (t / NC) % NC, b = t % NC;
    ft.tab[(a * kMaxClasses + b) * face_stride<NC>() + c] = dtab[c * kTab + a * kMaxClasses + b];
  }
  if (threadIdx.x < NC * NC) {
    const int o = (threadIdx.x / NC) * kMaxClasses + threadIdx.x % NC;
    ft.wall[o] = dwall[o];
  }
}

template <int NC>
__device__ __forceinline__ void add_face_pair(double (&acc)[kMaxClasses], const FaceTables& ft, int pair,
                                              double prod) {
  const double* w = ft.tab + pair * face_stride<NC>();
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] += w[c] * prod;
}

template <int NC>
__device__ __forceinline__ void add_face(double (&acc)[kMaxClasses], const FaceTables& ft, int la, int lb,
                                         double prod) {
  add_face_pair<NC>(acc, ft, la * kMaxClasses + lb, prod);
}

// (xp - xq)(yp - yq) with the differences taken in the field's own type (an
// FP32 difference is exact when the two are within a factor of two, else
// off by at most one rounding) and the product in FP64.
template <typename T>
__device__ __forceinline__ double face_prod(T xp, T xq, T yp, T yq) {
  return static_cast<double>(xp - xq) * static_cast<double>(yp - yq);
}

// Scalar form: any grid; grid-stride over voxels.  NC = number of classes.
template <typename T, int BC, int NC>
__global__ __launch_bounds__(kBlock) void k_faceprod(Geom g, const uint8_t* __restrict__ lab,
                                                     const double* __restrict__ dtab, const double* __restrict__ dwall,
                                                     const T* __restrict__ yb, const T* __restrict__ y, double weight,
                                                     double* __restrict__ partial) {
  __shared__ FaceTables ft;
  const double prev = slot_prefetch<NC>(partial);
  load_face_tables<NC>(ft, dtab, dwall);
  __syncthreads();
  double acc[kMaxClasses];
#pragma unroll
  for (int c = 0; c < kMaxClasses; ++c) acc[c] = 0.0;
  const int sx = g.ny * g.nz, sy = g.nz;
  const int n = static_cast<int>(g.n);
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < n; p += gridDim.x * kBlock) {
    const int k = p % g.nz;
    const int t = p / g.nz;
    const int j = t % g.ny;
    const int i = t / g.ny;
    const int lp = lab[p];
    const double ybp = static_cast<double>(yb[p]), yp = static_cast<double>(y[p]);
    auto face = [&](int q) {
      add_face<NC>(acc, ft, lp, lab[q], face_prod<T>(yb[p], yb[q], y[p], y[q]));
    };
    if (i < g.nx - 1) face(p + sx);
    if (j < g.ny - 1) face(p + sy);
    if (k < g.nz - 1) face(p + 1);
    if (BC) {
      const int nw = (i == 0) + (i == g.nx - 1) + (j == 0) + (j == g.ny - 1) + (k == 0) + (k == g.nz - 1);
      if (nw) {
        const double v = ybp * yp * nw;
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] += ft.wall[c * kMaxClasses + lp] * v;
      }
    }
  }
  block_accumulate<NC>(acc, weight, partial, prev);
}

// z-vectorised form (nz % 4 == 0, 4-value aligned fields): the z-segments of
// the vectorised sweeps; a lane owns four z voxels of one row and marches over
// kFaceLP planes; the +z face of its last voxel pairs with the next lane's first
// (shuffle), the next segment's first (load) or nothing at the wall.
template <typename T, int BC, int NC>
__global__ __launch_bounds__(kBlock) void k_faceprod4(Geom g, ColumnGrid cg, const uint8_t* __restrict__ lab,
                                                      const double* __restrict__ dtab,
                                                      const double* __restrict__ dwall, const T* __restrict__ yb,
                                                      const T* __restrict__ y, double weight,
                                                      double* __restrict__ partial) {
  __shared__ FaceTables ft;
  const double prev = slot_prefetch<NC>(partial);
  load_face_tables<NC>(ft, dtab, dwall);
  __syncthreads();
  double acc[kMaxClasses];
#pragma unroll
  for (int c = 0; c < kMaxClasses; ++c) acc[c] = 0.0;
  const int L = xcd_remap(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
  const ColumnTile c = column_tile(cg, L, kFaceLP, static_cast<int>(threadIdx.x));
  const int i0 = c.i0, kq = c.kq, j = c.j, k4 = c.k4, rw = cg.rw;
  const int nz4 = g.nz >> 2;
  const bool live = j < g.ny && k4 < nz4;
  if (live) {
    const int sx4 = g.ny * nz4;
    const uint32_t* l4 = reinterpret_cast<const uint32_t*>(lab);
    const int dyp = j < g.ny - 1 ? nz4 : 0;
    const bool wall_hi = k4 == nz4 - 1, edge_hi = !wall_hi && kq == rw - 1;
    int q = (i0 * g.ny + j) * nz4 + k4;
    Vec4<T> bc = ld4<T>(yb, q), vc = ld4<T>(y, q);
    uint32_t lc = l4[q];
#pragma unroll 2
    for (int sp = 0; sp < kFaceLP; ++sp) {
      const int i = i0 + sp;
      if (i >= g.nx) break;
      const int qn = i < g.nx - 1 ? q + sx4 : q;
      const Vec4<T> bn = ld4<T>(yb, qn), vn = ld4<T>(y, qn);
      const uint32_t ln = l4[qn];
      const Vec4<T> by = ld4<T>(yb, q + dyp), vy = ld4<T>(y, q + dyp);
      const uint32_t ly = l4[q + dyp];
      T bz = __shfl_down(bc.v[0], 1, rw), vz = __shfl_down(vc.v[0], 1, rw);
      int lz = label_byte(__shfl_down(lc, 1, rw), 0);
      if (wall_hi) {
        bz = bc.v[3];
        vz = vc.v[3];
        lz = label_byte(lc, 3);
      } else if (edge_hi) {
        bz = yb[4 * q + 4];
        vz = y[4 * q + 4];
        lz = lab[4 * q + 4];
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int le = label_byte(lc, e);
        const double bp = static_cast<double>(bc.v[e]), vp = static_cast<double>(vc.v[e]);
        // +x and +y faces (the voxel itself at the far walls: product 0)
        add_face<NC>(acc, ft, le, label_byte(ln, e), face_prod<T>(bc.v[e], bn.v[e], vc.v[e], vn.v[e]));
        add_face<NC>(acc, ft, le, label_byte(ly, e), face_prod<T>(bc.v[e], by.v[e], vc.v[e], vy.v[e]));
        // +z face
        const T bq = e < 3 ? bc.v[e + 1] : bz;
        const T vq = e < 3 ? vc.v[e + 1] : vz;
        add_face<NC>(acc, ft, le, e < 3 ? label_byte(lc, e + 1) : lz, face_prod<T>(bc.v[e], bq, vc.v[e], vq));
        if (BC) {
          const int nw = (i == 0) + (i == g.nx - 1) + (j == 0) + (j == g.ny - 1) + (e == 0 && k4 == 0) +
                         (e == 3 && wall_hi);
          if (nw) {
            const double v = bp * vp * nw;
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[c] += ft.wall[c * kMaxClasses + le] * v;
          }
        }
      }
      bc = bn;
      vc = vn;
      lc = ln;
      q += sx4;
    }
  }
  block_accumulate<NC>(acc, weight, partial, prev);
}

// acc[c] += sum over slots b of partial[b][c]: thread t sums the slots
// b = t, t + 256, ... of every class, then a fixed-order tree over the 256
// threads (bit-reproducible).
__global__ __launch_bounds__(kBlock) void k_faceprod_final(const double* __restrict__ partial, int nb,
                                                           double* __restrict__ acc) {
  __shared__ double red[kBlock][kMaxClasses + 1];
  const int t = threadIdx.x;
  double v[kMaxClasses];
#pragma unroll
  for (int c = 0; c < kMaxClasses; ++c) v[c] = 0.0;
  for (int b = t; b < nb; b += kBlock)
#pragma unroll
    for (int c = 0; c < kMaxClasses; ++c) v[c] += partial[b * kMaxClasses + c];
#pragma unroll
  for (int c = 0; c < kMaxClasses; ++c) red[t][c] = v[c];
  __syncthreads();
  for (int half = kBlock / 2; half > 0; half >>= 1) {
    if (t < half)
#pragma unroll
      for (int c = 0; c < kMaxClasses; ++c) red[t][c] += red[t + half][c];
    __syncthreads();
  }
  if (t < kMaxClasses) acc[t] += red[0][t];
}

// The face products of one lane, taken inside a sweep whose stencil source
// is ybar (sweep_column4's per-plane hook): the sweep hands over ybar on the
// lane's four voxels and their +x, +y, +z neighbours with the labels, and
// this adds the same FP64 face terms as k_faceprod4 against y (loaded here).
// load() fetches y on the lane's voxels of its first plane and their +x, +y,
// +z neighbours before the sweep starts, so these loads are in flight
// together with the sweep's own; the hook uses them for plane i and then
// fetches the next plane's (the +x values become the centre values), which
// the sweep's work on that plane covers.
// DB (a Taylor term of the linearised operator): the hook also adds
// wd * ybar * y into dbar on the lane's voxels, the diagonal's share.
template <typename T, int BC, int NC, bool DB>
struct FaceAcc {
  const Geom& g;
  const FaceTables& ft;
  int j, k4, kq, rw, i_end;
  bool wall_hi;
  Vec4<T> vc, vn, vy, dv;
  T vz_edge;
  const T* yf;
  T* dbar;
  T wd;
  double acc[kMaxClasses];

  __device__ __forceinline__ FaceAcc(const Geom& g_, const FaceTables& ft_, int j_, int k4_, int kq_, int rw_,
                                     int i_end_, T* dbar_, T wd_)
      : g(g_), ft(ft_), j(j_), k4(k4_), kq(kq_), rw(rw_), i_end(i_end_), wall_hi(k4_ == (g_.nz >> 2) - 1),
        yf(nullptr), dbar(dbar_), wd(wd_) {
#pragma unroll
    for (int c = 0; c < kMaxClasses; ++c) acc[c] = 0.0;
  }

  // y on plane i: the +x and +y neighbours and the z segment edge (the
  // centre values are already held), and dbar
  __device__ __forceinline__ void fetch(int i) {
    const int nz4 = g.nz >> 2, sx4 = g.ny * nz4;
    const int q = (i * g.ny + j) * nz4 + k4;
    const int qn = i < g.nx - 1 ? q + sx4 : q;
    const int dyp = j < g.ny - 1 ? nz4 : 0;
    vn = ld4<T>(yf, qn);
    vy = ld4<T>(yf, q + dyp);
    const bool edge_hi = !wall_hi && kq == rw - 1;
    vz_edge = edge_hi ? yf[4 * q + 4] : T(0);
    if (DB) dv = ld4<T>(dbar, q);
  }

  __device__ __forceinline__ void load(const T* __restrict__ y, int i) {
    const int nz4 = g.nz >> 2;
    yf = y;
    vc = ld4<T>(y, (i * g.ny + j) * nz4 + k4);
    fetch(i);
  }

  __device__ __forceinline__ void operator()(int i, int q, const Vec4<T>& bc, const Vec4<T>& bn, const Vec4<T>& by,
                                             T bz, uint32_t lc, uint32_t ln, uint32_t ly, int lz) {
    const bool edge_hi = !wall_hi && kq == rw - 1;
    T vz = __shfl_down(vc.v[0], 1, rw);
    if (wall_hi) vz = vc.v[3];
    else if (edge_hi) vz = vz_edge;
    // face class pairs a * 8 + b of the four voxels, one per byte (labels are
    // below 8, so the bytes do not carry)
    const uint32_t pa = lc << 3;
    const uint32_t px = pa + ln, py = pa + ly, pz = pa + ((lc >> 8) | (static_cast<uint32_t>(lz) << 24));
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int le = label_byte(lc, e);
      const double bp = static_cast<double>(bc.v[e]), vp = static_cast<double>(vc.v[e]);
      add_face_pair<NC>(acc, ft, label_byte(px, e), face_prod<T>(bc.v[e], bn.v[e], vc.v[e], vn.v[e]));
      add_face_pair<NC>(acc, ft, label_byte(py, e), face_prod<T>(bc.v[e], by.v[e], vc.v[e], vy.v[e]));
      const T bq = e < 3 ? bc.v[e + 1] : bz;
      const T vq = e < 3 ? vc.v[e + 1] : vz;
      add_face_pair<NC>(acc, ft, label_byte(pz, e), face_prod<T>(bc.v[e], bq, vc.v[e], vq));
      if (BC) {
        const int nw = (i == 0) + (i == g.nx - 1) + (j == 0) + (j == g.ny - 1) + (e == 0 && k4 == 0) +
                       (e == 3 && wall_hi);
        if (nw) {
          const double v = bp * vp * nw;
#pragma unroll
          for (int c = 0; c < NC; ++c) acc[c] += ft.wall[c * kMaxClasses + le] * v;
        }
      }
    }
    if (DB) {
#pragma unroll
      for (int e = 0; e < 4; ++e) dv.v[e] += wd * bc.v[e] * vc.v[e];
      st4<T>(dbar, q, dv);
    }
    if (i + 1 < i_end) {
      vc = vn;
      fetch(i + 1);
    }
  }
};

// One z-vectorised sweep of kind KIND (a Taylor term of the reverse pass, of
// A or of the linearised operator, or the adjoint right-hand side) with the
// face products of its stencil source against y in the same pass: one plane
// per lane, workgroups as in k_sweep4 with lp = 1; workgroup b adds
// weight * (its sums) into slot b.  kTermJ also adds weight * ybar * y into
// dbar.
template <typename T, int BC, int KIND, int NC, int LP>
__global__ __launch_bounds__(kBlock) void k_sweep_face4(Geom g, ColumnGrid cg, Coef cf, SweepArgs a,
                                                        const T* __restrict__ y, const double* __restrict__ dtab,
                                                        const double* __restrict__ dwall, double weight,
                                                        double* __restrict__ partial, T* __restrict__ dbar) {
  __shared__ LdsCoef<T> s;
  __shared__ FaceTables ft;
  const double prev = slot_prefetch<NC>(partial);
  const int L = xcd_remap(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
  const int tid = static_cast<int>(threadIdx.x);
  const ColumnTile c = column_tile(cg, L, LP, tid);
  const int i0 = c.i0, kq = c.kq, j = c.j, k4 = c.k4, rw = cg.rw;
  // both tables are staged after the first field loads are in flight; every
  // thread passes this barrier once
  auto ready = [&]() {
    load_tables(s, cf, tid, kBlock);
    load_face_tables<NC>(ft, dtab, dwall);
    __syncthreads();
  };
  FaceAcc<T, BC, NC, KIND == kTermJ> face(g, ft, j, k4, kq, rw, min(i0 + LP, g.nx), dbar, static_cast<T>(weight));
  const bool live = j < g.ny && k4 < (g.nz >> 2);
  if (live) face.load(y, i0);
  sweep_column4<T, BC, LP, KIND, kGeneric, false>(g, cf.labels, s, a, i0, j, k4, kq, rw, live, ready, face);
  block_accumulate<NC>(face.acc, weight, partial, prev);
}

// Launch shape of k_sweep_face4: the sweeps' z-segments, Tiling::flp planes
// per lane.
Tiling sweep_face_tiling(const Tiling& tl) {
  Tiling f = tl;
  f.lp = (tl.flp == 2 || tl.flp == 4) ? tl.flp : 1;
  f.nt = 0;
  return f;
}

template <typename T, int BC, int KIND>
hipError_t sweep_face_typed(const Geom& g, const Tiling& tl, const Coef& cf, const SweepArgs& a, int nclass,
                            const void* y, const double* dtab, const double* dwall, double weight, double* partial,
                            void* dbar, hipStream_t st) {
  const Tiling ft = sweep_face_tiling(tl);
  const int rows = kBlock / ft.rw;
  const ColumnGrid cg(((g.nz >> 2) + ft.rw - 1) / ft.rw, (g.ny + rows - 1) / rows, ft.rw);
  const dim3 grid(static_cast<unsigned>(sweep_blocks(g, ft))), block(kBlock);
  const T* yy = static_cast<const T*>(y);
  T* db = static_cast<T*>(dbar);
#define EXPINT_SWEEP_FACE(NC_, LP_)                                                                     \
  k_sweep_face4<T, BC, KIND, NC_, LP_><<<grid, block, 0, st>>>(g, cg, cf, a, yy, dtab, dwall, weight,      \
                                                              partial, db)
#define EXPINT_SWEEP_FACE_LP(NC_)                     \
  switch (ft.lp) {                                    \
    case 1: EXPINT_SWEEP_FACE(NC_, 1); break;         \
    case 2: EXPINT_SWEEP_FACE(NC_, 2); break;         \
    default: EXPINT_SWEEP_FACE(NC_, 4); break;        \
  }
  switch (nclass) {
    case 1: EXPINT_SWEEP_FACE_LP(1); break;
    case 2: EXPINT_SWEEP_FACE_LP(2); break;
    case 3: EXPINT_SWEEP_FACE_LP(3); break;
    case 4: EXPINT_SWEEP_FACE_LP(4); break;
    default: EXPINT_SWEEP_FACE_LP(8); break;
  }
#undef EXPINT_SWEEP_FACE_LP
#undef EXPINT_SWEEP_FACE
  return hipGetLastError();
}

template <int KIND>
hipError_t sweep_face(expint_dtype dt, expint_bc bc, const Geom& g, const Tiling& tl, const Coef& cf,
                      const SweepArgs& a, int nclass, const void* y, const double* dtab, const double* dwall,
                      double weight, double* partial, void* dbar, hipStream_t st) {
  if (dt == EXPINT_F64) {
    if (bc == EXPINT_NOFLUX)
      return sweep_face_typed<double, 0, KIND>(g, tl, cf, a, nclass, y, dtab, dwall, weight, partial, dbar, st);
    return sweep_face_typed<double, 1, KIND>(g, tl, cf, a, nclass, y, dtab, dwall, weight, partial, dbar, st);
  }
  if (bc == EXPINT_NOFLUX)
    return sweep_face_typed<float, 0, KIND>(g, tl, cf, a, nclass, y, dtab, dwall, weight, partial, dbar, st);
  return sweep_face_typed<float, 1, KIND>(g, tl, cf, a, nclass, y, dtab, dwall, weight, partial, dbar, st);
}

// Tiling of the vectorised face products: the z-segments of the sweeps'
// tiling, kFaceLP planes per lane.
Tiling face_tiling(const Tiling& tl) {
  Tiling f = tl;
  f.lp = kFaceLP;
  return f;
}

template <typename T, int BC, int NC>
void faceprod_nc(const Geom& g, const Tiling& tl, bool vec, const uint8_t* labels, const double* dtab,
                 const double* dwall, const T* yb, const T* y, double weight, double* partial, hipStream_t st) {
  const dim3 block(kBlock);
  if (vec) {
    const Tiling ft = face_tiling(tl);
    const int rows = kBlock / ft.rw;
    const ColumnGrid cg(((g.nz >> 2) + ft.rw - 1) / ft.rw, (g.ny + rows - 1) / rows, ft.rw);
    const dim3 grid(static_cast<unsigned>(sweep_blocks(g, ft)));
    k_faceprod4<T, BC, NC><<<grid, block, 0, st>>>(g, cg, labels, dtab, dwall, yb, y, weight, partial);
  } else {
    k_faceprod<T, BC, NC><<<dim3(kReduceBlocks), block, 0, st>>>(g, labels, dtab, dwall, yb, y, weight, partial);
  }
}

template <typename T, int BC>
void faceprod_bc(const Geom& g, const Tiling& tl, bool vec, const uint8_t* labels, int nclass, const double* dtab,
                 const double* dwall, const T* yb, const T* y, double weight, double* partial, hipStream_t st) {
  switch (nclass) {
    case 1: faceprod_nc<T, BC, 1>(g, tl, vec, labels, dtab, dwall, yb, y, weight, partial, st); break;
    case 2: faceprod_nc<T, BC, 2>(g, tl, vec, labels, dtab, dwall, yb, y, weight, partial, st); break;
    case 3: faceprod_nc<T, BC, 3>(g, tl, vec, labels, dtab, dwall, yb, y, weight, partial, st); break;
    case 4: faceprod_nc<T, BC, 4>(g, tl, vec, labels, dtab, dwall, yb, y, weight, partial, st); break;
    default: faceprod_nc<T, BC, 8>(g, tl, vec, labels, dtab, dwall, yb, y, weight, partial, st); break;
  }
}

template <typename T>
hipError_t faceprod_typed(expint_bc bc, const Geom& g, const Tiling& tl, const uint8_t* labels, int nclass,
                          const double* dtab, const double* dwall, const void* ybar, const void* y, double weight,
                          double* partial, hipStream_t st) {
  auto* a = static_cast<const T*>(ybar);
  auto* b = static_cast<const T*>(y);
  const uintptr_t m = 4 * sizeof(T) - 1;
  const bool vec = tl.vec && vec_sweep_ok(g, true) && (reinterpret_cast<uintptr_t>(a) & m) == 0 &&
                   (reinterpret_cast<uintptr_t>(b) & m) == 0 && (reinterpret_cast<uintptr_t>(labels) & 3) == 0;
  if (bc == EXPINT_NOFLUX) faceprod_bc<T, 0>(g, tl, vec, labels, nclass, dtab, dwall, a, b, weight, partial, st);
  else faceprod_bc<T, 1>(g, tl, vec, labels, nclass, dtab, dwall, a, b, weight, partial, st);
  return hipGetLastError();
}

}  // namespace

int64_t faceprod_slots(const Geom& g, const Tiling& tl) {
  int64_t n = kReduceBlocks;
  if (tl.vec && vec_sweep_ok(g, true)) {
    n = std::max<int64_t>(n, sweep_blocks(g, face_tiling(tl)));
    n = std::max<int64_t>(n, sweep_blocks(g, sweep_face_tiling(tl)));
  }
  return n;
}

bool sweep_face_ok(expint_dtype dt, const Geom& g, const Tiling& tl, const Coef& cf,
                   std::initializer_list<const void*> fields) {
  if (!tl.vec || !cf.labels_form || !vec_sweep_ok(g, true) || !tiling_valid(sweep_face_tiling(tl))) return false;
  if ((reinterpret_cast<uintptr_t>(cf.labels) & 3) != 0) return false;
  const uintptr_t m = 4 * dtype_bytes(dt) - 1;
  for (const void* p : fields)
    if ((reinterpret_cast<uintptr_t>(p) & m) != 0) return false;
  return true;
}

hipError_t launch_term_face(expint_dtype dt, expint_bc bc, const Geom& g, const Tiling& tl, const Coef& cf,
                            const TermOp& op, int nclass, const void* y, const double* dtab, const double* dwall,
                            double weight, double* partial, void* dbar, hipStream_t st) {
  if (op.flavor != kGeneric || (op.ju != nullptr) != (dbar != nullptr) ||
      !sweep_face_ok(dt, g, tl, cf, {op.src, op.bsrc, op.acc_in, op.y_out, op.acc_out, op.u, op.bsrc2, op.ju, y, dbar}))
    return hipErrorInvalidValue;
  SweepArgs a{};
  a.op = op;
  if (op.ju) return sweep_face<kTermJ>(dt, bc, g, tl, cf, a, nclass, y, dtab, dwall, weight, partial, dbar, st);
  return sweep_face<kTerm>(dt, bc, g, tl, cf, a, nclass, y, dtab, dwall, weight, partial, nullptr, st);
}

hipError_t launch_adj_rhs_face(expint_dtype dt, expint_bc bc, const Geom& g, const Tiling& tl, const Coef& cf,
                               const void* gv, const void* u, const void* lam_in, void* lam_out, double rho,
                               int nclass, const double* dtab, const double* dwall, double weight, double* partial,
                               hipStream_t st) {
  if (!sweep_face_ok(dt, g, tl, cf, {gv, u, lam_in, lam_out})) return hipErrorInvalidValue;
  SweepArgs a{};
  a.x = gv;
  a.out = lam_out;
  a.aux0 = lam_in;
  a.aux1 = u;
  a.rho = rho;
  return sweep_face<kAdjRhs>(dt, bc, g, tl, cf, a, nclass, u, dtab, dwall, weight, partial, nullptr, st);
}

hipError_t launch_faceprod(expint_dtype dt, expint_bc bc, const Geom& g, const Tiling& tl, const uint8_t* labels,
                           int nclass, const double* dtab, const double* dwall, const void* ybar, const void* y,
                           double weight, double* partial, hipStream_t st) {
  if (dt == EXPINT_F64) return faceprod_typed<double>(bc, g, tl, labels, nclass, dtab, dwall, ybar, y, weight, partial, st);
  return faceprod_typed<float>(bc, g, tl, labels, nclass, dtab, dwall, ybar, y, weight, partial, st);
}

hipError_t launch_faceprod_final(const double* partial, int64_t slots, double* acc, hipStream_t st) {
  k_faceprod_final<<<1, kBlock, 0, st>>>(partial, static_cast<int>(slots), acc);
  return hipGetLastError();
}

}  // namespace expint
