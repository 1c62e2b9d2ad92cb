// Internal declarations shared by the host runtime and the HIP kernels of the
// exponential-integrator library.  Nothing here crosses the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <initializer_list>

#include "expint.h"

namespace expint {

constexpr int kMaxClasses = EXPINT_MAX_CLASSES;
constexpr int kTab = kMaxClasses * kMaxClasses;
constexpr int kBlock = 256;        // threads per workgroup of the field kernels
constexpr int kReduceBlocks = 1024;  // fixed partial count -> deterministic reductions

// a * b * c if it is at most `limit` (all of them >= 0), else -1: element
// counts of grids from 32-bit dimensions without signed overflow.
inline int64_t product_within(int64_t a, int64_t b, int64_t c, int64_t limit) {
  if (a < 0 || b < 0 || c < 0) return -1;
  if (b != 0 && a > limit / b) return -1;
  const int64_t ab = a * b;
  if (c != 0 && ab > limit / c) return -1;
  return ab * c;
}

// The int a C caller stored in an enumeration field or argument.  A C caller
// may store any int there; reading it as the enumeration type before it is
// validated would be undefined, so validation reads it through this.
template <typename E>
inline int enum_value(const E& e) {
  static_assert(sizeof(E) == sizeof(int), "C enumerations are int-sized");
  int v;
  __builtin_memcpy(&v, &e, sizeof v);
  return v;
}

inline constexpr int dtype_bytes(expint_dtype dt) { return dt == EXPINT_F64 ? 8 : 4; }

// Unsigned division by a divisor d (1 <= d < 2^31) fixed at launch, for
// dividends below 2^31, as a multiply and a shift: with s = 31 + ceil(log2 d)
// and m = ceil(2^s / d) (below 2^32), floor(x * m / 2^s) = floor(x / d).
// (m d - 2^s < d and x < 2^31 <= 2^s / d keep x (m d - 2^s) / (d 2^s) below
// 1/d, less than the gap between x / d and the next integer.)  With a dividend
// that is uniform over the wavefront the kernels compute it on the scalar
// unit, where a runtime division would take a float reciprocal on the vector
// unit.
struct FastDiv {
  uint32_t d = 1, m = 1u << 31, s = 31;
  FastDiv() = default;
  explicit FastDiv(uint32_t divisor) : d(divisor) {
    uint32_t l = 0;
    while ((1ull << l) < divisor) ++l;
    s = 31 + l;
    m = static_cast<uint32_t>(((1ull << s) + divisor - 1) / divisor);
  }
  __host__ __device__ uint32_t div(uint32_t x) const {
    return static_cast<uint32_t>((static_cast<uint64_t>(x) * m) >> s);
  }
};

// Tile decomposition of the z-vectorised sweeps: workgroup L covers
// z-segment L % gzs (rw lanes of 4 voxels), row block (L / gzs) % gy of
// kBlock / rw rows and the plane group L / (gzs gy); rw is a power of two.
struct ColumnGrid {
  FastDiv zs, y;  // gzs, gy
  int rw, rw_log2;
  ColumnGrid() = default;
  ColumnGrid(int gzs, int gy, int rw_) : zs(static_cast<uint32_t>(gzs)), y(static_cast<uint32_t>(gy)), rw(rw_), rw_log2(0) {
    while ((1 << rw_log2) < rw) ++rw_log2;
  }
};

struct Geom {
  int nx, ny, nz;
  int64_t n;
};

// Launch shape of the voxel kernels: blockDim = (bx, by), workgroups cover
// z in chunks of bx and y in chunks of by, one x-plane per workgroup row.
struct Shape {
  int bx, by;  // threads along z and y, bx * by == kBlock
  int gx, gy;  // workgroups along z and y
};
Shape choose_shape(const Geom& g);
// Workgroups of one scan launch (gx * gy * nx, one x-plane per workgroup row).
int64_t field_block_count(const Geom& g);

// Tiling of the stencil sweeps: a workgroup of bx (z) x by (y) threads covers
// a bx-by-by patch of lp consecutive x-planes; each thread marches through its
// lp planes (1, 2 or 4) keeping the x-neighbours in registers.  vec != 0
// selects the z-vectorised sweep instead (label form, nz % 4 == 0): a lane
// owns four consecutive z voxels, a 256-thread workgroup covers 256 / rw rows
// of one z-segment of rw lanes (rw in 16, 32, 64) and lp x-planes.
struct Tiling {
  int bx = 64, by = 4, lp = 4;
  int vec = 0, rw = 64;
  int nt = 0;  // z-vectorised Taylor-term sweeps of A: non-temporal output stores
  // x-planes per lane of the adjoint's fused reverse sweeps (1, 2 or 4); set
  // per context, not by the sweep autotuner
  int flp = 1;
};
// Whether the z-vectorised sweep handles this grid and coefficient form.
bool vec_sweep_ok(const Geom& g, bool labels_form);
bool tiling_valid(const Tiling& t);
int64_t sweep_blocks(const Geom& g, const Tiling& t);
Tiling default_tiling(const Geom& g);

// Device-side diffusion coefficients of one operator, already divided by h^2.
//  label form : labels (uint8 per voxel), tab[a * 8 + b] = K(D_a, D_b) / h^2,
//               wallc[a] = D_a / h^2 (zero-Dirichlet ghost faces only)
//  dense form : fx/fy/fz[p] = K between p and its +x/+y/+z neighbour, / h^2,
//               wallv[p] = D_p / h^2
struct Coef {
  bool labels_form;
  const uint8_t* labels;
  const void* tab;
  const void* wallc;
  const void* fx;
  const void* fy;
  const void* fz;
  const void* wallv;
};

// One fused Taylor-term sweep (all pointers device, same dtype):
//   a   = A src
//   y   = c * a + cb * bsrc                    (bsrc may be NULL)
//   v   = ca * acc_in + cs * src + y           (acc_in may be NULL)
//   u != NULL : u += v                         (last sweep of a step)
//   otherwise : y_out = y and acc_out = v      (each only if non-NULL)
// `flavor` names the pointer pattern so the kernel can be specialised;
// classify_term() sets it.
enum TermFlavor {
  kGeneric = 0,
  kSkip = 1,      // y_out only
  kFlushY = 2,    // acc_out = acc_in + cs*src + y (ca == 1), and y_out
  kFlushNoY = 3,  // the same without y_out
  kFirst = 4,     // y = c*a + cb*bsrc; acc_out = cs*src + y; y_out
};

//
// bsrc2 != NULL adds a second source vector to the term, y += cb2 * bsrc2
// (the phi2 vector of the augmented matrix with both omega columns); such
// sweeps take the generic flavour.  Single-term sweeps only.
//
// ju != NULL makes the sweep one of the linearised operator
// J = A + rho diag(1 - 2 u_n): a = A src + jrho (1 - 2 ju) src, with ju = u_n
// read at each voxel only (so ju may be the u the last sweep adds into).
// Single-term sweeps only.
//
// A pair sweep (pair != 0, label form only) evaluates two consecutive terms:
//   y   = c * A src + cb * bsrc                (term j, kept on chip)
//   w   = c2 * A y                             (term j + 1)
//   v   = ca * acc_in + cs * src + y + w
//   u != NULL : u += v
//   otherwise : y_out = w and acc_out = v      (each only if non-NULL)
// A pair sweep reads src and bsrc around its tile, so neither may alias an
// output of the same sweep.
struct TermOp {
  const void* src = nullptr;
  const void* bsrc = nullptr;
  const void* acc_in = nullptr;
  void* y_out = nullptr;
  void* acc_out = nullptr;
  void* u = nullptr;
  double c = 0.0, cb = 0.0, ca = 0.0, cs = 0.0;
  double c2 = 0.0;
  const void* ju = nullptr;
  double jrho = 0.0;
  const void* bsrc2 = nullptr;  // a second source: y += cb2 * bsrc2 (generic flavour)
  double cb2 = 0.0;
  int flavor = kGeneric;
  int pair = 0;
};

void classify_term(TermOp& op);

// Tiling of the pair sweeps: a workgroup of 256 threads covers 64 (z) x ty
// (y) output columns of lp consecutive x-planes; ty == 0 means the pair
// sweeps are not used (every term is its own sweep).
struct PairTiling {
  int ty = 0, lp = 8;
};
bool pair_tiling_valid(const PairTiling& t);
// Whether pair sweeps handle this grid (an x-plane of fields below 4 GiB).
bool pair_grid_ok(const Geom& g, expint_dtype dt);
int64_t pair_blocks(const Geom& g, const PairTiling& t);

// ---- launchers (stencil.hip, pair.hip) ----
hipError_t launch_pair(expint_dtype dt, expint_bc bc, const Geom& g, const PairTiling& tl, const Coef& cf,
                       const TermOp& op, hipStream_t st);
hipError_t launch_term(expint_dtype dt, expint_bc bc, const Geom& g, const Tiling& tl, const Coef& cf,
                       const TermOp& op, hipStream_t st);
// launch_term for op.ju != NULL (stencil_lin.hip)
hipError_t launch_term_lin(expint_dtype dt, expint_bc bc, const Geom& g, const Tiling& tl, const Coef& cf,
                           const TermOp& op, hipStream_t st);
hipError_t launch_rhs(expint_dtype dt, expint_bc bc, const Geom& g, const Tiling& tl, const Coef& cf, const void* u,
                      void* b, double rho, hipStream_t st);
hipError_t launch_apply(expint_dtype dt, expint_bc bc, const Geom& g, const Tiling& tl, const Coef& cf,
                        const void* x, void* y, hipStream_t st);

// ||A||_1 and input validation, FP64.  partial: 2 * field_block_count(g)
// doubles of workspace; out[0] = max column sum of |A|, out[1] = 1 if a label >= nclass or
// a D value is negative / not finite (else 0).
hipError_t launch_scan_labels(expint_bc bc, const Geom& g, const uint8_t* labels, int nclass, const double* tab64,
                              const double* wall64, double* partial, double* out, hipStream_t st);
// Dense form: also writes the face coefficients of dtype dt.
hipError_t launch_scan_dense(expint_dtype dt, expint_bc bc, const Geom& g, const void* D, double inv_h2, void* fx,
                             void* fy, void* fz, void* wallv, double* partial, double* out, hipStream_t st);

// Deterministic two-pass FP64 reductions: op 0 sum x, 1 sum x*y, 2 max|x|,
// 3 count of non-finite x, 4 sum x*y*(1-y), 5 sum (x-y)^2,
// 6 sum x*(1-2y).  partial:
// kReduceBlocks doubles; out: 1 double, overwritten or (accumulate) added to.
hipError_t launch_reduce(expint_dtype dt, int op, const void* x, const void* y, int64_t n, double* partial,
                         double* out, hipStream_t st, bool accumulate = false);

// lambda_out = lambda_in + A g + rho (1 - 2 u) g  (adjoint of one step's
// right-hand side; lambda_out may equal lambda_in).
hipError_t launch_adj_rhs(expint_dtype dt, expint_bc bc, const Geom& g, const Tiling& tl, const Coef& cf,
                          const void* gv, const void* u, const void* lam_in, void* lam_out, double rho,
                          hipStream_t st);

// Class-diffusivity derivatives of <ybar, A y> (label form), accumulated on
// the device: workgroup b of the launch adds
//   weight * ( sum over its interior faces p|q of dtab[c][l_p][l_q] (ybar_p - ybar_q)(y_p - y_q)
//            + sum over its zero-Dirichlet wall faces of dwall[c][l_p] ybar_p y_p )
// into partial[b * 8 + c], with dtab[c] = -(dK/dD_c)/h^2 and dwall[c][a] =
// -[a == c]/h^2, so the slots accumulate <ybar, (dA/dD_c) y>.  The launch
// uses the z-vectorised form in tiling tl when tl.vec is set and the fields are
// 4-value aligned, else a scalar grid-stride form; partial needs
// faceprod_slots(g, tl) * 8 doubles, zeroed before the first launch.
// launch_faceprod_final adds the slot sums (fixed order) into acc[0..7].
// dtab: 8 x 64 FP64, dwall: 8 x 8 FP64 (device).
int64_t faceprod_slots(const Geom& g, const Tiling& tl);
hipError_t launch_faceprod(expint_dtype dt, expint_bc bc, const Geom& g, const Tiling& tl, const uint8_t* labels,
                           int nclass, const double* dtab, const double* dwall, const void* ybar, const void* y,
                           double weight, double* partial, hipStream_t st);
hipError_t launch_faceprod_final(const double* partial, int64_t slots, double* acc, hipStream_t st);

// A sweep and the face products of its stencil source in one pass (the
// z-vectorised shape of tl with one plane per lane; label form; every field
// 4-value aligned: sweep_face_ok).  launch_term_face: the Taylor-term sweep op
// (generic flavour) plus weight <op.src, (dA/dD_c) y>; for a term of the
// linearised operator (op.ju set, dbar given) also dbar += weight op.src * y,
// as launch_diag_accumulate; launch_adj_rhs_face: launch_adj_rhs plus
// weight <gv, (dA/dD_c) u>.  The face products go into the same slots as
// launch_faceprod (partial holds faceprod_slots(g, tl) * 8 doubles).
// hipErrorInvalidValue where the fused form does not apply.
bool sweep_face_ok(expint_dtype dt, const Geom& g, const Tiling& tl, const Coef& cf,
                   std::initializer_list<const void*> fields);
hipError_t launch_term_face(expint_dtype dt, expint_bc bc, const Geom& g, const Tiling& tl, const Coef& cf,
                            const TermOp& op, int nclass, const void* y, const double* dtab, const double* dwall,
                            double weight, double* partial, void* dbar, hipStream_t st);
hipError_t launch_adj_rhs_face(expint_dtype dt, expint_bc bc, const Geom& g, const Tiling& tl, const Coef& cf,
                               const void* gv, const void* u, const void* lam_in, void* lam_out, double rho,
                               int nclass, const double* dtab, const double* dwall, double weight, double* partial,
                               hipStream_t st);

// Pointwise helpers.
hipError_t launch_axpy(expint_dtype dt, int64_t n, double a, const void* x, void* y, hipStream_t st);  // y += a x
hipError_t launch_copy(expint_dtype dt, int64_t n, const void* x, void* y, hipStream_t st);
hipError_t launch_axpby(expint_dtype dt, int64_t n, double a, const void* x, double b, const void* y, void* out,
                        hipStream_t st);  // out = a x + b y
hipError_t launch_fill(expint_dtype dt, int64_t n, double v, void* y, hipStream_t st);
// d += w ybar y pointwise (the adjoint of the linearised operator's diagonal)
hipError_t launch_diag_accumulate(expint_dtype dt, int64_t n, double w, const void* ybar, const void* y, void* d,
                                  hipStream_t st);
// d = f(u + x) - f(u) for f(v) = rho v (1 - v), evaluated as rho x (1 - 2u - x)
// (the same polynomial without the cancellation of the difference).
hipError_t launch_reaction_increment(expint_dtype dt, int64_t n, double rho, const void* u, const void* x, void* d,
                                     hipStream_t st);

}  // namespace expint
