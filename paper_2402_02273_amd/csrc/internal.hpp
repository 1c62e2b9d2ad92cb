// Internal declarations shared by the host runtime and the HIP kernels of the
// exponential-integrator library.  Nothing here crosses the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "expint.h"

namespace expint {

constexpr int kMaxClasses = EXPINT_MAX_CLASSES;
constexpr int kTab = kMaxClasses * kMaxClasses;
constexpr int kBlock = 256;        // threads per workgroup of the field kernels
constexpr int kReduceBlocks = 1024;  // fixed partial count -> deterministic reductions

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
// Workgroups of one voxel-kernel launch (gx * gy * nx).
int64_t field_block_count(const Geom& g);

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
//   y   = c * a + cb * bsrc            (bsrc may be NULL)
//   acc = (acc_in ? acc_in : alpha * src) + y
//   u != NULL : u += acc               (last term of a step; nothing else written)
//   otherwise : y_out = y (if non-NULL), acc_out = acc
struct TermOp {
  const void* src;
  const void* bsrc;
  const void* acc_in;
  void* y_out;
  void* acc_out;
  void* u;
  double c, cb, alpha;
};

// ---- launchers (stencil.hip) ----
hipError_t launch_term(expint_dtype dt, expint_bc bc, const Geom& g, const Coef& cf, const TermOp& op,
                       hipStream_t st);
hipError_t launch_rhs(expint_dtype dt, expint_bc bc, const Geom& g, const Coef& cf, const void* u, void* b,
                      double rho, hipStream_t st);
hipError_t launch_apply(expint_dtype dt, expint_bc bc, const Geom& g, const Coef& cf, const void* x, void* y,
                        hipStream_t st);

// ||A||_1 and input validation, FP64.  partial: 2 * field_block_count(g)
// doubles of workspace; out[0] = max column sum of |A|, out[1] = 1 if a label >= nclass or
// a D value is negative / not finite (else 0).
hipError_t launch_scan_labels(expint_bc bc, const Geom& g, const uint8_t* labels, int nclass, const double* tab64,
                              const double* wall64, double* partial, double* out, hipStream_t st);
// Dense form: also writes the face coefficients of dtype dt.
hipError_t launch_scan_dense(expint_dtype dt, expint_bc bc, const Geom& g, const void* D, double inv_h2, void* fx,
                             void* fy, void* fz, void* wallv, double* partial, double* out, hipStream_t st);

// Deterministic two-pass FP64 reductions: op 0 sum x, 1 sum x*y, 2 max|x|,
// 3 count of non-finite x.  partial: kReduceBlocks doubles; out: 1 double.
hipError_t launch_reduce(expint_dtype dt, int op, const void* x, const void* y, int64_t n, double* partial,
                         double* out, hipStream_t st);

// Pointwise helpers.
hipError_t launch_axpy(expint_dtype dt, int64_t n, double a, const void* x, void* y, hipStream_t st);  // y += a x
hipError_t launch_copy(expint_dtype dt, int64_t n, const void* x, void* y, hipStream_t st);
hipError_t launch_fill(expint_dtype dt, int64_t n, double v, void* y, hipStream_t st);

}  // namespace expint
