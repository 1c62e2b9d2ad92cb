// Modal (per-axis mode product) form of tau phi1(tau A) for uniform D.
#pragma once

#include <vector>

#include "internal.hpp"

namespace expint {

enum ModalPrec { kPrecF64 = 0, kPrecF32 = 1, kPrecBF16 = 2, kPrecF16 = 3 };
enum ModalEpi { kEpiStore = 0, kEpiMul = 1, kEpiAddU = 2 };

// One mode product.  The field is viewed as (pre, n, post); side 0 maps
// out[p][i'][q] = sum_i Qop[i'][i] in[p][i][q] (post >= 1), side 1 maps
// out[p][i'] = sum_i Qop[i'][i] in[p][i] (post == 1).  q is the n x n operator
// in the element type of the precision (split precisions: hi matrix followed
// by the lo matrix).  kEpiMul (side 0, x axis, pre == 1) multiplies element
// (i, j, k) by tau phi1(tauD (lam_x[i] + lam_y[j] + lam_z[k])); kEpiAddU
// (side 1) adds the result into out.
struct ModalArgs {
  const void* in = nullptr;
  void* out = nullptr;
  const void* q = nullptr;
  int pre = 1, n = 1;
  long post = 1;
  const double* lam_x = nullptr;
  const double* lam_y = nullptr;
  const double* lam_z = nullptr;
  double tauD = 0.0, tau = 0.0;
  int nz = 1;
};

hipError_t launch_mode_product(int prec, int side, int epi, const ModalArgs& a, hipStream_t st);

// Mode products in the zero-flux (cosine) basis by fast transforms: the
// orthonormal DCT-II (forward, Q^T) or DCT-III (inverse, Q) of every pencil
// along the middle axis of (pre, n, post) (side 0) or along the contiguous
// axis (side 1, post == 1), n a power of two from 32 to 256 (dct_axis_ok).
enum DctMode { kDctFwd = 0, kDctInv = 1, kDctFwdMulInv = 2, kDctRhsFwd = 3 };
struct DctArgs {
  const void* in = nullptr;
  void* out = nullptr;
  int pre = 1, n = 1;
  long post = 1;
  const double* tw = nullptr;  // 2n: cos, -sin of 2 pi e / n for e < n (16-byte aligned)
  const double* mk = nullptr;  // 2n: cos, sin of pi k / (2n) for k < n (16-byte aligned)
  double c0 = 0.0, c1 = 0.0;   // set by launch_mode_dct: sqrt(1/n), sqrt(2/n)
  // kDctFwdMulInv (side 0, x axis, pre == 1): between the two transforms
  // element (i, j, k) is multiplied by tau phi1(tauD (lam_x[i] + lam_y[j] +
  // lam_z[k])), as kEpiMul does
  const double* lam_x = nullptr;
  const double* lam_y = nullptr;
  const double* lam_z = nullptr;
  double tauD = 0.0, tau = 0.0;
  int nz = 1;
  // kDctRhsFwd (side 1, z axis, pre == nx ny): `in` is the state u and the
  // pass transforms b = dh2 L u + rho u (1 - u) instead, L the zero-flux
  // 7-point Laplacian of the nx x ny x n grid (faces at the walls left out)
  double dh2 = 0.0, rho = 0.0;
  int nx = 1, ny = 1;
};
bool dct_axis_ok(int n);
// A side-0 pass addresses a thread's elements from a 32-bit offset within a
// tile row: false where a pass along an axis of n points with `post` columns
// would need more (FP64 x axis: ny nz of 2^26 or more), so that axis keeps
// the dense products.
bool dct_rows_ok(int prec, int n, int side, long post);
// prec kPrecF64 or kPrecF32; mode DctMode; epi kEpiStore or (kDctInv, side 1)
// kEpiAddU; kDctRhsFwd needs side 1 and ny a multiple of the workgroup's
// pencil count (32 suffices).  hipErrorInvalidValue for anything else.
hipError_t launch_mode_dct(int prec, int side, int mode, int epi, const DctArgs& a, hipStream_t st);
// The tables of DctArgs for an axis of n points (host arrays).
void dct_tables(int n, std::vector<double>& tw, std::vector<double>& mk);
hipError_t launch_label_mask(const uint8_t* labels, int64_t n, unsigned* mask, hipStream_t st);

}  // namespace expint
