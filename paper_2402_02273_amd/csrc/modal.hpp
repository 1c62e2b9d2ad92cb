// Modal (per-axis mode product) form of tau phi1(tau A) for uniform D.
#pragma once

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
hipError_t launch_label_mask(const uint8_t* labels, int64_t n, unsigned* mask, hipStream_t st);

}  // namespace expint
