// Class-diffusivity derivatives of the bilinear form <ybar, A y> for the
// discrete adjoint of the exponential Euler step (label form).
//
// With the conservative operator (A y)_p = sum_q K_pq (y_q - y_p) / h^2,
//   <ybar, A y> = - sum over faces p|q of K_pq (ybar_p - ybar_q)(y_p - y_q) / h^2
//                 - sum over zero-Dirichlet wall faces of D_p ybar_p y_p / h^2,
// so its derivative with respect to the diffusivity D_c of tissue class c is
// a weighted sum of face products: the weights -dK(D_a, D_b)/dD_c / h^2 (and
// -[a == c] / h^2 at walls) come precomputed per class pair in FP64.  Every
// face is visited once (the +x, +y, +z faces of each voxel); partial sums are
// per workgroup in FP64 and combined in a fixed order, so results are
// bit-reproducible.

#include "internal.hpp"

namespace expint {

namespace {

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T, int BC>
__global__ __launch_bounds__(kBlock) void k_faceprod(Geom g, const uint8_t* __restrict__ lab, int nclass,
                                                     const double* __restrict__ dtab, const double* __restrict__ dwall,
                                                     const T* __restrict__ yb, const T* __restrict__ y,
                                                     double* __restrict__ partial) {
  __shared__ double st[kMaxClasses * kTab];
  __shared__ double sw[kMaxClasses * kMaxClasses];
  __shared__ double red[kBlock / 64][kMaxClasses];
  for (int t = threadIdx.x; t < kMaxClasses * kTab; t += kBlock) st[t] = dtab[t];
  if (threadIdx.x < kMaxClasses * kMaxClasses) sw[threadIdx.x] = dwall[threadIdx.x];
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
    const double* row = st + lp * kMaxClasses;  // + c * kTab + l_q
    auto face = [&](int q) {
      const double prod = (ybp - static_cast<double>(yb[q])) * (yp - static_cast<double>(y[q]));
      const double* w = row + lab[q];
#pragma unroll
      for (int c = 0; c < kMaxClasses; ++c)
        if (c < nclass) acc[c] += w[c * kTab] * prod;
    };
    if (i < g.nx - 1) face(p + sx);
    if (j < g.ny - 1) face(p + sy);
    if (k < g.nz - 1) face(p + 1);
    if (BC) {
      const int nw = (i == 0) + (i == g.nx - 1) + (j == 0) + (j == g.ny - 1) + (k == 0) + (k == g.nz - 1);
      if (nw) {
        const double v = ybp * yp * nw;
#pragma unroll
        for (int c = 0; c < kMaxClasses; ++c)
          if (c < nclass) acc[c] += sw[c * kMaxClasses + lp] * v;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < kMaxClasses; ++c) {
    const double v = wave_sum(acc[c]);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][c] = v;
  }
  __syncthreads();
  if (threadIdx.x < kMaxClasses) {
    double v = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) v += red[w][threadIdx.x];
    partial[blockIdx.x * kMaxClasses + threadIdx.x] = v;
  }
}

// acc[c] += weight * sum over workgroups of partial[b][c].  Thread t sums the
// partials b = t, t + 256, ... of every class, then a fixed-order tree over
// the 256 threads: the combination order never changes (bit-reproducible).
__global__ __launch_bounds__(kBlock) void k_faceprod_final(const double* __restrict__ partial, int nb, double weight,
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
  if (t < kMaxClasses) acc[t] += weight * red[0][t];
}

}  // namespace

hipError_t launch_faceprod(expint_dtype dt, expint_bc bc, const Geom& g, const uint8_t* labels, int nclass,
                           const double* dtab, const double* dwall, const void* ybar, const void* y, double weight,
                           double* partial, double* acc, hipStream_t st) {
  const dim3 grid(kReduceBlocks), block(kBlock);
  if (dt == EXPINT_F64) {
    auto* a = static_cast<const double*>(ybar);
    auto* b = static_cast<const double*>(y);
    if (bc == EXPINT_NOFLUX) k_faceprod<double, 0><<<grid, block, 0, st>>>(g, labels, nclass, dtab, dwall, a, b, partial);
    else k_faceprod<double, 1><<<grid, block, 0, st>>>(g, labels, nclass, dtab, dwall, a, b, partial);
  } else {
    auto* a = static_cast<const float*>(ybar);
    auto* b = static_cast<const float*>(y);
    if (bc == EXPINT_NOFLUX) k_faceprod<float, 0><<<grid, block, 0, st>>>(g, labels, nclass, dtab, dwall, a, b, partial);
    else k_faceprod<float, 1><<<grid, block, 0, st>>>(g, labels, nclass, dtab, dwall, a, b, partial);
  }
  k_faceprod_final<<<1, kBlock, 0, st>>>(partial, kReduceBlocks, weight, acc);
  return hipGetLastError();
}

}  // namespace expint
