// Voxel kernels of the stencil-Taylor path: the 7-point variable-coefficient
// diffusion operator of section 2.1 (conservative flux form, harmonic face
// means), the right-hand side A u + rho u (1 - u) of the incremental
// exponential Euler step (section 2.2), and one fused Taylor term of the
// scaled augmented series with its running sum (section 2.2).
//
// Layout: z fastest, flat index (i * ny + j) * nz + k.  A workgroup covers a
// bx-by-by patch of one x-plane; lanes run along z so every field access of
// a wavefront is one contiguous, coalesced segment.  Workgroups are dealt to
// the 8 XCDs round-robin by the dispatcher; block ids are remapped so each XCD
// sweeps a contiguous run of x-planes and the +-x neighbour planes a
// workgroup reads sit in the same XCD's L2.

#include "internal.hpp"
#include "sweep_device.hpp"
#include "sweep_launch.hpp"

namespace expint {

Shape choose_shape(const Geom& g) {
  Shape s;
  s.bx = g.nz >= 64 ? 64 : (g.nz >= 32 ? 32 : 16);
  s.by = kBlock / s.bx;
  s.gx = (g.nz + s.bx - 1) / s.bx;
  s.gy = (g.ny + s.by - 1) / s.by;
  return s;
}

bool tiling_valid(const Tiling& t) {
  const bool lp_ok = t.lp == 1 || t.lp == 2 || t.lp == 4;
  if (t.vec) return (t.rw == 16 || t.rw == 32 || t.rw == 64) && lp_ok && (t.nt == 0 || t.nt == 1);
  return (t.bx == 64 || t.bx == 32 || t.bx == 16) && t.by * t.bx == kBlock && lp_ok && t.nt == 0;
}

bool vec_sweep_ok(const Geom& g, bool labels_form) { return labels_form && g.nz % 4 == 0; }

int64_t sweep_blocks(const Geom& g, const Tiling& t) {
  if (t.vec) {
    const int64_t nz4 = g.nz / 4, rows = kBlock / t.rw;
    return ((nz4 + t.rw - 1) / t.rw) * ((g.ny + rows - 1) / rows) * ((g.nx + t.lp - 1) / t.lp);
  }
  const int64_t gx = (g.nz + t.bx - 1) / t.bx, gy = (g.ny + t.by - 1) / t.by, gz = (g.nx + t.lp - 1) / t.lp;
  return gx * gy * gz;
}

Tiling default_tiling(const Geom& g) {
  // widest z-row with the least padding; ties to the wider row
  Tiling t;
  int best_waste = -1;
  for (int bx : {64, 32, 16}) {
    const int waste = ((g.nz + bx - 1) / bx) * bx - g.nz;
    if (best_waste < 0 || waste < best_waste) {
      best_waste = waste;
      t.bx = bx;
    }
  }
  t.by = kBlock / t.bx;
  t.lp = 4;
  return t;
}

int64_t field_block_count(const Geom& g) {
  const Shape s = choose_shape(g);
  return static_cast<int64_t>(s.gx) * s.gy * g.nx;
}

namespace {

struct Vox {
  int i, j, k;
  int64_t p;
  bool ok;
};

__device__ __forceinline__ Vox voxel_of(const Geom& g, int gx, int gy) {
  const int L = xcd_remap(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
  const int bxi = L % gx;
  const int t = L / gx;
  const int byi = t % gy;
  Vox v;
  v.i = t / gy;
  v.j = byi * static_cast<int>(blockDim.y) + static_cast<int>(threadIdx.y);
  v.k = bxi * static_cast<int>(blockDim.x) + static_cast<int>(threadIdx.x);
  v.ok = v.k < g.nz && v.j < g.ny && v.i < g.nx;
  v.p = (static_cast<int64_t>(v.i) * g.ny + v.j) * g.nz + v.k;
  return v;
}

// ---------------------------------------------------------------------------
// FP64 scan: ||A||_1 = max_p (|a_pp| + sum_{q != p} |a_qp|) and validation.
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-wide max of two values; thread 0 receives the result.
__device__ __forceinline__ void block_max2(double& a, double& b) {
  __shared__ double sa[kBlock / 64], sb[kBlock / 64];
  const int t = threadIdx.y * blockDim.x + threadIdx.x;
  a = wave_max(a);
  b = wave_max(b);
  if ((t & 63) == 0) {
    sa[t >> 6] = a;
    sb[t >> 6] = b;
  }
  __syncthreads();
  if (t == 0) {
    for (int w = 1; w < kBlock / 64; ++w) {
      a = fmax(a, sa[w]);
      b = fmax(b, sb[w]);
    }
  }
}

__device__ __forceinline__ double harmonic(double a, double b) {
  const double s = a + b;
  return s > 0.0 ? 2.0 * a * b / s : 0.0;
}

template <int BC>
__global__ __launch_bounds__(kBlock) void k_scan_labels(Geom g, int gx, int gy, const uint8_t* __restrict__ lab,
                                                        int nclass, const double* __restrict__ tab64,
                                                        const double* __restrict__ wall64, double* partial) {
  const Vox v = voxel_of(g, gx, gy);
  double col = 0.0, bad = 0.0;
  if (v.ok) {
    const int64_t sx = static_cast<int64_t>(g.ny) * g.nz, sy = g.nz;
    auto cls = [&](int64_t q) -> int {
      const int l = lab[q];
      if (l >= nclass) bad = 1.0;
      return l < nclass ? l : 0;
    };
    const int lp = cls(v.p);
    double off = 0.0, ghost = 0.0;
    const double wl = wall64[lp];
    if (v.i > 0) off += tab64[lp * kMaxClasses + cls(v.p - sx)]; else if (BC) ghost += wl;
    if (v.i < g.nx - 1) off += tab64[lp * kMaxClasses + cls(v.p + sx)]; else if (BC) ghost += wl;
    if (v.j > 0) off += tab64[lp * kMaxClasses + cls(v.p - sy)]; else if (BC) ghost += wl;
    if (v.j < g.ny - 1) off += tab64[lp * kMaxClasses + cls(v.p + sy)]; else if (BC) ghost += wl;
    if (v.k > 0) off += tab64[lp * kMaxClasses + cls(v.p - 1)]; else if (BC) ghost += wl;
    if (v.k < g.nz - 1) off += tab64[lp * kMaxClasses + cls(v.p + 1)]; else if (BC) ghost += wl;
    col = (off + ghost) + off;
  }
  block_max2(col, bad);
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    partial[blockIdx.x] = col;
    partial[gridDim.x + blockIdx.x] = bad;
  }
}

template <typename T, int BC>
__global__ __launch_bounds__(kBlock) void k_scan_dense(Geom g, int gx, int gy, const T* __restrict__ D,
                                                       double inv_h2, T* __restrict__ fx, T* __restrict__ fy,
                                                       T* __restrict__ fz, T* __restrict__ wallv,
                                                       double* partial) {
  const Vox v = voxel_of(g, gx, gy);
  double col = 0.0, bad = 0.0;
  if (v.ok) {
    const int64_t sx = static_cast<int64_t>(g.ny) * g.nz, sy = g.nz;
    auto val = [&](int64_t q) -> double {
      const double d = static_cast<double>(D[q]);
      if (!(d >= 0.0) || !isfinite(d)) bad = 1.0;
      return (d >= 0.0 && isfinite(d)) ? d : 0.0;
    };
    const double dp = val(v.p);
    double off = 0.0, ghost = 0.0;
    double k;
    if (v.i > 0) off += harmonic(dp, val(v.p - sx)); else if (BC) ghost += dp;
    k = v.i < g.nx - 1 ? harmonic(dp, val(v.p + sx)) : 0.0;
    if (v.i < g.nx - 1) off += k; else if (BC) ghost += dp;
    fx[v.p] = static_cast<T>(k * inv_h2);
    if (v.j > 0) off += harmonic(dp, val(v.p - sy)); else if (BC) ghost += dp;
    k = v.j < g.ny - 1 ? harmonic(dp, val(v.p + sy)) : 0.0;
    if (v.j < g.ny - 1) off += k; else if (BC) ghost += dp;
    fy[v.p] = static_cast<T>(k * inv_h2);
    if (v.k > 0) off += harmonic(dp, val(v.p - 1)); else if (BC) ghost += dp;
    k = v.k < g.nz - 1 ? harmonic(dp, val(v.p + 1)) : 0.0;
    if (v.k < g.nz - 1) off += k; else if (BC) ghost += dp;
    fz[v.p] = static_cast<T>(k * inv_h2);
    wallv[v.p] = static_cast<T>(dp * inv_h2);
    col = ((off + ghost) + off) * inv_h2;
  }
  block_max2(col, bad);
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    partial[blockIdx.x] = col;
    partial[gridDim.x + blockIdx.x] = bad;
  }
}

// Single workgroup: max over nb partials of both halves.
__global__ __launch_bounds__(kBlock) void k_final_max2(const double* __restrict__ partial, int nb, double* out) {
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nb; i += kBlock) {
    a = fmax(a, partial[i]);
    b = fmax(b, partial[nb + i]);
  }
  block_max2(a, b);
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = b;
  }
}

// ---------------------------------------------------------------------------
// Deterministic reductions (fixed grid, fixed combination order).
// ---------------------------------------------------------------------------

template <int OP>
__device__ __forceinline__ double combine(double a, double b) {
  if (OP == 2) return fmax(a, b);
  return a + b;
}

template <int OP>
__device__ __forceinline__ double block_reduce(double v) {
  __shared__ double sw[kBlock / 64];
  v = (OP == 2) ? wave_max(v) : wave_sum(v);
  const int t = threadIdx.x;
  if ((t & 63) == 0) sw[t >> 6] = v;
  __syncthreads();
  if (t == 0)
    for (int w = 1; w < kBlock / 64; ++w) v = combine<OP>(v, sw[w]);
  return v;
}

template <typename T, int OP>
__global__ __launch_bounds__(kBlock) void k_reduce(const T* __restrict__ x, const T* __restrict__ y, int64_t n,
                                                   double* partial) {
  double acc = 0.0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < n; p += stride) {
    const double v = static_cast<double>(x[p]);
    if (OP == 0) acc += v;
    if (OP == 1) acc += v * static_cast<double>(y[p]);
    if (OP == 2) acc = fmax(acc, fabs(v));
    if (OP == 3) acc += isfinite(v) ? 0.0 : 1.0;
    if (OP == 4) {
      const double w = static_cast<double>(y[p]);
      acc += v * w * (1.0 - w);
    }
    if (OP == 5) {
      const double d = v - static_cast<double>(y[p]);
      acc += d * d;
    }
    if (OP == 6) acc += v * (1.0 - 2.0 * static_cast<double>(y[p]));
  }
  acc = block_reduce<OP>(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

template <int OP>
__global__ __launch_bounds__(kBlock) void k_reduce_final(const double* __restrict__ partial, int nb, double* out,
                                                         int accumulate) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += kBlock) acc = combine<OP>(acc, partial[i]);
  acc = block_reduce<OP>(acc);
  if (threadIdx.x == 0) out[0] = accumulate ? combine<OP>(out[0], acc) : acc;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_axpy(int64_t n, T a, const T* __restrict__ x, T* __restrict__ y) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (p < n) y[p] += a * x[p];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_axpby(int64_t n, T a, const T* __restrict__ x, T b,
                                                  const T* __restrict__ y, T* __restrict__ out) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (p < n) out[p] = a * x[p] + b * y[p];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy(int64_t n, const T* __restrict__ x, T* __restrict__ y) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (p < n) y[p] = x[p];
}

// d += w ybar y, pointwise
template <typename T>
__global__ __launch_bounds__(kBlock) void k_diag_accumulate(int64_t n, T w, const T* __restrict__ ybar,
                                                            const T* __restrict__ y, T* __restrict__ d) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (p < n) d[p] += w * ybar[p] * y[p];
}

// d = f(u + x) - f(u), f(v) = rho v (1 - v), as rho x (1 - 2u - x)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_reaction_increment(int64_t n, T rho, const T* __restrict__ u,
                                                               const T* __restrict__ x, T* __restrict__ d) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (p < n) {
    const T xv = x[p];
    d[p] = rho * xv * (T(1) - T(2) * u[p] - xv);
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(int64_t n, T v, T* __restrict__ y) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (p < n) y[p] = v;
}

int field_blocks(const Geom& g, const Shape& s) { return s.gx * s.gy * g.nx; }

}  // namespace

hipError_t launch_term(expint_dtype dt, expint_bc bc, const Geom& g, const Tiling& tl, const Coef& cf,
                       const TermOp& op, hipStream_t st) {
  if (op.ju) return launch_term_lin(dt, bc, g, tl, cf, op, st);
  SweepArgs a{};
  a.op = op;
  return sweep<kTerm>(dt, bc, g, tl, cf, a, st);
}

hipError_t launch_rhs(expint_dtype dt, expint_bc bc, const Geom& g, const Tiling& tl, const Coef& cf, const void* u,
                      void* b, double rho, hipStream_t st) {
  SweepArgs a{};
  a.x = u;
  a.out = b;
  a.rho = rho;
  return sweep<kRhs>(dt, bc, g, tl, cf, a, st);
}

hipError_t launch_apply(expint_dtype dt, expint_bc bc, const Geom& g, const Tiling& tl, const Coef& cf,
                        const void* x, void* y, hipStream_t st) {
  SweepArgs a{};
  a.x = x;
  a.out = y;
  return sweep<kApply>(dt, bc, g, tl, cf, a, st);
}

hipError_t launch_adj_rhs(expint_dtype dt, expint_bc bc, const Geom& g, const Tiling& tl, const Coef& cf,
                          const void* gv, const void* u, const void* lam_in, void* lam_out, double rho,
                          hipStream_t st) {
  SweepArgs a{};
  a.x = gv;
  a.out = lam_out;
  a.aux0 = lam_in;
  a.aux1 = u;
  a.rho = rho;
  return sweep<kAdjRhs>(dt, bc, g, tl, cf, a, st);
}

hipError_t launch_scan_labels(expint_bc bc, const Geom& g, const uint8_t* labels, int nclass, const double* tab64,
                              const double* wall64, double* partial, double* out, hipStream_t st) {
  const Shape s = choose_shape(g);
  const int nb = field_blocks(g, s);
  const dim3 grid(nb), block(s.bx, s.by);
  if (bc == EXPINT_NOFLUX)
    k_scan_labels<0><<<grid, block, 0, st>>>(g, s.gx, s.gy, labels, nclass, tab64, wall64, partial);
  else
    k_scan_labels<1><<<grid, block, 0, st>>>(g, s.gx, s.gy, labels, nclass, tab64, wall64, partial);
  k_final_max2<<<1, kBlock, 0, st>>>(partial, nb, out);
  return hipGetLastError();
}

hipError_t launch_scan_dense(expint_dtype dt, expint_bc bc, const Geom& g, const void* D, double inv_h2, void* fx,
                             void* fy, void* fz, void* wallv, double* partial, double* out, hipStream_t st) {
  const Shape s = choose_shape(g);
  const int nb = field_blocks(g, s);
  const dim3 grid(nb), block(s.bx, s.by);
  if (dt == EXPINT_F64) {
    auto* d = static_cast<const double*>(D);
    auto f = [](void* p) { return static_cast<double*>(p); };
    if (bc == EXPINT_NOFLUX)
      k_scan_dense<double, 0><<<grid, block, 0, st>>>(g, s.gx, s.gy, d, inv_h2, f(fx), f(fy), f(fz), f(wallv), partial);
    else
      k_scan_dense<double, 1><<<grid, block, 0, st>>>(g, s.gx, s.gy, d, inv_h2, f(fx), f(fy), f(fz), f(wallv), partial);
  } else {
    auto* d = static_cast<const float*>(D);
    auto f = [](void* p) { return static_cast<float*>(p); };
    if (bc == EXPINT_NOFLUX)
      k_scan_dense<float, 0><<<grid, block, 0, st>>>(g, s.gx, s.gy, d, inv_h2, f(fx), f(fy), f(fz), f(wallv), partial);
    else
      k_scan_dense<float, 1><<<grid, block, 0, st>>>(g, s.gx, s.gy, d, inv_h2, f(fx), f(fy), f(fz), f(wallv), partial);
  }
  k_final_max2<<<1, kBlock, 0, st>>>(partial, nb, out);
  return hipGetLastError();
}

template <typename T, int OP>
static void reduce_op(const T* x, const T* y, int64_t n, double* partial, double* out, int acc, hipStream_t st) {
  k_reduce<T, OP><<<kReduceBlocks, kBlock, 0, st>>>(x, y, n, partial);
  k_reduce_final<OP><<<1, kBlock, 0, st>>>(partial, kReduceBlocks, out, acc);
}

template <typename T>
static void reduce_typed(int op, const T* x, const T* y, int64_t n, double* partial, double* out, int acc,
                         hipStream_t st) {
  switch (op) {
    case 0: reduce_op<T, 0>(x, y, n, partial, out, acc, st); break;
    case 1: reduce_op<T, 1>(x, y, n, partial, out, acc, st); break;
    case 2: reduce_op<T, 2>(x, y, n, partial, out, acc, st); break;
    case 3: reduce_op<T, 3>(x, y, n, partial, out, acc, st); break;
    case 4: reduce_op<T, 4>(x, y, n, partial, out, acc, st); break;
    case 5: reduce_op<T, 5>(x, y, n, partial, out, acc, st); break;
    default: reduce_op<T, 6>(x, y, n, partial, out, acc, st); break;
  }
}

hipError_t launch_reduce(expint_dtype dt, int op, const void* x, const void* y, int64_t n, double* partial,
                         double* out, hipStream_t st, bool accumulate) {
  if (dt == EXPINT_F64)
    reduce_typed<double>(op, static_cast<const double*>(x), static_cast<const double*>(y), n, partial, out,
                         accumulate ? 1 : 0, st);
  else
    reduce_typed<float>(op, static_cast<const float*>(x), static_cast<const float*>(y), n, partial, out,
                        accumulate ? 1 : 0, st);
  return hipGetLastError();
}

hipError_t launch_axpy(expint_dtype dt, int64_t n, double a, const void* x, void* y, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>((n + kBlock - 1) / kBlock)), block(kBlock);
  if (dt == EXPINT_F64)
    k_axpy<double><<<grid, block, 0, st>>>(n, a, static_cast<const double*>(x), static_cast<double*>(y));
  else
    k_axpy<float><<<grid, block, 0, st>>>(n, static_cast<float>(a), static_cast<const float*>(x),
                                          static_cast<float*>(y));
  return hipGetLastError();
}

hipError_t launch_axpby(expint_dtype dt, int64_t n, double a, const void* x, double b, const void* y, void* out,
                        hipStream_t st) {
  const dim3 grid(static_cast<unsigned>((n + kBlock - 1) / kBlock)), block(kBlock);
  if (dt == EXPINT_F64)
    k_axpby<double><<<grid, block, 0, st>>>(n, a, static_cast<const double*>(x), b, static_cast<const double*>(y),
                                            static_cast<double*>(out));
  else
    k_axpby<float><<<grid, block, 0, st>>>(n, static_cast<float>(a), static_cast<const float*>(x),
                                           static_cast<float>(b), static_cast<const float*>(y),
                                           static_cast<float*>(out));
  return hipGetLastError();
}

hipError_t launch_copy(expint_dtype dt, int64_t n, const void* x, void* y, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>((n + kBlock - 1) / kBlock)), block(kBlock);
  if (dt == EXPINT_F64)
    k_copy<double><<<grid, block, 0, st>>>(n, static_cast<const double*>(x), static_cast<double*>(y));
  else
    k_copy<float><<<grid, block, 0, st>>>(n, static_cast<const float*>(x), static_cast<float*>(y));
  return hipGetLastError();
}

hipError_t launch_reaction_increment(expint_dtype dt, int64_t n, double rho, const void* u, const void* x, void* d,
                                     hipStream_t st) {
  const dim3 grid(static_cast<unsigned>((n + kBlock - 1) / kBlock)), block(kBlock);
  if (dt == EXPINT_F64)
    k_reaction_increment<double><<<grid, block, 0, st>>>(n, rho, static_cast<const double*>(u),
                                                         static_cast<const double*>(x), static_cast<double*>(d));
  else
    k_reaction_increment<float><<<grid, block, 0, st>>>(n, static_cast<float>(rho), static_cast<const float*>(u),
                                                        static_cast<const float*>(x), static_cast<float*>(d));
  return hipGetLastError();
}

hipError_t launch_diag_accumulate(expint_dtype dt, int64_t n, double w, const void* ybar, const void* y, void* d,
                                  hipStream_t st) {
  const dim3 grid(static_cast<unsigned>((n + kBlock - 1) / kBlock)), block(kBlock);
  if (dt == EXPINT_F64)
    k_diag_accumulate<double><<<grid, block, 0, st>>>(n, w, static_cast<const double*>(ybar),
                                                      static_cast<const double*>(y), static_cast<double*>(d));
  else
    k_diag_accumulate<float><<<grid, block, 0, st>>>(n, static_cast<float>(w), static_cast<const float*>(ybar),
                                                     static_cast<const float*>(y), static_cast<float*>(d));
  return hipGetLastError();
}

hipError_t launch_fill(expint_dtype dt, int64_t n, double v, void* y, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>((n + kBlock - 1) / kBlock)), block(kBlock);
  if (dt == EXPINT_F64)
    k_fill<double><<<grid, block, 0, st>>>(n, v, static_cast<double*>(y));
  else
    k_fill<float><<<grid, block, 0, st>>>(n, static_cast<float>(v), static_cast<float*>(y));
  return hipGetLastError();
}

}  // namespace expint
