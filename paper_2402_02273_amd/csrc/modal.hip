// Modal form of tau phi1(tau A) for a uniform diffusivity on a box.
//
// With constant D the operator of section 2.1 is a Kronecker sum of three
// 1D second-difference operators, each diagonalised by an orthonormal basis
// with closed-form eigenpairs (cosine modes for zero flux, sine modes for a
// zero ghost).  Then tau phi1(tau A) b = Q (tau phi1(tau D Lambda) .* Q^T b)
// with Q = Q_x (x) Q_y (x) Q_z, i.e. three dense per-axis mode products, a
// diagonal multiplier and three more mode products.  phi1(z) = (e^z - 1)/z
// (section 2.2).
//
// A mode product along one axis views the field as (pre, n, post) and maps
// out[p][i'][q] = sum_i Qop[i'][i] in[p][i][q].  Two GEMM shapes:
//   left  (x and y axes): C_p (n x post) = Qop (n x n) * B_p (n x post)
//   right (z axis, post = 1): C (pre x n) = B (pre x n) * Qop^T
// Every precision runs on the matrix cores in a pipelined LDS-staged GEMM
// (k_mode_gemm, k_mode_gemm_f32, k_mode_gemm_f64: all n modes per tile at
// n >= 256, so the field is read once).  Arithmetic:
//   kPrecF64             v_mfma_f64_16x16x4_f64, FP64 products and sums;
//   kPrecF32             v_mfma_f32_32x32x2_f32, FP32 products and sums;
//   kPrecBF16 / kPrecF16 v_mfma_f32_32x32x16 with FP32 accumulation on hi + lo
//                        split operands: x = hi + lo with hi = rnd(x),
//                        lo = rnd(x - hi); the product uses hi*hi + hi*lo + lo*hi.
//                        For FP16 the lo parts are scaled by 2^11 (kept out of
//                        the subnormal range) and the cross terms accumulate
//                        separately, rescaled at the end.
// The earlier kernels (k_mode: 64 x 64 tiles, 4 waves, K staged in chunks of
// 32; strip kernels for the split precisions) remain behind
// EXPINT_MODAL_KERNEL=strip.
// Every dimension of the grid must be a multiple of 32 (checked on the host).

#include "modal.hpp"

#include <cstdlib>
#include <initializer_list>
#include <type_traits>

namespace expint {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int TM = 64, TN = 64, KC = 32, KP = KC + 8;  // tile, K chunk, padded LDS row
constexpr float kF16LoScale = 2048.0f;                 // 2^11

template <int PREC>
struct Elem;
template <>
struct Elem<kPrecF64> { using T = double; using E = double; };
template <>
struct Elem<kPrecF32> { using T = float; using E = float; };
template <>
struct Elem<kPrecBF16> { using T = float; using E = __bf16; };
template <>
struct Elem<kPrecF16> { using T = float; using E = _Float16; };

template <int PREC>
constexpr bool is_split() { return PREC == kPrecBF16 || PREC == kPrecF16; }

template <int PREC>
struct Lds {
  using E = typename Elem<PREC>::E;
  alignas(16) E a_hi[TM][KP];  // A rows m, k contiguous
  alignas(16) E b_hi[TN][KP];  // B columns n, k contiguous
  alignas(16) E a_lo[is_split<PREC>() ? TM : 1][KP];
  alignas(16) E b_lo[is_split<PREC>() ? TN : 1][KP];
};

// Splits a float into hi + lo parts of the matrix-core element type.
template <int PREC>
__device__ __forceinline__ void split(float x, typename Elem<PREC>::E& hi, typename Elem<PREC>::E& lo) {
  using E = typename Elem<PREC>::E;
  hi = static_cast<E>(x);
  const float r = x - static_cast<float>(hi);
  lo = static_cast<E>(PREC == kPrecF16 ? r * kF16LoScale : r);
}

// Field tile stored with k contiguous: dst[row][k], row < rows, k < KC.
// Source element (row, k) at src[row * rs + k * ks], zero outside (nrow, nk).
// Consecutive threads walk the memory-contiguous index (coalesced loads).
template <int PREC, typename T>
__device__ __forceinline__ void stage_field(Lds<PREC>& s, bool to_a, const T* __restrict__ src, long rs, long ks,
                                            int rows, int nrow, int nk) {
  using E = typename Elem<PREC>::E;
  for (int idx = threadIdx.x; idx < rows * KC; idx += 256) {
    int row, k;
    if (ks == 1) {
      row = idx / KC;
      k = idx % KC;
    } else {
      row = idx % rows;
      k = idx / rows;
    }
    const T val = (row < nrow && k < nk) ? src[row * rs + k * ks] : T(0);
    if constexpr (is_split<PREC>()) {
      E hi, lo;
      split<PREC>(static_cast<float>(val), hi, lo);
      if (to_a) {
        s.a_hi[row][k] = hi;
        s.a_lo[row][k] = lo;
      } else {
        s.b_hi[row][k] = hi;
        s.b_lo[row][k] = lo;
      }
    } else {
      if (to_a) s.a_hi[row][k] = val;
      else s.b_hi[row][k] = val;
    }
  }
}

// Operator tile rows r (< rows) x k (< KC) from the precomputed matrix
// (n x n, k contiguous; for split precisions hi at q and lo at q + n*n).
template <int PREC>
__device__ __forceinline__ void stage_op(Lds<PREC>& s, bool to_a, const typename Elem<PREC>::E* __restrict__ q, int n,
                                         int r0, int k0) {
  using E = typename Elem<PREC>::E;
  const long nn = static_cast<long>(n) * n;
  for (int idx = threadIdx.x; idx < 64 * KC; idx += 256) {
    const int row = idx / KC, k = idx % KC;
    const bool ok = r0 + row < n && k0 + k < n;
    const long off = static_cast<long>(r0 + row) * n + k0 + k;
    const E hi = ok ? q[off] : E(0);
    if (to_a) s.a_hi[row][k] = hi;
    else s.b_hi[row][k] = hi;
    if constexpr (is_split<PREC>()) {
      const E lo = ok ? q[nn + off] : E(0);
      if (to_a) s.a_lo[row][k] = lo;
      else s.b_lo[row][k] = lo;
    }
  }
}

__device__ __forceinline__ double phi1_times_tau(double z, double tau) {
  return z == 0.0 ? tau : tau * expm1(z) / z;
}
__device__ __forceinline__ float phi1_times_tau(float z, float tau) {
  return z == 0.f ? tau : tau * expm1f(z) / z;
}

// tau phi1(z) for z = zr + zc <= 0 from er = exp(zr) and ec = exp(zc):
// e^z - 1 by one FP64 fma (its relative error stays near 1e-12 down to the
// smallest nonzero |z| of a grid), then the FP32 quotient.
__device__ __forceinline__ float phi1_sep(double zr, double er, double zc, double ec, float tau) {
  const float z = static_cast<float>(zr + zc);
  const float num = static_cast<float>(fma(er, ec, -1.0));
  return z == 0.f ? tau : tau * num * __builtin_amdgcn_rcpf(z);
}

// One 64 x 64 output tile of a mode product.
//   SIDE 0 (left):  out[p][m][q] = sum_k Qop[m][k] in[p][k][q]   (view pre, n, post)
//   SIDE 1 (right): out[p][m]    = sum_k in[p][k] Qop[m][k]     (view pre, n)
// EPI: store, multiply by tau phi1(tau D lambda) (left, x axis: pre == 1),
// or add into u (right).
template <int PREC, int SIDE, int EPI>
__global__ __launch_bounds__(256) void k_mode(ModalArgs a) {
  using T = typename Elem<PREC>::T;
  using E = typename Elem<PREC>::E;
  __shared__ Lds<PREC> s;
  const T* __restrict__ in = static_cast<const T*>(a.in);
  T* __restrict__ out = static_cast<T*>(a.out);
  const E* __restrict__ q = static_cast<const E*>(a.q);
  const int n = a.n, pre = a.pre;
  const long post = a.post;
  // tile coordinates: rows are output rows (left: modes i'; right: p), cols
  // are output columns (left: q; right: modes)
  const int tiles_n = SIDE == 0 ? static_cast<int>((post + TN - 1) / TN) : (n + TN - 1) / TN;
  const int tiles_m = SIDE == 0 ? (n + TM - 1) / TM : (pre + TM - 1) / TM;
  long bid = blockIdx.x;
  const int tn = static_cast<int>(bid % tiles_n);
  bid /= tiles_n;
  const int tm = static_cast<int>(bid % tiles_m);
  const int p = SIDE == 0 ? static_cast<int>(bid / tiles_m) : 0;
  const int m0 = tm * TM, n0 = tn * TN;
  const T* inp = in + (SIDE == 0 ? static_cast<long>(p) * n * post : 0);

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  f32x16 acc = {}, accx = {};
  T vacc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) vacc[i][j] = T(0);

  for (int k0 = 0; k0 < n; k0 += KC) {
    __syncthreads();
    if (SIDE == 0) {
      stage_op<PREC>(s, true, q, n, m0, k0);  // A = Qop rows m
      // B columns = q (post), rows = k: element (col, k) at inp[(k0 + k) * post + n0 + col]
      stage_field<PREC, T>(s, false, inp + static_cast<long>(k0) * post + n0, 1, post, TN,
                           static_cast<int>(post - n0 < TN ? post - n0 : TN), n - k0);
    } else {
      // A rows = p, k contiguous: element (row, k) at in[(m0 + row) * n + k0 + k]
      stage_field<PREC, T>(s, true, in + static_cast<long>(m0) * n + k0, n, 1, TM, pre - m0 < TM ? pre - m0 : TM,
                           n - k0);
      stage_op<PREC>(s, false, q, n, n0, k0);  // B columns = Qop rows
    }
    __syncthreads();
    if (is_split<PREC>()) {
      const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
#pragma unroll
      for (int ks = 0; ks < KC; ks += 16) {
        const int kk = ks + (lane >> 5) * 8;
        if constexpr (PREC == kPrecBF16) {
          const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&s.a_hi[wm + (lane & 31)][kk]);
          const bf16x8 al = *reinterpret_cast<const bf16x8*>(&s.a_lo[wm + (lane & 31)][kk]);
          const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&s.b_hi[wn + (lane & 31)][kk]);
          const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&s.b_lo[wn + (lane & 31)][kk]);
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
          accx = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, accx, 0, 0, 0);
          accx = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, accx, 0, 0, 0);
        } else if constexpr (PREC == kPrecF16) {
          const f16x8 ah = *reinterpret_cast<const f16x8*>(&s.a_hi[wm + (lane & 31)][kk]);
          const f16x8 al = *reinterpret_cast<const f16x8*>(&s.a_lo[wm + (lane & 31)][kk]);
          const f16x8 bh = *reinterpret_cast<const f16x8*>(&s.b_hi[wn + (lane & 31)][kk]);
          const f16x8 bl = *reinterpret_cast<const f16x8*>(&s.b_lo[wn + (lane & 31)][kk]);
          acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bh, acc, 0, 0, 0);
          accx = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bl, accx, 0, 0, 0);
          accx = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, bh, accx, 0, 0, 0);
        }
      }
    } else if constexpr (PREC == kPrecF32) {
      // FP32 on the matrix cores: v_mfma_f32_32x32x2_f32, lane l holding
      // A[l % 32][k + l / 32] and B[k + l / 32][l % 32]; FP32 products and sums
      const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
#pragma unroll
      for (int ks = 0; ks < KC; ks += 2) {
        const float av = s.a_hi[wm + (lane & 31)][ks + (lane >> 5)];
        const float bv = s.b_hi[wn + (lane & 31)][ks + (lane >> 5)];
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
      }
    } else {
      const int rm = (threadIdx.x >> 4) * 4, rn = (threadIdx.x & 15) * 4;
#pragma unroll 8
      for (int k = 0; k < KC; ++k) {
        T av[4], bv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          av[i] = static_cast<T>(s.a_hi[rm + i][k]);
          bv[i] = static_cast<T>(s.b_hi[rn + i][k]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) vacc[i][j] += av[i] * bv[j];
      }
    }
  }

  // epilogue: output element (row, col) of the tile
  auto emit = [&](int row, int col, T v) {
    const int gm = m0 + row, gn = n0 + col;
    if (SIDE == 0) {
      if (gm >= n || gn >= post) return;
      const long idx = static_cast<long>(p) * n * post + static_cast<long>(gm) * post + gn;
      if (EPI == kEpiMul) {
        // x axis (pre == 1): element (i, j, k) = (gm, gn / nz, gn % nz)
        const int jj = static_cast<int>(gn / a.nz), kk = static_cast<int>(gn % a.nz);
        const T z = static_cast<T>(a.tauD * (a.lam_x[gm] + a.lam_y[jj] + a.lam_z[kk]));
        v = v * phi1_times_tau(z, static_cast<T>(a.tau));
      }
      out[idx] = v;
    } else {
      if (gm >= pre || gn >= n) return;
      const long idx = static_cast<long>(gm) * n + gn;
      if (EPI == kEpiAddU) out[idx] = out[idx] + v;
      else out[idx] = v;
    }
  };
  if (is_split<PREC>() || PREC == kPrecF32) {
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const float xs = PREC == kPrecF16 ? 1.0f / kF16LoScale : (PREC == kPrecF32 ? 0.0f : 1.0f);  // F32: no accx
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      const int col = wn + (lane & 31);
      emit(row, col, static_cast<T>(acc[r] + accx[r] * xs));
    }
  } else {
    const int rm = (threadIdx.x >> 4) * 4, rn = (threadIdx.x & 15) * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) emit(rm + i, rn + j, vacc[i][j]);
  }
}

// ---------------------------------------------------------------------------
// Matrix-core strip kernels (split precisions).  One wavefront owns a whole
// output strip and streams its operands straight from memory into MFMA
// fragments; no LDS, no workgroup barriers.
//   left  (x, y axes): strip = all n output modes x 32 columns q of one p;
//                      the field column block B_p[:, q0 .. q0+32) is read once.
//   right (z axis):    strip = 32 rows p x all n output modes; the field rows
//                      are read once.
// The per-axis operator (n x n hi + lo, <= 256 KB at n = 256) is read from
// L2 by every wavefront; each of its fragments feeds NB (1 or 2) blocks of 32
// in the other GEMM dimension.  MT output tiles of 32 are held at once (2, 4
// or 8; fp16 needs a second accumulator for its scaled cross terms); larger n
// loops over blocks of MT tiles, re-reading the field block.
// Fragment layouts of v_mfma_f32_32x32x16_{bf16,f16} (checked on the device):
// A row = lane % 32, B column = lane % 32, k = 8 * (lane / 32) + element;
// D[row][col] with col = lane % 32, row = 8 (r / 4) + 4 (lane / 32) + r % 4.
// ---------------------------------------------------------------------------

template <int PREC>
struct Frag;
template <>
struct Frag<kPrecBF16> {
  using V = bf16x8;
  static __device__ __forceinline__ f32x16 mma(V a, V b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Frag<kPrecF16> {
  using V = f16x8;
  static __device__ __forceinline__ f32x16 mma(V a, V b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

template <int PREC>
__device__ __forceinline__ void split8(const float (&v)[8], typename Frag<PREC>::V& hi, typename Frag<PREC>::V& lo) {
  using E = typename Elem<PREC>::E;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    E h, l;
    split<PREC>(v[e], h, l);
    hi[e] = h;
    lo[e] = l;
  }
}

template <int PREC, int EPI, int MT, int NB>
__global__ __launch_bounds__(256) void k_mode_left_mfma(ModalArgs a) {
  using E = typename Elem<PREC>::E;
  using V = typename Frag<PREC>::V;
  constexpr bool two_acc = PREC == kPrecF16;
  const float* __restrict__ in = static_cast<const float*>(a.in);
  float* __restrict__ out = static_cast<float*>(a.out);
  const E* __restrict__ qhi = static_cast<const E*>(a.q);
  const int n = a.n;
  const long post = a.post;
  const long nn = static_cast<long>(n) * n;
  const E* __restrict__ qlo = qhi + nn;
  const int lane = threadIdx.x & 63;
  const long strips_per_p = (post + 32 * NB - 1) / (32 * NB);
  const long strip = static_cast<long>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (strip >= strips_per_p * a.pre) return;  // whole wavefront
  const int p = static_cast<int>(strip / strips_per_p);
  const long q0 = (strip % strips_per_p) * 32 * NB;
  long col[NB];
  bool col_ok[NB];
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    col[u] = q0 + 32 * u + (lane & 31);
    col_ok[u] = col[u] < post;
  }
  const float* __restrict__ inp = in + static_cast<long>(p) * n * post;
  const int kh = (lane >> 5) * 8;
  for (int mb = 0; mb < n; mb += MT * 32) {
    f32x16 acc[MT][NB], accx[two_acc ? MT : 1][two_acc ? NB : 1];
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        acc[t][u] = f32x16{};
        if (two_acc) accx[two_acc ? t : 0][two_acc ? u : 0] = f32x16{};
      }
    // the field fragments of the next K step are loaded before the current
    // step's matrix-core work (one step of register double buffering)
    float bnext[NB][8];
#pragma unroll
    for (int u = 0; u < NB; ++u)
#pragma unroll
      for (int e = 0; e < 8; ++e) bnext[u][e] = col_ok[u] ? inp[static_cast<long>(kh + e) * post + col[u]] : 0.f;
    for (int k0 = 0; k0 < n; k0 += 16) {
      V bh[NB], bl[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        float bv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) bv[e] = bnext[u][e];
        split8<PREC>(bv, bh[u], bl[u]);
      }
      if (k0 + 16 < n) {
#pragma unroll
        for (int u = 0; u < NB; ++u)
#pragma unroll
          for (int e = 0; e < 8; ++e)
            bnext[u][e] = col_ok[u] ? inp[static_cast<long>(k0 + 16 + kh + e) * post + col[u]] : 0.f;
      }
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        const int m = mb + t * 32 + (lane & 31);
        if (mb + t * 32 < n) {
          // one operator fragment feeds the NB column blocks
          const long off = static_cast<long>(m) * n + k0 + kh;
          const V ah = *reinterpret_cast<const V*>(qhi + off);
          const V al = *reinterpret_cast<const V*>(qlo + off);
#pragma unroll
          for (int u = 0; u < NB; ++u) {
            acc[t][u] = Frag<PREC>::mma(ah, bh[u], acc[t][u]);
            if (two_acc) {
              auto& x = accx[two_acc ? t : 0][two_acc ? u : 0];
              x = Frag<PREC>::mma(ah, bl[u], x);
              x = Frag<PREC>::mma(al, bh[u], x);
            } else {
              acc[t][u] = Frag<PREC>::mma(ah, bl[u], acc[t][u]);
              acc[t][u] = Frag<PREC>::mma(al, bh[u], acc[t][u]);
            }
          }
        }
      }
    }
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      if (mb + t * 32 >= n) continue;
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        if (!col_ok[u]) continue;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int m = mb + t * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          float v = acc[t][u][r];
          if (two_acc) v += accx[two_acc ? t : 0][two_acc ? u : 0][r] * (1.0f / kF16LoScale);
          if (EPI == kEpiMul) {
            const int jj = static_cast<int>(col[u] / a.nz), kk = static_cast<int>(col[u] % a.nz);
            const float z = static_cast<float>(a.tauD * (a.lam_x[m] + a.lam_y[jj] + a.lam_z[kk]));
            v *= phi1_times_tau(z, static_cast<float>(a.tau));
          }
          out[static_cast<long>(p) * n * post + static_cast<long>(m) * post + col[u]] = v;
        }
      }
    }
  }
}

template <int PREC, int EPI, int NT, int NB>
__global__ __launch_bounds__(256) void k_mode_right_mfma(ModalArgs a) {
  using E = typename Elem<PREC>::E;
  using V = typename Frag<PREC>::V;
  constexpr bool two_acc = PREC == kPrecF16;
  const float* __restrict__ in = static_cast<const float*>(a.in);
  float* __restrict__ out = static_cast<float*>(a.out);
  const E* __restrict__ qhi = static_cast<const E*>(a.q);
  const int n = a.n, pre = a.pre;
  const E* __restrict__ qlo = qhi + static_cast<long>(n) * n;
  const int lane = threadIdx.x & 63;
  const long strip = static_cast<long>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const long strips = (pre + 32 * NB - 1) / (32 * NB);
  if (strip >= strips) return;  // whole wavefront
  const long p0 = strip * 32 * NB;
  bool row_ok[NB];
  const float* __restrict__ inrow[NB];
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const long prow = p0 + 32 * u + (lane & 31);
    row_ok[u] = prow < pre;
    inrow[u] = in + (row_ok[u] ? prow : p0) * n;
  }
  const int kh = (lane >> 5) * 8;
  for (int nb = 0; nb < n; nb += NT * 32) {
    f32x16 acc[NT][NB], accx[two_acc ? NT : 1][two_acc ? NB : 1];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        acc[t][u] = f32x16{};
        if (two_acc) accx[two_acc ? t : 0][two_acc ? u : 0] = f32x16{};
      }
    float4 n0[NB], n1[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      n0[u] = *reinterpret_cast<const float4*>(inrow[u] + kh);
      n1[u] = *reinterpret_cast<const float4*>(inrow[u] + kh + 4);
    }
    for (int k0 = 0; k0 < n; k0 += 16) {
      V ah[NB], al[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        float av[8] = {n0[u].x, n0[u].y, n0[u].z, n0[u].w, n1[u].x, n1[u].y, n1[u].z, n1[u].w};
        if (!row_ok[u])
#pragma unroll
          for (int e = 0; e < 8; ++e) av[e] = 0.f;
        split8<PREC>(av, ah[u], al[u]);
      }
      if (k0 + 16 < n) {  // next K step's field fragments, ahead of the matrix-core work
#pragma unroll
        for (int u = 0; u < NB; ++u) {
          n0[u] = *reinterpret_cast<const float4*>(inrow[u] + k0 + 16 + kh);
          n1[u] = *reinterpret_cast<const float4*>(inrow[u] + k0 + 16 + kh + 4);
        }
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (nb + t * 32 < n) {
          // one operator fragment feeds the NB row blocks
          const long off = static_cast<long>(nb + t * 32 + (lane & 31)) * n + k0 + kh;
          const V bh = *reinterpret_cast<const V*>(qhi + off);
          const V bl = *reinterpret_cast<const V*>(qlo + off);
#pragma unroll
          for (int u = 0; u < NB; ++u) {
            acc[t][u] = Frag<PREC>::mma(ah[u], bh, acc[t][u]);
            if (two_acc) {
              auto& x = accx[two_acc ? t : 0][two_acc ? u : 0];
              x = Frag<PREC>::mma(ah[u], bl, x);
              x = Frag<PREC>::mma(al[u], bh, x);
            } else {
              acc[t][u] = Frag<PREC>::mma(ah[u], bl, acc[t][u]);
              acc[t][u] = Frag<PREC>::mma(al[u], bh, acc[t][u]);
            }
          }
        }
      }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (nb + t * 32 >= n) continue;
      const int colk = nb + t * 32 + (lane & 31);
#pragma unroll
      for (int u = 0; u < NB; ++u) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const long row = p0 + 32 * u + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          if (row >= pre) continue;
          float v = acc[t][u][r];
          if (two_acc) v += accx[two_acc ? t : 0][two_acc ? u : 0][r] * (1.0f / kF16LoScale);
          const long idx = row * n + colk;
          if (EPI == kEpiAddU) out[idx] = out[idx] + v;
          else out[idx] = v;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// LDS-staged matrix-core GEMM for the split precisions.  A workgroup of
// TMW x TNW waves computes a (64 TMW) x (64 TNW) output tile
// C[m][c] = sum_k A[m][k] B[k][c]; each wave owns a 64 x 64 block = 2 x 2
// MFMA tiles of 32.  K advances in chunks of 32 staged in LDS (two buffers;
// the global loads of the next two chunks are held in registers while the
// current chunk's matrix-core work runs).  Both LDS arrays keep k contiguous
// per row (A by m, B by c), so a fragment (8 consecutive k of one row or
// column) is one 16-byte LDS read; the 80-byte row pitch keeps those reads
// free of bank conflicts.
//   left  (SIDE 0): A = Qop (n x n, pre-split hi / lo), B[k][c] = in[p][k][q0 + c]
//                   (fp32, split while staging); C -> out[p][m][q]
//   right (SIDE 1): A[m][k] = in[p0 + m][k] (fp32, split while staging),
//                   B[k][c] = Qop[c][k]; C -> out[p0 + m][c]
// With n = 256 the launch spans all modes in one tile (left 256 x 128, right
// 128 x 256), so every field element is read from memory once.  Rows and
// columns beyond the problem are staged as zeros and not stored.
// ---------------------------------------------------------------------------
constexpr int GK = 32;       // K chunk
constexpr int GKP = GK + 8;  // padded LDS row (80 bytes for 16-bit elements)

template <int PREC, int TMW, int TNW>
struct GemmLds {
  using E = typename Elem<PREC>::E;
  alignas(16) E a_hi[2][64 * TMW][GKP];
  alignas(16) E a_lo[2][64 * TMW][GKP];
  alignas(16) E b_hi[2][64 * TNW][GKP];
  alignas(16) E b_lo[2][64 * TNW][GKP];
};

// NE consecutive 16-bit elements as NE / 8 16-byte vectors.
template <int NE>
struct EV {
  uint4 v[NE / 8];
};

// The 16 bytes of a buffer load as a uint4.
typedef int i32x4_buf __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 as_uint4(i32x4_buf v) {
  return make_uint4(static_cast<unsigned>(v.x), static_cast<unsigned>(v.y), static_cast<unsigned>(v.z),
                    static_cast<unsigned>(v.w));
}

template <int PREC, int NE>
__device__ __forceinline__ void split_n(const float (&v)[NE], EV<NE>& hi, EV<NE>& lo) {
  using E = typename Elem<PREC>::E;
  E h[NE], l[NE];
#pragma unroll
  for (int e = 0; e < NE; ++e) split<PREC>(v[e], h[e], l[e]);
  __builtin_memcpy(&hi, h, sizeof(h));
  __builtin_memcpy(&lo, l, sizeof(l));
}

// Output tile of one GEMM workgroup.  Left: (p, mode tile, column tile);
// right: (row tile, mode tile).  mrows / ncols bound the whole problem.
struct GemmTile {
  long m0, c0, mrows, ncols;
  int p;
};

template <int SIDE, int GM, int GN>
__device__ __forceinline__ GemmTile gemm_tile(const ModalArgs& a) {
  GemmTile t;
  t.p = 0;
  if (SIDE == 0) {
    const long ct = (a.post + GN - 1) / GN, mt = (a.n + GM - 1) / GM;
    long b = blockIdx.x;
    const long cti = b % ct;
    b /= ct;
    t.m0 = (b % mt) * GM;
    t.p = static_cast<int>(b / mt);
    t.c0 = cti * GN;
    t.mrows = a.n;
    t.ncols = a.post;
  } else {
    const long ct = (a.n + GN - 1) / GN;
    t.m0 = (blockIdx.x / ct) * GM;
    t.c0 = (blockIdx.x % ct) * GN;
    t.mrows = a.pre;
    t.ncols = a.n;
  }
  return t;
}

// Row table of the phi1 multiplier (left product, kEpiMul): exp(z) is
// separable, exp(z_row + z_col) = exp(z_row) exp(z_col), so each row's
// tauD lambda_x and its exponential are formed once per tile (FP64, LDS:
// rowv[0, GM) and rowv[GM, 2 GM)) and each column's once per lane; per element
// the multiplier is then tau (e_row e_col - 1) / z.  z <= 0, and z == 0 only
// for the constant mode, where e_row e_col - 1 is exactly 0 too.  The caller
// publishes the table with a barrier.
template <int GM>
__device__ __forceinline__ void phi1_rows(const ModalArgs& a, const GemmTile& tl, double* rowv) {
  const int tid = threadIdx.x;
  if (tid < GM) {
    const long row = tl.m0 + tid;
    const double zr = row < tl.mrows ? a.tauD * a.lam_x[row] : 0.0;
    rowv[tid] = zr;
    rowv[GM + tid] = exp(zr);
  }
}

// Stores a wave's 64 x 64 block, 2 x 2 accumulator tiles of 32 x 32 with
// D[row][col] at col = lane % 32, row = 8 (r / 4) + 4 (lane / 32) + r % 4:
// plain, times tau phi1 (kEpiMul, rows from rowv) or added into the output
// (kEpiAddU).
template <int SIDE, int EPI, int GM, int GN>
__device__ __forceinline__ void gemm_epilogue(const ModalArgs& a, const GemmTile& tl, const f32x16 (&acc)[2][2],
                                              const double* rowv, int wm, int wn, int lane) {
  float* __restrict__ out = static_cast<float*>(a.out);
  const int n = a.n;
  const long m0 = tl.m0, c0 = tl.c0, mrows = tl.mrows, ncols = tl.ncols;
  const int p = tl.p;
  const int fr = lane & 31;
  const long rs = SIDE == 0 ? a.post : n;  // row stride of the output
  float* const obase = out + (SIDE == 0 ? static_cast<long>(p) * n * a.post : 0);
  if (m0 + GM <= mrows && c0 + GN <= ncols && rs * GM < (1L << 31)) {
    // interior tile: no per-element bounds, a uniform base per 32 x 32 block
    // and a 32-bit offset per element
    const int irs = static_cast<int>(rs);
    const int lane_off = 4 * (lane >> 5) * irs + fr;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        float* const tb = obase + (m0 + wm + 32 * t) * rs + c0 + wn + 32 * u;
        double zc = 0.0, ec = 1.0;  // kEpiMul: tauD (lambda_y + lambda_z) of this lane's column, its exp
        if (SIDE == 0 && EPI == kEpiMul) {
          const long col = c0 + wn + 32 * u + fr;
          zc = a.tauD * (a.lam_y[col / a.nz] + a.lam_z[col % a.nz]);
          ec = exp(zc);
        }
        // add into u: all 16 loads of the block before its stores (a load
        // after a store to the same buffer would wait for the store's address)
        float old[16];
        if (SIDE == 1 && EPI == kEpiAddU) {
#pragma unroll
          for (int r = 0; r < 16; ++r) old[r] = tb[(8 * (r >> 2) + (r & 3)) * irs + lane_off];
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int off = (8 * (r >> 2) + (r & 3)) * irs + lane_off;
          float v = acc[t][u][r];
          if (SIDE == 0 && EPI == kEpiMul) {
            const int rl = wm + 32 * t + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            v *= phi1_sep(rowv[rl], rowv[GM + rl], zc, ec, static_cast<float>(a.tau));
          }
          if (SIDE == 1 && EPI == kEpiAddU) tb[off] = old[r] + v;
          else tb[off] = v;
        }
      }
    return;
  }
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const long col = c0 + wn + 32 * u + fr;
      if (col >= ncols) continue;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const long row = m0 + wm + 32 * t + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (row >= mrows) continue;
        float v = acc[t][u][r];
        if (SIDE == 0) {
          if (EPI == kEpiMul) {
            const int rl = static_cast<int>(row - m0);
            const double zc = a.tauD * (a.lam_y[col / a.nz] + a.lam_z[col % a.nz]);
            v *= phi1_sep(rowv[rl], rowv[GM + rl], zc, exp(zc), static_cast<float>(a.tau));
          }
          out[static_cast<long>(p) * n * a.post + row * a.post + col] = v;
        } else {
          const long idx = row * n + col;
          if (EPI == kEpiAddU) out[idx] = out[idx] + v;
          else out[idx] = v;
        }
      }
    }
}

template <int PREC, int SIDE, int EPI, int TMW, int TNW>
__global__ __launch_bounds__(64 * TMW * TNW) void k_mode_gemm(ModalArgs a) {
  using E = typename Elem<PREC>::E;
  using V = typename Frag<PREC>::V;
  constexpr bool two_acc = PREC == kPrecF16;
  constexpr int NT = 64 * TMW * TNW;  // threads
  constexpr int GM = 64 * TMW, GN = 64 * TNW;
  constexpr int EA = GM * GK / NT, EB = GN * GK / NT;  // staged elements per thread of A and B
  // the operator is A on the left, B on the right; the field the other one
  constexpr int EO = SIDE == 0 ? EA : EB, EF = SIDE == 0 ? EB : EA;
  static_assert(EO % 8 == 0 && EF % 4 == 0, "16-byte staging pieces");
  __shared__ GemmLds<PREC, TMW, TNW> s;
  const float* __restrict__ in = static_cast<const float*>(a.in);
  const E* __restrict__ qhi = static_cast<const E*>(a.q);
  const int n = a.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / TNW) * 64, wn = (wave % TNW) * 64;  // the wave's block
  const GemmTile tl = gemm_tile<SIDE, GM, GN>(a);
  const long m0 = tl.m0, c0 = tl.c0, mrows = tl.mrows, ncols = tl.ncols;
  const int p = tl.p;
  const float* __restrict__ inp = in + (SIDE == 0 ? static_cast<long>(p) * n * a.post : 0);

  // Staging pieces.  Operator rows (and right-side field rows): thread t ->
  // row t / (32 / E), k offset (t % (32 / E)) * E.  Left-side field (columns
  // q, k strided by post): thread t -> column t % GN, k offset (t / GN) * EF.
  const int orow_l = tid / (GK / EO), ok_ = (tid % (GK / EO)) * EO;
  const int frow_l = SIDE == 0 ? tid % GN : tid / (GK / EF);
  const int fk_ = SIDE == 0 ? (tid / GN) * EF : (tid % (GK / EF)) * EF;
  const long orow = (SIDE == 0 ? m0 : c0) + orow_l;
  const bool op_ok = orow < (SIDE == 0 ? mrows : ncols);
  const long fidx = (SIDE == 0 ? c0 : m0) + frow_l;  // field column (left) / row (right)
  const bool fld_ok = fidx < (SIDE == 0 ? ncols : mrows);

  // Loads go through buffer resources: a uniform base (the operator; this
  // product's field slab) with a loop-invariant 32-bit byte offset per lane
  // and the chunk's k offset in a scalar register, so a load costs no vector
  // address arithmetic.  The host keeps every offset below 2^31 bytes.  A lane
  // whose row or column lies outside the problem points past the resource's
  // size, and its loads return 0: the LDS tile is zero-padded without selects.
  constexpr uint32_t kPast = 0x80000000u;
  constexpr int kRsrcWord3 = 0x00020000;  // raw 32-bit buffer, gfx9 family
  const uint32_t fslab = static_cast<uint32_t>(SIDE == 0 ? static_cast<long>(n) * a.post : static_cast<long>(a.pre) * n);
  const __amdgpu_buffer_rsrc_t rq = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<E*>(qhi), 0, static_cast<int>(2u * static_cast<uint32_t>(n) * n * sizeof(E)), kRsrcWord3);
  const __amdgpu_buffer_rsrc_t rf =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(inp), 0, static_cast<int>(fslab * 4u), kRsrcWord3);
  const uint32_t vo_op = op_ok ? static_cast<uint32_t>((orow * n + ok_) * sizeof(E)) : kPast;
  const uint32_t vo_f = fld_ok ? static_cast<uint32_t>(SIDE == 0 ? (static_cast<long>(fk_) * a.post + fidx) * 4
                                                                  : (fidx * n + fk_) * 4)
                               : kPast;
  const uint32_t lo_bytes = static_cast<uint32_t>(n) * n * sizeof(E);  // qlo follows qhi

  // Two chunks in flight between global load and LDS write.  The operator
  // part is already split; the field part stays fp32 until the LDS write
  // (splitting at load time would wait for the load at once).  Loads are
  // unconditional, at clamped rows / columns, so the number in flight is known
  // to the compiler; out-of-range rows / columns are zeroed at the LDS write.
  struct Pending {
    EV<EO> op_hi, op_lo;
    float fld[EF];
  } pend0, pend1;  // named, not an array: a runtime index would put them in scratch
  auto load_chunk = [&](int k0, Pending& pd) __attribute__((always_inline)) {
    const int sk = k0 * static_cast<int>(sizeof(E));
#pragma unroll
    for (int i = 0; i < EO / 8; ++i) {
      pd.op_hi.v[i] = as_uint4(__builtin_amdgcn_raw_buffer_load_b128(rq, vo_op + 16 * i, sk, 0));
      pd.op_lo.v[i] = as_uint4(__builtin_amdgcn_raw_buffer_load_b128(rq, vo_op + 16 * i, sk + static_cast<int>(lo_bytes), 0));
    }
    if (SIDE == 0) {
#pragma unroll
      for (int e = 0; e < EF; ++e)
        pd.fld[e] = __builtin_bit_cast(
            float, __builtin_amdgcn_raw_buffer_load_b32(rf, vo_f, static_cast<int>((k0 + e) * a.post * 4), 0));
    } else {
#pragma unroll
      for (int i = 0; i < EF / 4; ++i) {
        const uint4 f = as_uint4(__builtin_amdgcn_raw_buffer_load_b128(rf, vo_f + 16 * i, k0 * 4, 0));
        pd.fld[4 * i] = __builtin_bit_cast(float, f.x);
        pd.fld[4 * i + 1] = __builtin_bit_cast(float, f.y);
        pd.fld[4 * i + 2] = __builtin_bit_cast(float, f.z);
        pd.fld[4 * i + 3] = __builtin_bit_cast(float, f.w);
      }
    }
  };
  auto store_chunk = [&](const Pending& pd, int buf) __attribute__((always_inline)) {
    EV<EF> f_hi, f_lo;
    split_n<PREC, EF>(pd.fld, f_hi, f_lo);
    E(*ohi)[GKP] = SIDE == 0 ? s.a_hi[buf] : s.b_hi[buf];
    E(*olo)[GKP] = SIDE == 0 ? s.a_lo[buf] : s.b_lo[buf];
#pragma unroll
    for (int i = 0; i < EO / 8; ++i) {
      *reinterpret_cast<uint4*>(&ohi[orow_l][ok_ + 8 * i]) = pd.op_hi.v[i];
      *reinterpret_cast<uint4*>(&olo[orow_l][ok_ + 8 * i]) = pd.op_lo.v[i];
    }
    E(*fhi)[GKP] = SIDE == 0 ? s.b_hi[buf] : s.a_hi[buf];
    E(*flo)[GKP] = SIDE == 0 ? s.b_lo[buf] : s.a_lo[buf];
#pragma unroll
    for (int i = 0; i < EF / 8; ++i) {
      *reinterpret_cast<uint4*>(&fhi[frow_l][fk_ + 8 * i]) = f_hi.v[i];
      *reinterpret_cast<uint4*>(&flo[frow_l][fk_ + 8 * i]) = f_lo.v[i];
    }
  };

  f32x16 acc[2][2], accx[two_acc ? 2 : 1][two_acc ? 2 : 1];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      acc[t][u] = f32x16{};
      if (two_acc) accx[two_acc ? t : 0][two_acc ? u : 0] = f32x16{};
    }
  const int fr = lane & 31, fk = (lane >> 5) * 8;  // fragment row / column and k offset
  const int nchunks = n / GK;
  // one chunk: loads of chunk c + 2 into the register set that held chunk c
  // (already in LDS), the matrix-core work on chunk c, chunk c + 1 from the
  // other set into the other LDS buffer, barrier
  auto iteration = [&](int c, auto which) __attribute__((always_inline)) {
    Pending& ld = decltype(which)::value == 0 ? pend0 : pend1;
    const Pending& nx = decltype(which)::value == 0 ? pend1 : pend0;
    const int buf = c & 1;
    load_chunk(min(c + 2, nchunks - 1) * GK, ld);  // past the end: a harmless reload
#pragma unroll
    for (int ks = 0; ks < GK; ks += 16) {
      V ah[2], al[2], bh[2], bl[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        ah[t] = *reinterpret_cast<const V*>(&s.a_hi[buf][wm + 32 * t + fr][ks + fk]);
        al[t] = *reinterpret_cast<const V*>(&s.a_lo[buf][wm + 32 * t + fr][ks + fk]);
        bh[t] = *reinterpret_cast<const V*>(&s.b_hi[buf][wn + 32 * t + fr][ks + fk]);
        bl[t] = *reinterpret_cast<const V*>(&s.b_lo[buf][wn + 32 * t + fr][ks + fk]);
      }
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          acc[t][u] = Frag<PREC>::mma(ah[t], bh[u], acc[t][u]);
          if (two_acc) {
            auto& x = accx[two_acc ? t : 0][two_acc ? u : 0];
            x = Frag<PREC>::mma(ah[t], bl[u], x);
            x = Frag<PREC>::mma(al[t], bh[u], x);
          } else {
            acc[t][u] = Frag<PREC>::mma(ah[t], bl[u], acc[t][u]);
            acc[t][u] = Frag<PREC>::mma(al[t], bh[u], acc[t][u]);
          }
        }
    }
    if (c + 1 < nchunks) store_chunk(nx, buf ^ 1);
    __syncthreads();
  };
  load_chunk(0, pend0);
  load_chunk(min(1, nchunks - 1) * GK, pend1);
  __shared__ double rowv[SIDE == 0 && EPI == kEpiMul ? 2 * GM : 1];
  if (SIDE == 0 && EPI == kEpiMul) phi1_rows<GM>(a, tl, rowv);
  store_chunk(pend0, 0);
  __syncthreads();  // also publishes rowv
  for (int c = 0; c < nchunks; c += 2) {
    iteration(c, std::integral_constant<int, 0>{});
    if (c + 1 < nchunks) iteration(c + 1, std::integral_constant<int, 1>{});
  }
  if (two_acc) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int r = 0; r < 16; ++r)
          acc[t][u][r] += accx[two_acc ? t : 0][two_acc ? u : 0][r] * (1.0f / kF16LoScale);
  }
  gemm_epilogue<SIDE, EPI, GM, GN>(a, tl, acc, rowv, wm, wn, lane);
}

template <int PREC, int SIDE, int EPI, int TMW, int TNW>
void launch_mode_gemm_t(const ModalArgs& a, hipStream_t st) {
  constexpr int GM = 64 * TMW, GN = 64 * TNW;
  long blocks;
  if (SIDE == 0) blocks = static_cast<long>(a.pre) * ((a.n + GM - 1) / GM) * ((a.post + GN - 1) / GN);
  else blocks = ((static_cast<long>(a.pre) + GM - 1) / GM) * ((a.n + GN - 1) / GN);
  k_mode_gemm<PREC, SIDE, EPI, TMW, TNW><<<dim3(static_cast<unsigned>(blocks)), dim3(64 * TMW * TNW), 0, st>>>(a);
}

// Tile shape: all 256 modes in one tile when n >= 256 (the field is then read
// once), else 128 x 128.
template <int PREC, int SIDE, int EPI>
void launch_mode_gemm(const ModalArgs& a, hipStream_t st) {
  const char* e = std::getenv("EXPINT_MODAL_GEMM_TILE");
  const bool big = e ? e[0] == 'b' : a.n >= 256;
  if (!big) launch_mode_gemm_t<PREC, SIDE, EPI, 2, 2>(a, st);
  else if (SIDE == 0) launch_mode_gemm_t<PREC, SIDE, EPI, 4, 2>(a, st);
  else launch_mode_gemm_t<PREC, SIDE, EPI, 2, 4>(a, st);
}

// ---------------------------------------------------------------------------
// FP32 mode products on the FP32 matrix cores, in the same LDS-staged GEMM
// structure: buffer loads of two K chunks held in registers, double-buffered
// LDS tiles with k contiguous per row (A by m, B by c), 64 x 64 per wave as
// 2 x 2 tiles of v_mfma_f32_32x32x2_f32, the shared epilogue.
// A fragment of that instruction is one element per lane: A[row = l % 32]
// [slot l / 32], B[slot l / 32][col = l % 32].  Which k sits in a slot is
// free as long as A and B agree, so each lane reads four consecutive k with
// one 16-byte LDS read (k = kb + 4 (l / 32) + j for the j-th of four
// instructions): one read per operand and tile feeds four instructions.  The
// 144-byte row pitch keeps those reads free of bank conflicts.  Products and
// sums are FP32 throughout.
// ---------------------------------------------------------------------------
constexpr int GKP32 = GK + 4;  // padded LDS row of floats

template <int TMW, int TNW>
struct GemmLds32 {
  alignas(16) float a[2][64 * TMW][GKP32];
  alignas(16) float b[2][64 * TNW][GKP32];
};

template <int SIDE, int EPI, int TMW, int TNW>
__global__ __launch_bounds__(64 * TMW * TNW) void k_mode_gemm_f32(ModalArgs a) {
  constexpr int NT = 64 * TMW * TNW;  // threads
  constexpr int GM = 64 * TMW, GN = 64 * TNW;
  constexpr int EA = GM * GK / NT, EB = GN * GK / NT;  // staged elements per thread of A and B
  constexpr int EO = SIDE == 0 ? EA : EB, EF = SIDE == 0 ? EB : EA;
  static_assert(EO % 4 == 0 && EF % 4 == 0, "16-byte staging pieces");
  __shared__ GemmLds32<TMW, TNW> s;
  const int n = a.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / TNW) * 64, wn = (wave % TNW) * 64;  // the wave's block
  const GemmTile tl = gemm_tile<SIDE, GM, GN>(a);
  const float* __restrict__ inp = static_cast<const float*>(a.in) + (SIDE == 0 ? static_cast<long>(tl.p) * n * a.post : 0);

  // Staging pieces, as in the split kernel: operator rows (and right-side
  // field rows) thread t -> row t / (32 / E), k offset (t % (32 / E)) * E;
  // left-side field thread t -> column t % GN, k offset (t / GN) * EF.
  const int orow_l = tid / (GK / EO), ok_ = (tid % (GK / EO)) * EO;
  const int frow_l = SIDE == 0 ? tid % GN : tid / (GK / EF);
  const int fk_ = SIDE == 0 ? (tid / GN) * EF : (tid % (GK / EF)) * EF;
  const long orow = (SIDE == 0 ? tl.m0 : tl.c0) + orow_l;
  const bool op_ok = orow < (SIDE == 0 ? tl.mrows : tl.ncols);
  const long fidx = (SIDE == 0 ? tl.c0 : tl.m0) + frow_l;
  const bool fld_ok = fidx < (SIDE == 0 ? tl.ncols : tl.mrows);

  // buffer resources; lanes outside the problem point past the end and read 0
  constexpr uint32_t kPast = 0x80000000u;
  constexpr int kRsrcWord3 = 0x00020000;  // raw 32-bit buffer, gfx9 family
  const uint32_t fslab = static_cast<uint32_t>(SIDE == 0 ? static_cast<long>(n) * a.post : static_cast<long>(a.pre) * n);
  const __amdgpu_buffer_rsrc_t rq = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<void*>(a.q), 0, static_cast<int>(static_cast<uint32_t>(n) * n * 4u), kRsrcWord3);
  const __amdgpu_buffer_rsrc_t rf =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(inp), 0, static_cast<int>(fslab * 4u), kRsrcWord3);
  const uint32_t vo_op = op_ok ? static_cast<uint32_t>((orow * n + ok_) * 4) : kPast;
  const uint32_t vo_f = fld_ok ? static_cast<uint32_t>(SIDE == 0 ? (static_cast<long>(fk_) * a.post + fidx) * 4
                                                                  : (fidx * n + fk_) * 4)
                               : kPast;

  struct Pending {
    uint4 op[EO / 4];
    float fld[EF];
  } pend0, pend1;  // named, not an array: a runtime index would put them in scratch
  auto load_chunk = [&](int k0, Pending& pd) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < EO / 4; ++i) pd.op[i] = as_uint4(__builtin_amdgcn_raw_buffer_load_b128(rq, vo_op + 16 * i, k0 * 4, 0));
    if (SIDE == 0) {
#pragma unroll
      for (int e = 0; e < EF; ++e)
        pd.fld[e] = __builtin_bit_cast(
            float, __builtin_amdgcn_raw_buffer_load_b32(rf, vo_f, static_cast<int>((k0 + e) * a.post * 4), 0));
    } else {
#pragma unroll
      for (int i = 0; i < EF / 4; ++i) {
        const uint4 f = as_uint4(__builtin_amdgcn_raw_buffer_load_b128(rf, vo_f + 16 * i, k0 * 4, 0));
        pd.fld[4 * i] = __builtin_bit_cast(float, f.x);
        pd.fld[4 * i + 1] = __builtin_bit_cast(float, f.y);
        pd.fld[4 * i + 2] = __builtin_bit_cast(float, f.z);
        pd.fld[4 * i + 3] = __builtin_bit_cast(float, f.w);
      }
    }
  };
  auto store_chunk = [&](const Pending& pd, int buf) __attribute__((always_inline)) {
    float(*o)[GKP32] = SIDE == 0 ? s.a[buf] : s.b[buf];
#pragma unroll
    for (int i = 0; i < EO / 4; ++i) *reinterpret_cast<uint4*>(&o[orow_l][ok_ + 4 * i]) = pd.op[i];
    float(*f)[GKP32] = SIDE == 0 ? s.b[buf] : s.a[buf];
#pragma unroll
    for (int i = 0; i < EF / 4; ++i)
      *reinterpret_cast<float4*>(&f[frow_l][fk_ + 4 * i]) =
          make_float4(pd.fld[4 * i], pd.fld[4 * i + 1], pd.fld[4 * i + 2], pd.fld[4 * i + 3]);
  };

  f32x16 acc[2][2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) acc[t][u] = f32x16{};
  const int fr = lane & 31, fk = (lane >> 5) * 4;  // fragment row / column and k offset
  const int nchunks = n / GK;
  auto iteration = [&](int c, auto which) __attribute__((always_inline)) {
    Pending& ld = decltype(which)::value == 0 ? pend0 : pend1;
    const Pending& nx = decltype(which)::value == 0 ? pend1 : pend0;
    const int buf = c & 1;
    load_chunk(min(c + 2, nchunks - 1) * GK, ld);  // past the end: a harmless reload
#pragma unroll
    for (int kb = 0; kb < GK; kb += 8) {
      float4 av[2], bv[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        av[t] = *reinterpret_cast<const float4*>(&s.a[buf][wm + 32 * t + fr][kb + fk]);
        bv[t] = *reinterpret_cast<const float4*>(&s.b[buf][wn + 32 * t + fr][kb + fk]);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int u = 0; u < 2; ++u)
            acc[t][u] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[t][j], bv[u][j], acc[t][u], 0, 0, 0);
    }
    if (c + 1 < nchunks) store_chunk(nx, buf ^ 1);
    __syncthreads();
  };
  load_chunk(0, pend0);
  load_chunk(min(1, nchunks - 1) * GK, pend1);
  __shared__ double rowv[SIDE == 0 && EPI == kEpiMul ? 2 * GM : 1];
  if (SIDE == 0 && EPI == kEpiMul) phi1_rows<GM>(a, tl, rowv);
  store_chunk(pend0, 0);
  __syncthreads();  // also publishes rowv
  for (int c = 0; c < nchunks; c += 2) {
    iteration(c, std::integral_constant<int, 0>{});
    if (c + 1 < nchunks) iteration(c + 1, std::integral_constant<int, 1>{});
  }
  gemm_epilogue<SIDE, EPI, GM, GN>(a, tl, acc, rowv, wm, wn, lane);
}

template <int SIDE, int EPI, int TMW, int TNW>
void launch_mode_gemm_f32_t(const ModalArgs& a, hipStream_t st) {
  constexpr int GM = 64 * TMW, GN = 64 * TNW;
  long blocks;
  if (SIDE == 0) blocks = static_cast<long>(a.pre) * ((a.n + GM - 1) / GM) * ((a.post + GN - 1) / GN);
  else blocks = ((static_cast<long>(a.pre) + GM - 1) / GM) * ((a.n + GN - 1) / GN);
  k_mode_gemm_f32<SIDE, EPI, TMW, TNW><<<dim3(static_cast<unsigned>(blocks)), dim3(64 * TMW * TNW), 0, st>>>(a);
}

// Tile shape as for the split products: all 256 modes in one tile when
// n >= 256, else 128 x 128.
template <int SIDE, int EPI>
void launch_mode_gemm_f32(const ModalArgs& a, hipStream_t st) {
  const char* e = std::getenv("EXPINT_MODAL_GEMM_TILE");
  const bool big = e ? e[0] == 'b' : a.n >= 256;
  if (!big) launch_mode_gemm_f32_t<SIDE, EPI, 2, 2>(a, st);
  else if (SIDE == 0) launch_mode_gemm_f32_t<SIDE, EPI, 4, 2>(a, st);
  else launch_mode_gemm_f32_t<SIDE, EPI, 2, 4>(a, st);
}

// ---------------------------------------------------------------------------
// FP64 mode products on the FP64 matrix cores (v_mfma_f64_16x16x4_f64), in
// the same LDS-staged structure with K chunks of 16.  A wave's 64 x 64 block
// is 4 x 4 tiles of 16 x 16.  Fragment layout (checked on the device): lane l
// holds A[l % 16][slot l / 16] and B[slot l / 16][l % 16]; output element r of
// lane l is D[l / 16 + 4 r][l % 16].  As in the FP32 kernel each lane reads
// four consecutive k (two 16-byte LDS reads) and feeds them to four
// instructions (k = kb + 4 (l / 16) + j for the j-th), so A and B agree on
// every slot.  Products and sums are FP64; the phi1 multiplier uses
// e^(zr + zc) - 1 = em_r em_c + em_r + em_c with em = expm1 of the row and
// column parts (FP64, a few ulps: both are <= 0, so the sum never cancels
// below half of em_r + em_c).
// ---------------------------------------------------------------------------
constexpr int GK64 = 16;          // K chunk
constexpr int GKP64 = GK64 + 2;   // padded LDS row of doubles (144 bytes)
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <int TMW, int TNW>
struct GemmLds64 {
  alignas(16) double a[2][64 * TMW][GKP64];
  alignas(16) double b[2][64 * TNW][GKP64];
};

template <int SIDE, int EPI, int GM, int GN>
__device__ __forceinline__ void gemm_epilogue_f64(const ModalArgs& a, const GemmTile& tl, const f64x4 (&acc)[4][4],
                                                  const double* rowv, int wm, int wn, int lane) {
  double* __restrict__ out = static_cast<double*>(a.out);
  const int n = a.n;
  const long m0 = tl.m0, c0 = tl.c0, mrows = tl.mrows, ncols = tl.ncols;
  const long rs = SIDE == 0 ? a.post : n;  // row stride of the output
  double* const obase = out + (SIDE == 0 ? static_cast<long>(tl.p) * n * a.post : 0);
  const int fc = lane & 15, fr = lane >> 4;
  const double tau = a.tau;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const long col = c0 + wn + 16 * u + fc;
    if (col >= ncols) continue;
    double zc = 0.0, emc = 0.0;  // kEpiMul: tauD (lambda_y + lambda_z) of this column, its expm1
    if (SIDE == 0 && EPI == kEpiMul) {
      zc = a.tauD * (a.lam_y[col / a.nz] + a.lam_z[col % a.nz]);
      emc = expm1(zc);
    }
    // add into u: the column's 16 loads before its stores (a load after a
    // store to the same buffer would wait for the store)
    double old[4][4];
    if (SIDE == 1 && EPI == kEpiAddU) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const long row = m0 + wm + 16 * t + fr + 4 * r;
          old[t][r] = row < mrows ? obase[row * rs + col] : 0.0;
        }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rl = wm + 16 * t + fr + 4 * r;  // row in the tile
        const long row = m0 + rl;
        if (row >= mrows) continue;
        double v = acc[t][u][r];
        if (SIDE == 0 && EPI == kEpiMul) {
          const double z = rowv[rl] + zc, emr = rowv[GM + rl];
          v *= z == 0.0 ? tau : tau * (fma(emr, emc, emr + emc) / z);
        }
        double* const o = obase + row * rs + col;
        if (SIDE == 1 && EPI == kEpiAddU) *o = old[t][r] + v;
        else *o = v;
      }
  }
}

template <int SIDE, int EPI, int TMW, int TNW>
__global__ __launch_bounds__(64 * TMW * TNW) void k_mode_gemm_f64(ModalArgs a) {
  constexpr int NT = 64 * TMW * TNW;  // threads
  constexpr int GM = 64 * TMW, GN = 64 * TNW;
  constexpr int EA = GM * GK64 / NT, EB = GN * GK64 / NT;  // staged elements per thread of A and B
  constexpr int EO = SIDE == 0 ? EA : EB, EF = SIDE == 0 ? EB : EA;
  static_assert(EO % 2 == 0 && EF % 2 == 0, "16-byte staging pieces");
  __shared__ GemmLds64<TMW, TNW> s;
  const int n = a.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / TNW) * 64, wn = (wave % TNW) * 64;  // the wave's block
  const GemmTile tl = gemm_tile<SIDE, GM, GN>(a);
  const double* __restrict__ inp =
      static_cast<const double*>(a.in) + (SIDE == 0 ? static_cast<long>(tl.p) * n * a.post : 0);

  // staging pieces as in the other kernels (E = 2 doubles per 16 bytes)
  const int orow_l = tid / (GK64 / EO), ok_ = (tid % (GK64 / EO)) * EO;
  const int frow_l = SIDE == 0 ? tid % GN : tid / (GK64 / EF);
  const int fk_ = SIDE == 0 ? (tid / GN) * EF : (tid % (GK64 / EF)) * EF;
  const long orow = (SIDE == 0 ? tl.m0 : tl.c0) + orow_l;
  const bool op_ok = orow < (SIDE == 0 ? tl.mrows : tl.ncols);
  const long fidx = (SIDE == 0 ? tl.c0 : tl.m0) + frow_l;
  const bool fld_ok = fidx < (SIDE == 0 ? tl.ncols : tl.mrows);

  // buffer resources; lanes outside the problem point past the end and read 0
  constexpr uint32_t kPast = 0x80000000u;
  constexpr int kRsrcWord3 = 0x00020000;  // raw 32-bit buffer, gfx9 family
  const uint32_t fslab = static_cast<uint32_t>(SIDE == 0 ? static_cast<long>(n) * a.post : static_cast<long>(a.pre) * n);
  const __amdgpu_buffer_rsrc_t rq = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<void*>(a.q), 0, static_cast<int>(static_cast<uint32_t>(n) * n * 8u), kRsrcWord3);
  const __amdgpu_buffer_rsrc_t rf =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(inp), 0, static_cast<int>(fslab * 8u), kRsrcWord3);
  const uint32_t vo_op = op_ok ? static_cast<uint32_t>((orow * n + ok_) * 8) : kPast;
  const uint32_t vo_f = fld_ok ? static_cast<uint32_t>(SIDE == 0 ? (static_cast<long>(fk_) * a.post + fidx) * 8
                                                                  : (fidx * n + fk_) * 8)
                               : kPast;

  struct Pending {
    uint4 op[EO / 2];
    uint2 fld[EF];
  } pend0, pend1;  // named, not an array: a runtime index would put them in scratch
  auto load_chunk = [&](int k0, Pending& pd) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < EO / 2; ++i) pd.op[i] = as_uint4(__builtin_amdgcn_raw_buffer_load_b128(rq, vo_op + 16 * i, k0 * 8, 0));
    if (SIDE == 0) {
#pragma unroll
      for (int e = 0; e < EF; ++e) {
        const auto w = __builtin_amdgcn_raw_buffer_load_b64(rf, vo_f, static_cast<int>((k0 + e) * a.post * 8), 0);
        pd.fld[e] = make_uint2(static_cast<unsigned>(w[0]), static_cast<unsigned>(w[1]));
      }
    } else {
#pragma unroll
      for (int i = 0; i < EF / 2; ++i) {
        const uint4 f = as_uint4(__builtin_amdgcn_raw_buffer_load_b128(rf, vo_f + 16 * i, k0 * 8, 0));
        pd.fld[2 * i] = make_uint2(f.x, f.y);
        pd.fld[2 * i + 1] = make_uint2(f.z, f.w);
      }
    }
  };
  auto store_chunk = [&](const Pending& pd, int buf) __attribute__((always_inline)) {
    double(*o)[GKP64] = SIDE == 0 ? s.a[buf] : s.b[buf];
#pragma unroll
    for (int i = 0; i < EO / 2; ++i) *reinterpret_cast<uint4*>(&o[orow_l][ok_ + 2 * i]) = pd.op[i];
    double(*f)[GKP64] = SIDE == 0 ? s.b[buf] : s.a[buf];
#pragma unroll
    for (int i = 0; i < EF / 2; ++i)
      *reinterpret_cast<uint4*>(&f[frow_l][fk_ + 2 * i]) =
          make_uint4(pd.fld[2 * i].x, pd.fld[2 * i].y, pd.fld[2 * i + 1].x, pd.fld[2 * i + 1].y);
  };

  f64x4 acc[4][4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[t][u] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int fr = lane & 15, fk = (lane >> 4) * 4;  // fragment row / column and k offset
  const int nchunks = n / GK64;
  auto iteration = [&](int c, auto which) __attribute__((always_inline)) {
    Pending& ld = decltype(which)::value == 0 ? pend0 : pend1;
    const Pending& nx = decltype(which)::value == 0 ? pend1 : pend0;
    const int buf = c & 1;
    load_chunk(min(c + 2, nchunks - 1) * GK64, ld);  // past the end: a harmless reload
    f64x4 bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double* pb = &s.b[buf][wn + 16 * u + fr][fk];
      const double2 b01 = *reinterpret_cast<const double2*>(pb);
      const double2 b23 = *reinterpret_cast<const double2*>(pb + 2);
      bv[u] = f64x4{b01.x, b01.y, b23.x, b23.y};
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double* pa = &s.a[buf][wm + 16 * t + fr][fk];
      const double2 a01 = *reinterpret_cast<const double2*>(pa);
      const double2 a23 = *reinterpret_cast<const double2*>(pa + 2);
      const f64x4 av = {a01.x, a01.y, a23.x, a23.y};
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[j], bv[u][j], acc[t][u], 0, 0, 0);
    }
    if (c + 1 < nchunks) store_chunk(nx, buf ^ 1);
    __syncthreads();
  };
  load_chunk(0, pend0);
  load_chunk(min(1, nchunks - 1) * GK64, pend1);
  // row table of the multiplier: z_row and expm1(z_row), FP64
  __shared__ double rowv[SIDE == 0 && EPI == kEpiMul ? 2 * GM : 1];
  if (SIDE == 0 && EPI == kEpiMul && tid < GM) {
    const long row = tl.m0 + tid;
    const double zr = row < tl.mrows ? a.tauD * a.lam_x[row] : 0.0;
    rowv[tid] = zr;
    rowv[GM + tid] = expm1(zr);
  }
  store_chunk(pend0, 0);
  __syncthreads();  // also publishes rowv
  for (int c = 0; c < nchunks; c += 2) {
    iteration(c, std::integral_constant<int, 0>{});
    if (c + 1 < nchunks) iteration(c + 1, std::integral_constant<int, 1>{});
  }
  gemm_epilogue_f64<SIDE, EPI, GM, GN>(a, tl, acc, rowv, wm, wn, lane);
}

template <int SIDE, int EPI, int TMW, int TNW>
void launch_mode_gemm_f64_t(const ModalArgs& a, hipStream_t st) {
  constexpr int GM = 64 * TMW, GN = 64 * TNW;
  long blocks;
  if (SIDE == 0) blocks = static_cast<long>(a.pre) * ((a.n + GM - 1) / GM) * ((a.post + GN - 1) / GN);
  else blocks = ((static_cast<long>(a.pre) + GM - 1) / GM) * ((a.n + GN - 1) / GN);
  k_mode_gemm_f64<SIDE, EPI, TMW, TNW><<<dim3(static_cast<unsigned>(blocks)), dim3(64 * TMW * TNW), 0, st>>>(a);
}

template <int SIDE, int EPI>
void launch_mode_gemm_f64(const ModalArgs& a, hipStream_t st) {
  const char* e = std::getenv("EXPINT_MODAL_GEMM_TILE");
  const bool big = e ? e[0] == 'b' : a.n >= 256;
  if (!big) launch_mode_gemm_f64_t<SIDE, EPI, 2, 2>(a, st);
  else if (SIDE == 0) launch_mode_gemm_f64_t<SIDE, EPI, 4, 2>(a, st);
  else launch_mode_gemm_f64_t<SIDE, EPI, 2, 4>(a, st);
}

// Which kernels run the mode products: the LDS-staged GEMMs (default) or the
// earlier ones (EXPINT_MODAL_KERNEL=strip: strip kernels for the split
// precisions, k_mode for FP32 and FP64).
bool modal_use_gemm() {
  const char* e = std::getenv("EXPINT_MODAL_KERNEL");
  return !(e && e[0] == 's');
}

// Output tiles held per wavefront (MT): fewer tiles, fewer accumulator
// registers, more wavefronts in flight (the field block is then re-read from
// L2).  Blocks of 32 held in the other GEMM dimension (NB, columns for the
// left product, rows for the right): each operator fragment then feeds NB
// blocks, which divides the operator's L2 traffic by NB.  Measured defaults
// at 256^3: bf16 split MT 4, NB 1; fp16 split (two accumulators) MT 2, NB 2.
// EXPINT_MODAL_TILES / EXPINT_MODAL_NB override them.
int modal_env(const char* name, int fallback, std::initializer_list<int> allowed) {
  const char* e = std::getenv(name);
  if (!e) return fallback;
  const int v = std::atoi(e);
  for (int a : allowed)
    if (v == a) return v;
  return fallback;
}

template <int PREC>
int modal_tiles() {
  return modal_env("EXPINT_MODAL_TILES", PREC == kPrecF16 ? 2 : 4, {2, 4, 8});
}

template <int PREC>
int modal_blocks() {
  return modal_env("EXPINT_MODAL_NB", PREC == kPrecF16 ? 2 : 1, {1, 2});
}

template <int PREC, int SIDE, int EPI, int T, int NB>
void launch_mode_mfma_t(const ModalArgs& a, hipStream_t st) {
  long strips;
  if (SIDE == 0) strips = static_cast<long>(a.pre) * ((a.post + 32 * NB - 1) / (32 * NB));
  else strips = (static_cast<long>(a.pre) + 32 * NB - 1) / (32 * NB);
  const dim3 grid(static_cast<unsigned>((strips + 3) / 4)), block(256);
  if (SIDE == 0) k_mode_left_mfma<PREC, EPI, T, NB><<<grid, block, 0, st>>>(a);
  else k_mode_right_mfma<PREC, EPI, T, NB><<<grid, block, 0, st>>>(a);
}

template <int PREC, int SIDE, int EPI, int NB>
void launch_mode_mfma_nb(const ModalArgs& a, hipStream_t st) {
  const int t = modal_tiles<PREC>();
  if (t == 2) launch_mode_mfma_t<PREC, SIDE, EPI, 2, NB>(a, st);
  else if (t == 8 && PREC == kPrecBF16 && NB == 1) launch_mode_mfma_t<PREC, SIDE, EPI, 8, 1>(a, st);
  else launch_mode_mfma_t<PREC, SIDE, EPI, 4, NB>(a, st);
}

// Whether the GEMM's 32-bit buffer offsets reach every byte of the operator
// (split precisions: hi and lo) and of one field slab (left: n x post,
// right: pre x n elements of elem bytes).
bool gemm_offsets_fit(const ModalArgs& a, long elem = 4) {
  const long slab = a.post == 1 ? static_cast<long>(a.pre) * a.n : static_cast<long>(a.n) * a.post;
  return slab * elem < (1L << 31) && elem * a.n * a.n < (1L << 31);
}

template <int PREC, int SIDE, int EPI>
void launch_mode_mfma(const ModalArgs& a, hipStream_t st) {
  if (modal_use_gemm() && gemm_offsets_fit(a)) {
    launch_mode_gemm<PREC, SIDE, EPI>(a, st);
    return;
  }
  if (modal_blocks<PREC>() == 2) launch_mode_mfma_nb<PREC, SIDE, EPI, 2>(a, st);
  else launch_mode_mfma_nb<PREC, SIDE, EPI, 1>(a, st);
}

template <int PREC, int SIDE, int EPI>
void launch_mode_t(const ModalArgs& a, hipStream_t st) {
  if constexpr (is_split<PREC>()) {
    launch_mode_mfma<PREC, SIDE, EPI>(a, st);
    return;
  }
  if (PREC == kPrecF32 && modal_use_gemm() && gemm_offsets_fit(a)) {
    launch_mode_gemm_f32<SIDE, EPI>(a, st);
    return;
  }
  if (PREC == kPrecF64 && modal_use_gemm() && gemm_offsets_fit(a, 8)) {
    launch_mode_gemm_f64<SIDE, EPI>(a, st);
    return;
  }
  long tiles;
  if (SIDE == 0) tiles = static_cast<long>(a.pre) * ((a.n + TM - 1) / TM) * ((a.post + TN - 1) / TN);
  else tiles = static_cast<long>((a.pre + TM - 1) / TM) * ((a.n + TN - 1) / TN);
  k_mode<PREC, SIDE, EPI><<<dim3(static_cast<unsigned>(tiles)), dim3(256), 0, st>>>(a);
}

}  // namespace

hipError_t launch_mode_product(int prec, int side, int epi, const ModalArgs& a, hipStream_t st) {
  if (!a.in || !a.out || !a.q || a.pre < 1 || a.n < 1 || a.post < 1) return hipErrorInvalidValue;
  if (side == 1 && a.post != 1) return hipErrorInvalidValue;
  if (epi == kEpiMul && (side != 0 || !a.lam_x || !a.lam_y || !a.lam_z)) return hipErrorInvalidValue;
#define EXPINT_MODE_CASE(P)                                                         \
  case P:                                                                           \
    if (side == 0) {                                                                \
      if (epi == kEpiMul) launch_mode_t<P, 0, kEpiMul>(a, st);                      \
      else launch_mode_t<P, 0, kEpiStore>(a, st);                                   \
    } else {                                                                        \
      if (epi == kEpiAddU) launch_mode_t<P, 1, kEpiAddU>(a, st);                    \
      else launch_mode_t<P, 1, kEpiStore>(a, st);                                   \
    }                                                                               \
    break;
  switch (prec) {
    EXPINT_MODE_CASE(kPrecF64)
    EXPINT_MODE_CASE(kPrecF32)
    EXPINT_MODE_CASE(kPrecBF16)
    EXPINT_MODE_CASE(kPrecF16)
    default: return hipErrorInvalidValue;
  }
#undef EXPINT_MODE_CASE
  return hipGetLastError();
}

// Labels present in the grid: bit c of *mask set if some voxel has class c.
__global__ void k_label_mask(const uint8_t* __restrict__ lab, int64_t n, unsigned* mask) {
  unsigned local = 0;
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; p < n;
       p += static_cast<int64_t>(gridDim.x) * blockDim.x)
    local |= 1u << (lab[p] & 31);
  // wave-level OR, then one vector atomic per wave
  for (int o = 32; o > 0; o >>= 1) local |= __shfl_xor(local, o, 64);
  if ((threadIdx.x & 63) == 0 && local) atomicOr(mask, local);
}

hipError_t launch_label_mask(const uint8_t* labels, int64_t n, unsigned* mask, hipStream_t st) {
  k_label_mask<<<dim3(kReduceBlocks), dim3(kBlock), 0, st>>>(labels, n, mask);
  return hipGetLastError();
}

}  // namespace expint
