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
// A workgroup of 4 waves computes a 64 x 64 output tile; the K dimension is
// staged through LDS in chunks of 32.  Arithmetic:
//   kPrecF64 / kPrecF32  plain vector FMA (4 x 4 outputs per thread);
//   kPrecBF16 / kPrecF16 matrix cores (v_mfma_f32_32x32x16, FP32 accumulate)
//                        on hi + lo split operands: x = hi + lo with hi = rnd(x),
//                        lo = rnd(x - hi); the product uses hi*hi + hi*lo + lo*hi.
//                        For FP16 the lo parts are scaled by 2^11 (kept out of
//                        the subnormal range) and the cross terms accumulate
//                        separately, rescaled at the end.
// Every dimension of the grid must be a multiple of 32 (checked on the host).

#include "modal.hpp"

#include <cstdlib>

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
  if (is_split<PREC>()) {
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const float xs = PREC == kPrecF16 ? 1.0f / kF16LoScale : 1.0f;
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
// The per-axis operator (n x n hi + lo, <= 256 KB at n = 256) is re-read from
// L2 by every wavefront.  MT output tiles of 32 are held at once (2, 4 or 8;
// fp16 needs a second accumulator for its scaled cross terms); larger n loops
// over blocks of MT tiles, re-reading the field block.
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

template <int PREC, int EPI, int MT>
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
  const long strips_per_p = (post + 31) / 32;
  const long strip = static_cast<long>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (strip >= strips_per_p * a.pre) return;  // whole wavefront
  const int p = static_cast<int>(strip / strips_per_p);
  const long q0 = (strip % strips_per_p) * 32;
  const long col = q0 + (lane & 31);
  const bool col_ok = col < post;
  const float* __restrict__ inp = in + static_cast<long>(p) * n * post;
  const int kh = (lane >> 5) * 8;
  for (int mb = 0; mb < n; mb += MT * 32) {
    f32x16 acc[MT], accx[two_acc ? MT : 1];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      acc[t] = f32x16{};
      if (two_acc) accx[two_acc ? t : 0] = f32x16{};
    }
    // the field fragment of the next K step is loaded before the current
    // step's matrix-core work (one step of register double buffering)
    float bnext[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) bnext[e] = col_ok ? inp[static_cast<long>(kh + e) * post + col] : 0.f;
    for (int k0 = 0; k0 < n; k0 += 16) {
      float bv[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) bv[e] = bnext[e];
      if (k0 + 16 < n) {
#pragma unroll
        for (int e = 0; e < 8; ++e) bnext[e] = col_ok ? inp[static_cast<long>(k0 + 16 + kh + e) * post + col] : 0.f;
      }
      V bh, bl;
      split8<PREC>(bv, bh, bl);
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        const int m = mb + t * 32 + (lane & 31);
        if (mb + t * 32 < n) {
          const long off = static_cast<long>(m) * n + k0 + kh;
          const V ah = *reinterpret_cast<const V*>(qhi + off);
          const V al = *reinterpret_cast<const V*>(qlo + off);
          acc[t] = Frag<PREC>::mma(ah, bh, acc[t]);
          if (two_acc) {
            accx[two_acc ? t : 0] = Frag<PREC>::mma(ah, bl, accx[two_acc ? t : 0]);
            accx[two_acc ? t : 0] = Frag<PREC>::mma(al, bh, accx[two_acc ? t : 0]);
          } else {
            acc[t] = Frag<PREC>::mma(ah, bl, acc[t]);
            acc[t] = Frag<PREC>::mma(al, bh, acc[t]);
          }
        }
      }
    }
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      if (mb + t * 32 >= n || !col_ok) continue;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = mb + t * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        float v = acc[t][r];
        if (two_acc) v += accx[two_acc ? t : 0][r] * (1.0f / kF16LoScale);
        if (EPI == kEpiMul) {
          const int jj = static_cast<int>(col / a.nz), kk = static_cast<int>(col % a.nz);
          const float z = static_cast<float>(a.tauD * (a.lam_x[m] + a.lam_y[jj] + a.lam_z[kk]));
          v *= phi1_times_tau(z, static_cast<float>(a.tau));
        }
        out[static_cast<long>(p) * n * post + static_cast<long>(m) * post + col] = v;
      }
    }
  }
}

template <int PREC, int EPI, int NT>
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
  const long strips = (pre + 31) / 32;
  if (strip >= strips) return;  // whole wavefront
  const long p0 = strip * 32;
  const long prow = p0 + (lane & 31);
  const bool row_ok = prow < pre;
  const float* __restrict__ inrow = in + (row_ok ? prow : p0) * n;
  const int kh = (lane >> 5) * 8;
  for (int nb = 0; nb < n; nb += NT * 32) {
    f32x16 acc[NT], accx[two_acc ? NT : 1];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      acc[t] = f32x16{};
      if (two_acc) accx[two_acc ? t : 0] = f32x16{};
    }
    float4 n0 = *reinterpret_cast<const float4*>(inrow + kh);
    float4 n1 = *reinterpret_cast<const float4*>(inrow + kh + 4);
    for (int k0 = 0; k0 < n; k0 += 16) {
      float av[8];
      const float4 v0 = n0, v1 = n1;
      if (k0 + 16 < n) {  // next K step's field fragment, ahead of the matrix-core work
        n0 = *reinterpret_cast<const float4*>(inrow + k0 + 16 + kh);
        n1 = *reinterpret_cast<const float4*>(inrow + k0 + 16 + kh + 4);
      }
      av[0] = v0.x; av[1] = v0.y; av[2] = v0.z; av[3] = v0.w;
      av[4] = v1.x; av[5] = v1.y; av[6] = v1.z; av[7] = v1.w;
      if (!row_ok)
#pragma unroll
        for (int e = 0; e < 8; ++e) av[e] = 0.f;
      V ah, al;
      split8<PREC>(av, ah, al);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (nb + t * 32 < n) {
          const long off = static_cast<long>(nb + t * 32 + (lane & 31)) * n + k0 + kh;
          const V bh = *reinterpret_cast<const V*>(qhi + off);
          const V bl = *reinterpret_cast<const V*>(qlo + off);
          acc[t] = Frag<PREC>::mma(ah, bh, acc[t]);
          if (two_acc) {
            accx[two_acc ? t : 0] = Frag<PREC>::mma(ah, bl, accx[two_acc ? t : 0]);
            accx[two_acc ? t : 0] = Frag<PREC>::mma(al, bh, accx[two_acc ? t : 0]);
          } else {
            acc[t] = Frag<PREC>::mma(ah, bl, acc[t]);
            acc[t] = Frag<PREC>::mma(al, bh, acc[t]);
          }
        }
      }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (nb + t * 32 >= n) continue;
      const int colk = nb + t * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const long row = p0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (row >= pre) continue;
        float v = acc[t][r];
        if (two_acc) v += accx[two_acc ? t : 0][r] * (1.0f / kF16LoScale);
        const long idx = row * n + colk;
        if (EPI == kEpiAddU) out[idx] = out[idx] + v;
        else out[idx] = v;
      }
    }
  }
}

// Output tiles held per wavefront: fewer tiles, fewer accumulator registers,
// more wavefronts in flight (the field block is then re-read from L2).
int modal_tiles() {
  static const int t = [] {
    const char* e = std::getenv("EXPINT_MODAL_TILES");
    const int v = e ? std::atoi(e) : 4;
    return (v == 2 || v == 4 || v == 8) ? v : 4;
  }();
  return t;
}

template <int PREC, int SIDE, int EPI, int T>
void launch_mode_mfma_t(const ModalArgs& a, hipStream_t st) {
  long strips;
  if (SIDE == 0) strips = static_cast<long>(a.pre) * ((a.post + 31) / 32);
  else strips = (static_cast<long>(a.pre) + 31) / 32;
  const dim3 grid(static_cast<unsigned>((strips + 3) / 4)), block(256);
  if (SIDE == 0) k_mode_left_mfma<PREC, EPI, T><<<grid, block, 0, st>>>(a);
  else k_mode_right_mfma<PREC, EPI, T><<<grid, block, 0, st>>>(a);
}

template <int PREC, int SIDE, int EPI>
void launch_mode_mfma(const ModalArgs& a, hipStream_t st) {
  const int t = modal_tiles();
  if (t == 2) launch_mode_mfma_t<PREC, SIDE, EPI, 2>(a, st);
  else if (t == 8 && PREC == kPrecBF16) launch_mode_mfma_t<PREC, SIDE, EPI, 8>(a, st);
  else launch_mode_mfma_t<PREC, SIDE, EPI, 4>(a, st);
}

template <int PREC, int SIDE, int EPI>
void launch_mode_t(const ModalArgs& a, hipStream_t st) {
  if constexpr (is_split<PREC>()) {
    launch_mode_mfma<PREC, SIDE, EPI>(a, st);
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
