// Mode products in the zero-flux basis by fast transforms (section 2.2's
// separable phi1 for uniform D).
//
// With zero flux the 1D eigenbasis is the orthonormal cosine basis
// Q[i][k] = c_k cos(pi k (i + 1/2) / n), so the forward mode product along an
// axis (Q^T) is the orthonormal DCT-II of every pencil along it and the
// inverse (Q) the orthonormal DCT-III.  A dense product costs 2n flops per
// element; these transforms cost O(log n), a few tens of flops per element,
// so a pass reads and writes the field once and needs no matrix cores.
//
// DCT-II through a complex DFT of the same length (Makhoul, "A fast cosine
// transform in one and multiple dimensions", IEEE TASSP 1980): reorder the
// pencil as v[m] = x[2m], v[n-1-m] = x[2m+1] (m < n/2), take V = DFT(v), and
// X[k] = c_k Re(e^{-i pi k/(2n)} V[k]).  The DCT-III runs it backwards:
// V[k] = e^{i pi k/(2n)} (X[k]/c_k - i X[n-k]/c_{n-k}) (the second term 0 at
// k = 0), v = the inverse DFT of V (1/n included), x[2m] = Re v[m],
// x[2m+1] = Re v[n-1-m].
//
// The DFT of length n = N1 N2 is taken in two passes (Cooley-Tukey): with
// b = b1 + N1 b2 and a = a1 + N2 a2,
//   out[a] = sum_{b1} w_{N1}^{b1 a2} w^{b1 a1} sum_{b2} in[b] w_{N2}^{b2 a1},
// w = e^{-2 pi i / n} (conjugate for the inverse).  Thread b1 of a pencil
// does the inner DFT over b2 in registers and multiplies by w^{b1 a1}; after
// an exchange through LDS, thread a1 does the outer DFT over b1.  The pass-1
// inputs are gathered from the real pencil in LDS (the reordering or the
// inverse's pre-twiddle applied on the way); pass 1 stores T[b1][a1] at slot
// b1 + (N1 + 1) a1 of a complex view of the same memory, so the lanes of one
// store are adjacent slots and the lanes of one pass-2 read are N1 + 1 slots
// apart: neither conflicts on LDS banks.
//
// Two real pencils share one complex DFT: the pencil a goes in as the real
// part and b as the imaginary part.  Forward, with Z = DFT(v_a + i v_b),
// V_a[k] = (Z[k] + conj Z[n-k]) / 2 and V_b[k] = (Z[k] - conj Z[n-k]) / (2i);
// Z[n-k] sits in lane (N2 - j) mod N2 of the same pencil team (register
// N1 - 1 - a2, or lane 0's own register (N1 - a2) mod N1) and is fetched by a
// lane shuffle.  Inverse, the DFT of the real v_a + i v_b is V_a + i V_b, so
// the inverse DFT of that sum gives v_a as its real part and v_b as its
// imaginary part.  This halves the DFT work of a pencil.
//
// A workgroup is NTH threads (dct_threads): TEAMS teams of TPP = max(N1, N2)
// threads, each team one complex DFT, so W = 2 TEAMS pencils.  FP64 runs 128
// threads, whose complex tiles take 35 KB of LDS (37 KB with the halo rows of
// the right-hand side pass) so that four workgroups share a CU; FP32 256
// (128 for the short axes, so that a tile holds at most 32 pencils: every
// grid dimension is a multiple of 32).  The field tile (W pencils of n
// values) is read from and written to global memory in the order that keeps
// accesses contiguous: W adjacent columns per row for side 0, whole pencils
// for side 1.  The fused x pass (kDctFwdMulInv)
// transforms forward, multiplies by the phi1 factor of each mode and
// transforms back, so the field crosses HBM once for all three.  The first
// pass of a step (kDctRhsFwd) reads the state u and forms the right-hand side
// A u + rho u (1 - u) on the way in (uniform D, zero flux), so the step needs
// no stencil sweep of its own.

#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "modal.hpp"

namespace expint {

namespace {

template <typename T>
struct CxT;
template <>
struct CxT<double> {
  using type = double2;
};
template <>
struct CxT<float> {
  using type = float2;
};

// The tile of workgroup L of nb.  The dispatcher deals workgroups to the 8
// XCDs round-robin, each with its own L2; adjacent side-0 tiles read the two
// halves of the same 128-byte lines, so XCD x takes the contiguous run of
// tiles [x nb/8, (x+1) nb/8) and every line is fetched into one L2 only.
__device__ __forceinline__ long dct_tile(long L, long nb) {
  if ((nb & 7) == 0) return (L & 7) * (nb >> 3) + (L >> 3);
  return L;
}

// Threads per workgroup of the transform kernels, and pencils per tile.
template <typename T, int TPP>
constexpr int dct_threads() {
  return sizeof(T) == 8 || TPP < 16 ? 128 : 256;
}
template <typename T, int TPP>
constexpr int dct_pencils() {
  return 2 * dct_threads<T, TPP>() / TPP;
}

template <typename C>
__device__ __forceinline__ C cmul(const C& a, const C& b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

template <int R>
constexpr int bitrev(int i) {
  int r = 0;
  for (int b = 1; b < R; b <<= 1) {
    r = (r << 1) | (i & 1);
    i >>= 1;
  }
  return r;
}

// cos and sin of 2 pi e / 16 for e < 4, correctly rounded to double
constexpr double kC16[4] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173};
constexpr double kS16[4] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};

// v * w^e with w = e^{-2 pi i / 16} (conjugated for the inverse), e < 8 a
// compile-time constant: e = 0 and e = 4 (a quarter turn) cost no multiply.
template <int E, bool INV, typename C>
__device__ __forceinline__ C twiddle16(const C& v) {
  using T = decltype(v.x);
  if constexpr (E == 0) {
    return v;
  } else if constexpr (E == 4) {
    return INV ? C{-v.y, v.x} : C{v.y, -v.x};  // times +i or -i
  } else {
    const T c = static_cast<T>(E < 4 ? kC16[E] : -kS16[E - 4]);
    const T s = static_cast<T>(E < 4 ? kS16[E] : kC16[E - 4]);
    // w^E = c - i s (forward), c + i s (inverse)
    return INV ? C{c * v.x - s * v.y, c * v.y + s * v.x} : C{c * v.x + s * v.y, c * v.y - s * v.x};
  }
}

// One butterfly stage of the R-point DIT DFT (blocks of LEN), unrolled at
// compile time.
template <int R, int LEN, int JJ, bool INV, typename C>
__device__ __forceinline__ void dit_stage(C (&y)[R]) {
  if constexpr (JJ < LEN / 2) {
#pragma unroll
    for (int s = 0; s < R; s += LEN) {
      const C u = y[s + JJ];
      const C v = twiddle16<JJ * (16 / LEN), INV>(y[s + JJ + LEN / 2]);
      y[s + JJ] = C{u.x + v.x, u.y + v.y};
      y[s + JJ + LEN / 2] = C{u.x - v.x, u.y - v.y};
    }
    dit_stage<R, LEN, JJ + 1, INV>(y);
  }
}
template <int R, int LEN, bool INV, typename C>
__device__ __forceinline__ void dit_stages(C (&y)[R]) {
  if constexpr (LEN <= R) {
    dit_stage<R, LEN, 0, INV>(y);
    dit_stages<R, LEN * 2, INV>(y);
  }
}

// In-place DFT of R <= 16 points in registers (radix 2, decimation in time,
// output in natural order), forward sign e^{-2 pi i / R} or its conjugate;
// the twiddles are the compile-time constants above.  No scaling.
template <int R, bool INV, typename C>
__device__ __forceinline__ void dft_reg(C (&x)[R]) {
  static_assert(R >= 2 && R <= 16 && (R & (R - 1)) == 0, "register DFTs of 2 to 16 points");
  C y[R];
#pragma unroll
  for (int i = 0; i < R; ++i) y[bitrev<R>(i)] = x[i];
  dit_stages<R, 2, INV>(y);
#pragma unroll
  for (int i = 0; i < R; ++i) x[i] = y[i];
}

// Two-pass DFT of the pencil w whose pass-1 inputs thread j (< N1) holds in
// x1 (index j + N1 b2 at x1[b2]).  On return thread j (< N2) holds output
// j + N2 a2 at y2[a2].  Ends with a barrier: the tile may be overwritten.
template <typename C, int N1, int N2, bool INV>
__device__ __forceinline__ void pencil_dft(C* lds, int w, int j, C (&x1)[N2], C (&y2)[N1],
                                           const double* __restrict__ tw) {
  constexpr int CS = (N1 + 1) * N2;
  C* const pc = lds + w * CS;
  if (j < N1) {
    dft_reg<N2, INV>(x1);
#pragma unroll
    for (int a1 = 0; a1 < N2; ++a1) {
      C v = x1[a1];
      if (a1 != 0 && j != 0) {
        const double2 te = reinterpret_cast<const double2*>(tw)[j * a1];  // j a1 < N1 N2
        const C t{static_cast<decltype(v.x)>(te.x), static_cast<decltype(v.x)>(INV ? -te.y : te.y)};
        v = cmul(t, v);
      }
      pc[j + (N1 + 1) * a1] = v;
    }
  }
  __syncthreads();
  if (j < N2) {
#pragma unroll
    for (int b1 = 0; b1 < N1; ++b1) y2[b1] = pc[b1 + (N1 + 1) * j];
    dft_reg<N1, INV>(y2);
  }
  __syncthreads();
}

// At least two waves per SIMD: the passes are latency-bound, and a register
// budget above 256 would halve the waves in flight (every pass fits now).
template <typename T, int N1, int N2, int SIDE, int MODE, int EPI>
__global__ __launch_bounds__((dct_threads<T, (N1 > N2 ? N1 : N2)>()), 2) void k_mode_dct(DctArgs a) {
  using C = typename CxT<T>::type;
  constexpr int N = N1 * N2;
  constexpr int TPP = N1 > N2 ? N1 : N2;       // threads per DFT
  constexpr int NTH = dct_threads<T, TPP>();   // threads per workgroup
  constexpr int TEAMS = NTH / TPP;             // DFTs per workgroup
  constexpr int W = dct_pencils<T, TPP>();     // pencils per workgroup, two per DFT
  constexpr int CS = (N1 + 1) * N2;            // complex slots per DFT
  constexpr int RS = N + 1;                    // real slots per pencil (the same memory)
  constexpr int PER = W * N / NTH;             // tile elements per thread
  // complex slots of the tile: the complex view, or the W + 2 halo rows of
  // the right-hand side pass if those take more
  constexpr int HALO_C = static_cast<int>(((W + 2) * RS * sizeof(T) + sizeof(C) - 1) / sizeof(C));
  constexpr int LDS_C = MODE == kDctRhsFwd && HALO_C > TEAMS * CS ? HALO_C : TEAMS * CS;
  static_assert(W * RS * sizeof(T) <= TEAMS * CS * sizeof(C), "the real view fits in the complex tiles");
  static_assert(N2 == TPP, "the pass-2 outputs of a DFT span its team");
  __shared__ C lds[LDS_C];
  __shared__ double rowt[MODE == kDctFwdMulInv ? 2 * N : 1];
  T* const lr = reinterpret_cast<T*>(lds);
  const int t = threadIdx.x, w = t / TPP, j = t % TPP;  // team, thread in the team

  const T* __restrict__ in = static_cast<const T*>(a.in);
  T* __restrict__ out = static_cast<T*>(a.out);
  const long tiles_per_p = SIDE == 0 ? a.post / W : 1;
  auto tile_base = [&](long tile, long& col0) {
    if (SIDE == 0) {
      const long p = tile / tiles_per_p;
      col0 = (tile - p * tiles_per_p) * W;
      return p * N * a.post + col0;
    }
    col0 = 0;
    return tile * W * N;
  };
  // Element r of this thread is tile element e = t + NTH r: pencil e % W and
  // index e / W on side 0 (W adjacent columns of one row are contiguous),
  // pencil e / N and index e % N on side 1.  NTH is a multiple of W, and N
  // and NTH divide one another, so each address is a per-thread part plus a
  // step in r that is uniform (global) or a compile-time constant (LDS): the
  // addresses cost no registers across the transforms.
  static_assert(NTH % W == 0 && (N % NTH == 0 || NTH % N == 0), "tile elements step evenly");
  auto lds_of = [&](int r) {  // real-view slot of element r
    if (SIDE == 0) return (t % W) * RS + t / W + r * (NTH / W);
    if (NTH <= N) return ((r * NTH) / N) * RS + t + (r * NTH) % N;
    return (t / N + r * (NTH / N)) * RS + t % N;
  };
  const long rstep = SIDE == 0 ? static_cast<long>(NTH / W) * a.post : NTH;  // elements from r to r + 1
  const unsigned lane_b =                                                    // this thread's bytes from the row
      static_cast<unsigned>(SIDE == 0 ? (t / W) * a.post + t % W : t) * static_cast<unsigned>(sizeof(T));

  if (MODE == kDctFwdMulInv) {
    // x-mode part of the multiplier: zr = tauD lam_x[k] and expm1(zr)
    for (int k = t; k < N; k += NTH) {
      const double zr = a.tauD * a.lam_x[k];
      rowt[k] = zr;
      rowt[N + k] = expm1(zr);
    }
  }
  // one tile per workgroup: all its loads in flight at once
  long col0 = 0;
  const long gbase = tile_base(dct_tile(blockIdx.x, gridDim.x), col0);
  auto gin = [&](int r) {
    return reinterpret_cast<const T*>(reinterpret_cast<const char*>(in + gbase + r * rstep) + lane_b);
  };
  auto gout = [&](int r) { return reinterpret_cast<T*>(reinterpret_cast<char*>(out + gbase + r * rstep) + lane_b); };
  if constexpr (MODE == kDctRhsFwd) {
    // The tile is W rows (x, y0 .. y0 + W - 1) of one x plane.  LDS rows
    // 0 .. W + 1 take u at y0 - 1 .. y0 + W; the x +- 1 rows come straight
    // into registers.  A neighbour across a wall is the voxel itself, so its
    // difference is exactly 0, as for a face left out.
    static_assert(SIDE == 1, "the right-hand side pass runs along z");
    static_assert((W + 2) * RS * sizeof(T) <= LDS_C * sizeof(C), "halo rows fit in the tile");
    constexpr int PH = ((W + 2) * N + NTH - 1) / NTH;
    const long r0 = gbase / N;
    const int x = static_cast<int>(r0 / a.ny), y0 = static_cast<int>(r0 - static_cast<long>(x) * a.ny);
    const long plane = static_cast<long>(a.ny) * N;
    const T* __restrict__ ux = in + static_cast<long>(x) * plane;
    {
      T h[PH];
#pragma unroll
      for (int r = 0; r < PH; ++r) {
        const int e = t + NTH * r;
        const int y = min(max(y0 - 1 + e / N, 0), a.ny - 1);
        h[r] = e < (W + 2) * N ? ux[static_cast<long>(y) * N + e % N] : T(0);
      }
#pragma unroll
      for (int r = 0; r < PH; ++r) {
        const int e = t + NTH * r;
        if (e < (W + 2) * N) lr[(e / N) * RS + e % N] = h[r];
      }
    }
    T xm[PER], xp[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const long o = gbase + t + NTH * r - static_cast<long>(x) * plane;  // offset in the plane
      xm[r] = ux[(x > 0 ? -plane : 0) + o];
      xp[r] = ux[(x < a.nx - 1 ? plane : 0) + o];
    }
    __syncthreads();
    T bv[PER];
    const T dh2 = static_cast<T>(a.dh2), rho = static_cast<T>(a.rho);
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = t + NTH * r, wr = e / N, z = e % N;
      const T* const row = lr + (wr + 1) * RS;
      const T c = row[z];
      const T lap = (xm[r] - c) + (xp[r] - c) + (lr[wr * RS + z] - c) + (lr[(wr + 2) * RS + z] - c) +
                    (row[z > 0 ? z - 1 : z] - c) + (row[z < N - 1 ? z + 1 : z] - c);
      bv[r] = dh2 * lap + rho * c * (T(1) - c);
    }
    __syncthreads();  // every halo read is done before the tile is overwritten
#pragma unroll
    for (int r = 0; r < PER; ++r) lr[lds_of(r)] = bv[r];
  } else {
    T v[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) v[r] = *gin(r);
#pragma unroll
    for (int r = 0; r < PER; ++r) lr[lds_of(r)] = v[r];
  }
  __syncthreads();
  {

    // the team's two pencils, real view
    T* const pa = lr + 2 * w * RS;
    T* const pb = pa + RS;
    C x1[N2], y2[N1];
    if (MODE != kDctInv) {
      // forward: pass-1 inputs from the reordered pencils
      if (j < N1) {
#pragma unroll
        for (int b2 = 0; b2 < N2; ++b2) {
          const int m = j + N1 * b2;
          const int i = m < N / 2 ? 2 * m : 2 * (N - 1 - m) + 1;
          x1[b2] = C{pa[i], pb[i]};
        }
      }
      __syncthreads();  // the real tile becomes the complex one
      pencil_dft<C, N1, N2, false>(lds, w, j, x1, y2, a.tw);
      {
        double zca = 0.0, emca = 0.0, zcb = 0.0, emcb = 0.0;
        if (MODE == kDctFwdMulInv) {
          const long qa = col0 + 2 * w, qb = qa + 1;  // columns (y mode, z mode) of the two x pencils
          zca = a.tauD * (a.lam_y[qa / a.nz] + a.lam_z[qa % a.nz]);
          zcb = a.tauD * (a.lam_y[qb / a.nz] + a.lam_z[qb % a.nz]);
          emca = expm1(zca);
          emcb = expm1(zcb);
        }
        const int jp = (TPP - j) & (TPP - 1);  // lane of Z[n - k] in the team
#pragma unroll
        for (int a2 = 0; a2 < N1; ++a2) {
          const int k = j + N2 * a2;
          const C zo = y2[(N1 - a2) & (N1 - 1)];
          const T sx = __shfl(y2[N1 - 1 - a2].x, jp, TPP);
          const T sy = __shfl(y2[N1 - 1 - a2].y, jp, TPP);
          const T nr = j == 0 ? zo.x : sx, ni = j == 0 ? zo.y : sy;
          const T zr = y2[a2].x, zi = y2[a2].y;
          const double2 cs = reinterpret_cast<const double2*>(a.mk)[k];
          const T c = static_cast<T>(cs.x), sn = static_cast<T>(cs.y);
          const T ck = static_cast<T>(0.5 * (k == 0 ? a.c0 : a.c1));
          T ya = ck * (c * (zr + nr) + sn * (zi - ni));
          T yb = ck * (c * (zi + ni) + sn * (nr - zr));
          if (MODE == kDctFwdMulInv) {
            const double zr0 = rowt[k], emr = rowt[N + k];
            const double za = zr0 + zca, zb = zr0 + zcb;
            ya = static_cast<T>(static_cast<double>(ya) *
                                (za == 0.0 ? a.tau : a.tau * (fma(emr, emca, emr + emca) / za)));
            yb = static_cast<T>(static_cast<double>(yb) *
                                (zb == 0.0 ? a.tau : a.tau * (fma(emr, emcb, emr + emcb) / zb)));
          }
          pa[k] = ya;
          pb[k] = yb;
        }
      }
      __syncthreads();
    }
    if (MODE == kDctInv || MODE == kDctFwdMulInv) {
      // inverse: pass-1 inputs V[k] = e^{i pi k/(2n)} (X[k]/c_k - i X[n-k]/c_{n-k})
      // of both pencils, packed as V_a + i V_b
      if (j < N1) {
        const T r0 = static_cast<T>(1.0 / a.c0), r1 = static_cast<T>(1.0 / a.c1);
#pragma unroll
        for (int b2 = 0; b2 < N2; ++b2) {
          const int k = j + N1 * b2;
          const double2 cs = reinterpret_cast<const double2*>(a.mk)[k];
          const T c = static_cast<T>(cs.x), sn = static_cast<T>(cs.y);
          const T yka = pa[k] * (k == 0 ? r0 : r1), ykb = pb[k] * (k == 0 ? r0 : r1);
          const T ynka = k == 0 ? T(0) : pa[N - k] * r1, ynkb = k == 0 ? T(0) : pb[N - k] * r1;
          const T ar = c * yka + sn * ynka, ai = sn * yka - c * ynka;
          const T br = c * ykb + sn * ynkb, bi = sn * ykb - c * ynkb;
          x1[b2] = C{ar - bi, ai + br};
        }
      }
      __syncthreads();
      pencil_dft<C, N1, N2, true>(lds, w, j, x1, y2, a.tw);
      if (j < N2) {
        const T inv_n = T(1) / T(N);
#pragma unroll
        for (int a2 = 0; a2 < N1; ++a2) {
          const int m = j + N2 * a2;
          const int i = m < N / 2 ? 2 * m : 2 * (N - 1 - m) + 1;
          pa[i] = y2[a2].x * inv_n;
          pb[i] = y2[a2].y * inv_n;
        }
      }
      __syncthreads();
    }

    if (EPI == kEpiAddU) {
      T old[PER];
#pragma unroll
      for (int r = 0; r < PER; ++r) old[r] = *gout(r);
#pragma unroll
      for (int r = 0; r < PER; ++r) *gout(r) = old[r] + lr[lds_of(r)];
    } else {
#pragma unroll
      for (int r = 0; r < PER; ++r) *gout(r) = lr[lds_of(r)];
    }
  }
}

template <typename T, int N1, int N2, int SIDE, int MODE, int EPI>
hipError_t launch_dct_k(const DctArgs& a, hipStream_t st) {
  constexpr int TPP = N1 > N2 ? N1 : N2, W = dct_pencils<T, TPP>();
  if (SIDE == 0 ? a.post % W != 0 : a.pre % W != 0) return hipErrorInvalidValue;
  // the right-hand side pass: a tile is W rows of one x plane
  if (MODE == kDctRhsFwd && (a.nx < 1 || a.ny < 1 || a.ny % W != 0 || static_cast<long>(a.nx) * a.ny != a.pre))
    return hipErrorInvalidValue;
  // a thread's offset within a tile row is 32-bit
  if (SIDE == 0 && static_cast<double>(dct_threads<T, TPP>() / W) * a.post * sizeof(T) >= 4294967296.0)
    return hipErrorInvalidValue;
  const long ntiles = SIDE == 0 ? a.pre * (a.post / W) : a.pre / W;
  k_mode_dct<T, N1, N2, SIDE, MODE, EPI>
      <<<dim3(static_cast<unsigned>(ntiles)), dct_threads<T, TPP>(), 0, st>>>(a);
  return hipGetLastError();
}

template <typename T, int N1, int N2>
hipError_t launch_dct_n(int side, int mode, int epi, const DctArgs& a, hipStream_t st) {
  if (side == 0) {
    if (mode == kDctFwd) return launch_dct_k<T, N1, N2, 0, kDctFwd, kEpiStore>(a, st);
    if (mode == kDctInv) return launch_dct_k<T, N1, N2, 0, kDctInv, kEpiStore>(a, st);
    return launch_dct_k<T, N1, N2, 0, kDctFwdMulInv, kEpiStore>(a, st);
  }
  if (mode == kDctFwd) return launch_dct_k<T, N1, N2, 1, kDctFwd, kEpiStore>(a, st);
  if (mode == kDctRhsFwd) return launch_dct_k<T, N1, N2, 1, kDctRhsFwd, kEpiStore>(a, st);
  if (epi == kEpiAddU) return launch_dct_k<T, N1, N2, 1, kDctInv, kEpiAddU>(a, st);
  return launch_dct_k<T, N1, N2, 1, kDctInv, kEpiStore>(a, st);
}

template <typename T>
hipError_t launch_dct_t(int side, int mode, int epi, const DctArgs& a, hipStream_t st) {
  switch (a.n) {
    case 32: return launch_dct_n<T, 4, 8>(side, mode, epi, a, st);
    case 64: return launch_dct_n<T, 8, 8>(side, mode, epi, a, st);
    case 128: return launch_dct_n<T, 8, 16>(side, mode, epi, a, st);
    case 256: return launch_dct_n<T, 16, 16>(side, mode, epi, a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool dct_axis_ok(int n) { return n == 32 || n == 64 || n == 128 || n == 256; }

namespace {
template <typename T, int TPP>
bool dct_rows_fit(long post) {
  return static_cast<double>(dct_threads<T, TPP>() / dct_pencils<T, TPP>()) * post * sizeof(T) < 4294967296.0;
}
}  // namespace

bool dct_rows_ok(int prec, int n, int side, long post) {
  if (side != 0) return true;
  const bool f64 = prec == kPrecF64, wide = n >= 128;
  return f64 ? (wide ? dct_rows_fit<double, 16>(post) : dct_rows_fit<double, 8>(post))
             : (wide ? dct_rows_fit<float, 16>(post) : dct_rows_fit<float, 8>(post));
}

void dct_tables(int n, std::vector<double>& tw, std::vector<double>& mk) {
  const double pi = 3.14159265358979323846;
  tw.assign(2 * static_cast<size_t>(n), 0.0);
  mk.assign(2 * static_cast<size_t>(n), 0.0);
  for (int e = 0; e < n; ++e) {
    const double th = 2.0 * pi * e / n;  // below 2 pi: the argument carries one rounding
    tw[2 * e] = std::cos(th);
    tw[2 * e + 1] = -std::sin(th);
  }
  for (int k = 0; k < n; ++k) {
    const double th = pi * k / (2.0 * n);
    mk[2 * k] = std::cos(th);
    mk[2 * k + 1] = std::sin(th);
  }
}

hipError_t launch_mode_dct(int prec, int side, int mode, int epi, const DctArgs& a, hipStream_t st) {
  if (!a.in || !a.out || !a.tw || !a.mk || a.pre < 1 || a.post < 1 || !dct_axis_ok(a.n)) return hipErrorInvalidValue;
  if (side == 1 && a.post != 1) return hipErrorInvalidValue;
  if (mode == kDctFwdMulInv && (side != 0 || a.pre != 1 || !a.lam_x || !a.lam_y || !a.lam_z))
    return hipErrorInvalidValue;
  if (epi == kEpiAddU && (side != 1 || mode != kDctInv)) return hipErrorInvalidValue;
  if (mode == kDctRhsFwd && side != 1) return hipErrorInvalidValue;
  if (epi != kEpiStore && epi != kEpiAddU) return hipErrorInvalidValue;
  DctArgs b = a;  // with the basis scale factors c_0 = sqrt(1/n), c_k = sqrt(2/n)
  b.c0 = std::sqrt(1.0 / a.n);
  b.c1 = std::sqrt(2.0 / a.n);
  if (prec == kPrecF64) return launch_dct_t<double>(side, mode, epi, b, st);
  if (prec == kPrecF32) return launch_dct_t<float>(side, mode, epi, b, st);
  return hipErrorInvalidValue;
}

}  // namespace expint
