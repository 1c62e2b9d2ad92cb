// Pair sweeps: two consecutive Taylor terms of the augmented series
// (section 2.2) in one pass over the grid (label form).
//
// Term j + 1 applies A to term j, so a tile of term j + 1 needs term j on the
// tile and a one-voxel halo around it.  A workgroup owns 64 (z) x TY (y)
// output columns of LP consecutive x-planes and marches along x:
//   stage 1  computes term j on plane p over the tile plus its y/z halo
//            ((TY + 2) x 66 voxels, from src read around it) into a ring of
//            four planes in LDS, together with the voxels' labels;
//   stage 2  computes term j + 1 on plane p - 1 of the tile from the three
//            ring planes p - 2 .. p, adds both terms into the running sum and
//            writes the outputs.
// One barrier per plane separates the stages; with four ring slots stage 1 of
// plane p + 1 never overwrites a slot that a wave may still read for plane
// p - 1.  Term j never reaches memory: against two single-term sweeps this
// saves one field write and one field read per voxel and one launch.
//
// Stage 1 works in "tasks" of one wavefront: task r < TY + 2 is staged row r
// (lanes along z), task TY + 2 holds the z-halo columns of all staged rows
// (lane 2r: column z0 - 1, lane 2r + 1: column z0 + 64).  Task t runs on wave
// t % 4; the wave that stages row r also writes output row r - 1, so stage 2
// of every wave reads rows it or its neighbours staged.
//
// Wall handling follows the single-term sweeps: a neighbour outside the box
// is the voxel itself (zero wall flux); zero-Dirichlet walls subtract
// D_p / h^2 times the value per wall face.  Staged voxels outside the box are
// never computed nor read.

#include "internal.hpp"
#include "sweep_device.hpp"

namespace expint {

namespace {

constexpr int kPairZ = 64;          // output columns along z = wavefront width
constexpr int kRow = kPairZ + 2;    // staged columns z0 - 1 .. z0 + 64
constexpr int kRing = 4;            // planes of term j held in LDS

// Load of a T at a byte offset from a base: plane bases are uniform (scalar
// registers) and the per-lane offsets 32-bit, so a load needs no per-lane
// 64-bit address arithmetic.
template <typename T>
__device__ __forceinline__ T ld_at(const T* base, uint32_t byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}

template <typename T, int BC, int TY, int LP>
__global__ __launch_bounds__(kBlock) void k_pair(Geom g, int gz, int gy, Coef cf, TermOp op) {
  constexpr int kRows = TY + 2;
  constexpr int kTasks = kRows + 1;
  constexpr int kSlots = (kTasks + 3) / 4;
  constexpr uint32_t W = sizeof(T);
  static_assert(kBlock == 256, "four wavefronts per workgroup");
  static_assert(2 * kRows <= 64, "z-halo columns of all staged rows fit one wavefront");
  __shared__ LdsCoef<T> s;
  __shared__ T zs[kRing][kRows][kRow];
  __shared__ uint8_t ls[kRing][kRows][kRow];
  load_tables(s, cf, static_cast<int>(threadIdx.x), kBlock);

  const int L = xcd_remap(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
  const int zt = L % gz;
  const int t = L / gz;
  const int yt = t % gy;
  const int x0 = (t / gy) * LP;
  const int z0 = zt * kPairZ, y0 = yt * TY;
  const int wave = static_cast<int>(threadIdx.x) >> 6, lane = static_cast<int>(threadIdx.x) & 63;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int64_t sx = static_cast<int64_t>(ny) * nz;
  const T* x = static_cast<const T*>(op.src);
  const T* bs = static_cast<const T*>(op.bsrc);
  const uint8_t* lab = cf.labels;
  const T c1 = static_cast<T>(op.c), cb = static_cast<T>(op.cb), c2 = static_cast<T>(op.c2);

  // Stage-1 tasks of this wave.  Per task: staged row / column, in-plane
  // element offsets of the voxel and its four lateral neighbours (clamped to
  // the voxel at walls; the same on every plane), the x-marching state (term-j
  // source on the planes before and at the one being computed) and the loads
  // of the next plane, fetched one plane ahead so that they are in flight
  // across the barrier and stage 2.
  int tr[kSlots], tc[kSlots], wyz[kSlots];
  uint32_t o0[kSlots], o2[kSlots], o3[kSlots], o4[kSlots], o5[kSlots];
  bool tv[kSlots];
  T xm[kSlots], xc[kSlots];
  int lm[kSlots], lc[kSlots];
  T fn[kSlots], f2[kSlots], f3[kSlots], f4[kSlots], f5[kSlots], fb[kSlots];
  int gn[kSlots], g2[kSlots], g3[kSlots], g4[kSlots], g5[kSlots];
  const int pb = x0 > 0 ? x0 - 1 : 0;  // first plane of term j this workgroup needs
#pragma unroll
  for (int sl = 0; sl < kSlots; ++sl) {
    const int task = wave + 4 * sl;
    int r = 0, cc = 0;
    bool act = false;
    if (task < kRows) {
      r = task;
      cc = lane + 1;
      act = true;
    } else if (task == kRows) {
      act = lane < 2 * kRows;
      r = lane >> 1;
      cc = (lane & 1) ? kRow - 1 : 0;
    }
    const int jj = y0 - 1 + r, kk = z0 - 1 + cc;
    tv[sl] = act && jj >= 0 && jj < ny && kk >= 0 && kk < nz;
    tr[sl] = r;
    tc[sl] = cc;
    const int q = tv[sl] ? jj * nz + kk : 0;
    o0[sl] = static_cast<uint32_t>(q);
    o2[sl] = static_cast<uint32_t>(tv[sl] && jj > 0 ? q - nz : q);
    o3[sl] = static_cast<uint32_t>(tv[sl] && jj < ny - 1 ? q + nz : q);
    o4[sl] = static_cast<uint32_t>(tv[sl] && kk > 0 ? q - 1 : q);
    o5[sl] = static_cast<uint32_t>(tv[sl] && kk < nz - 1 ? q + 1 : q);
    wyz[sl] = BC ? (jj == 0) + (jj == ny - 1) + (kk == 0) + (kk == nz - 1) : 0;
    xm[sl] = xc[sl] = T(0);
    lm[sl] = lc[sl] = 0;
    fn[sl] = f2[sl] = f3[sl] = f4[sl] = f5[sl] = fb[sl] = T(0);
    gn[sl] = g2[sl] = g3[sl] = g4[sl] = g5[sl] = 0;
    if (tv[sl]) {
      const int64_t pm = pb > 0 ? pb - 1 : pb;
      xm[sl] = ld_at(x + pm * sx, o0[sl] * W);
      xc[sl] = ld_at(x + pb * sx, o0[sl] * W);
      lm[sl] = lab[pm * sx + o0[sl]];
      lc[sl] = lab[pb * sx + o0[sl]];
    }
  }

  // loads of stage 1 for plane p: the +x neighbour, the four lateral
  // neighbours, their labels and bsrc (planes are fetched in order from pb)
  auto fetch = [&](int p) {
    const int64_t pn = p < nx - 1 ? p + 1 : p;
    const T* xp = x + p * sx;
    const T* xn = x + pn * sx;
    const uint8_t* lp = lab + p * sx;
    const uint8_t* ln = lab + pn * sx;
#pragma unroll
    for (int sl = 0; sl < kSlots; ++sl) {
      if (!tv[sl]) continue;
      fn[sl] = ld_at(xn, o0[sl] * W);
      f2[sl] = ld_at(xp, o2[sl] * W);
      f3[sl] = ld_at(xp, o3[sl] * W);
      f4[sl] = ld_at(xp, o4[sl] * W);
      f5[sl] = ld_at(xp, o5[sl] * W);
      gn[sl] = ln[o0[sl]];
      g2[sl] = lp[o2[sl]];
      g3[sl] = lp[o3[sl]];
      g4[sl] = lp[o4[sl]];
      g5[sl] = lp[o5[sl]];
      if (bs) fb[sl] = ld_at(bs + p * sx, o0[sl] * W);
    }
  };

  // stage 1: term j on plane p from the fetched values, into ring slot p % 4
  auto stage1 = [&](int p) {
    const int slot = p & (kRing - 1);
#pragma unroll
    for (int sl = 0; sl < kSlots; ++sl) {
      if (!tv[sl]) continue;
      const T xp = xc[sl];
      const int lp = lc[sl];
      const T* row = s.tab + lp * kMaxClasses;
      T ax = row[lm[sl]] * (xm[sl] - xp) + row[gn[sl]] * (fn[sl] - xp) + row[g2[sl]] * (f2[sl] - xp) +
             row[g3[sl]] * (f3[sl] - xp) + row[g4[sl]] * (f4[sl] - xp) + row[g5[sl]] * (f5[sl] - xp);
      if (BC) ax -= s.wall[lp] * xp * T(wyz[sl] + (p == 0) + (p == nx - 1));
      T y = c1 * ax;
      if (bs) y += cb * fb[sl];
      zs[slot][tr[sl]][tc[sl]] = y;
      ls[slot][tr[sl]][tc[sl]] = static_cast<uint8_t>(lp);
      xm[sl] = xp;
      xc[sl] = fn[sl];
      lm[sl] = lp;
      lc[sl] = gn[sl];
    }
  };

  // stage 2: term j + 1 on output plane i, running sum and outputs.  Output
  // row of slot sl: staged row r = wave + 4 sl holds output row r - 1.
  const T* acc_in = static_cast<const T*>(op.acc_in);  // may equal acc_out (same voxel only)
  T* y_out = static_cast<T*>(op.y_out);
  T* acc_out = static_cast<T*>(op.acc_out);
  T* u = static_cast<T*>(op.u);
  const T ca = static_cast<T>(op.ca), cs = static_cast<T>(op.cs);
  const bool use_src = op.cs != 0.0;
  const int k = z0 + lane;
  auto stage2 = [&](int i) {
    const int sc = i & (kRing - 1);
    const int sm = i > 0 ? (i - 1) & (kRing - 1) : sc;
    const int sp = i < nx - 1 ? (i + 1) & (kRing - 1) : sc;
    const int wx = BC ? (i == 0) + (i == nx - 1) : 0;
    const int64_t pl = i * sx;
#pragma unroll
    for (int sl = 0; sl < kSlots; ++sl) {
      const int r = wave + 4 * sl;
      if (r < 1 || r > TY) continue;
      const int j = y0 + r - 1;
      if (j >= ny || k >= nz) continue;
      const uint32_t bo = static_cast<uint32_t>(j * nz + k) * W;
      T v = T(0);
      if (acc_in) v = ca * ld_at(acc_in + pl, bo);
      if (use_src) v += cs * ld_at(x + pl, bo);
      const int cc = lane + 1;
      const int rm = j > 0 ? r - 1 : r, rp = j < ny - 1 ? r + 1 : r;
      const int cm = k > 0 ? cc - 1 : cc, cp = k < nz - 1 ? cc + 1 : cc;
      const T yc = zs[sc][r][cc];
      const int l0 = ls[sc][r][cc];
      const T* row = s.tab + l0 * kMaxClasses;
      T ay = row[ls[sm][r][cc]] * (zs[sm][r][cc] - yc) + row[ls[sp][r][cc]] * (zs[sp][r][cc] - yc) +
             row[ls[sc][rm][cc]] * (zs[sc][rm][cc] - yc) + row[ls[sc][rp][cc]] * (zs[sc][rp][cc] - yc) +
             row[ls[sc][r][cm]] * (zs[sc][r][cm] - yc) + row[ls[sc][r][cp]] * (zs[sc][r][cp] - yc);
      if (BC) {
        const int nw = wx + (j == 0) + (j == ny - 1) + (k == 0) + (k == nz - 1);
        ay -= s.wall[l0] * yc * T(nw);
      }
      const T w = c2 * ay;
      v += yc + w;
      if (u) {
        T* up = reinterpret_cast<T*>(reinterpret_cast<char*>(u + pl) + bo);
        *up = *up + v;
      } else {
        if (y_out) *reinterpret_cast<T*>(reinterpret_cast<char*>(y_out + pl) + bo) = w;
        if (acc_out) *reinterpret_cast<T*>(reinterpret_cast<char*>(acc_out + pl) + bo) = v;
      }
    }
  };

  // term j is needed on planes pb .. pe; the outputs are planes x0 .. xe - 1
  const int xe = min(x0 + LP, nx);
  const int pe = min(x0 + LP, nx - 1);
  fetch(pb);
  __syncthreads();  // class tables
  stage1(pb);
  if (x0 > pb) {
    fetch(x0);
    stage1(x0);
  }
  if (x0 + 1 <= pe) fetch(x0 + 1);
#pragma unroll 1
  for (int i = x0; i < xe; ++i) {
    if (i + 1 <= pe) stage1(i + 1);
    if (i + 2 <= pe) fetch(i + 2);
    __syncthreads();
    stage2(i);
  }
}

template <typename T, int BC, int TY>
hipError_t pair_lp(const Geom& g, const PairTiling& tl, const Coef& cf, const TermOp& op, hipStream_t st) {
  const int gz = (g.nz + kPairZ - 1) / kPairZ, gy = (g.ny + TY - 1) / TY;
  const dim3 grid(static_cast<unsigned>(pair_blocks(g, tl))), block(kBlock);
  switch (tl.lp) {
    case 4: k_pair<T, BC, TY, 4><<<grid, block, 0, st>>>(g, gz, gy, cf, op); break;
    case 8: k_pair<T, BC, TY, 8><<<grid, block, 0, st>>>(g, gz, gy, cf, op); break;
    default: k_pair<T, BC, TY, 16><<<grid, block, 0, st>>>(g, gz, gy, cf, op); break;
  }
  return hipGetLastError();
}

template <typename T, int BC>
hipError_t pair_ty(const Geom& g, const PairTiling& tl, const Coef& cf, const TermOp& op, hipStream_t st) {
  if (tl.ty == 4) return pair_lp<T, BC, 4>(g, tl, cf, op, st);
  return pair_lp<T, BC, 8>(g, tl, cf, op, st);
}

}  // namespace

bool pair_tiling_valid(const PairTiling& t) {
  return (t.ty == 4 || t.ty == 8) && (t.lp == 4 || t.lp == 8 || t.lp == 16);
}

int64_t pair_blocks(const Geom& g, const PairTiling& t) {
  const int64_t gz = (g.nz + kPairZ - 1) / kPairZ, gy = (g.ny + t.ty - 1) / t.ty, gx = (g.nx + t.lp - 1) / t.lp;
  return gz * gy * gx;
}

bool pair_grid_ok(const Geom& g, expint_dtype dt) {
  // in-plane byte offsets are 32-bit
  return static_cast<int64_t>(g.ny) * g.nz * dtype_bytes(dt) < (int64_t(1) << 32);
}

hipError_t launch_pair(expint_dtype dt, expint_bc bc, const Geom& g, const PairTiling& tl, const Coef& cf,
                       const TermOp& op, hipStream_t st) {
  if (!pair_tiling_valid(tl) || !cf.labels_form || !op.pair || !op.src || op.ju || op.bsrc2 || !pair_grid_ok(g, dt))
    return hipErrorInvalidValue;
  if (op.y_out == op.src || op.acc_out == op.src || op.u == op.src) return hipErrorInvalidValue;
  if (op.bsrc && (op.y_out == op.bsrc || op.acc_out == op.bsrc || op.u == op.bsrc)) return hipErrorInvalidValue;
  if (dt == EXPINT_F64) {
    if (bc == EXPINT_NOFLUX) return pair_ty<double, 0>(g, tl, cf, op, st);
    return pair_ty<double, 1>(g, tl, cf, op, st);
  }
  if (bc == EXPINT_NOFLUX) return pair_ty<float, 0>(g, tl, cf, op, st);
  return pair_ty<float, 1>(g, tl, cf, op, st);
}

}  // namespace expint
