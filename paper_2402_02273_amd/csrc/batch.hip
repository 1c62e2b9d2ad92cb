// Batched sweeps: one launch advances op t of every active instance of a
// batch of independent grids (different sizes, coefficients and plans).
//
// The launch's work list is the concatenation of each instance's tiles; a
// workgroup walks it with a grid stride (w = blockIdx.x, blockIdx.x + grid,
// ...), finds the instance owning tile w by binary search over the per-op
// block offsets, loads that instance's class table into LDS and runs the same
// column sweep as the single-grid kernels (sweep_device.hpp) with the
// instance's own tile shape (bx x by threads of a 1-D workgroup, lp planes).
// Every workgroup exits after its last work item: no inter-workgroup waits.

#include "batch.hpp"
#include "sweep_device.hpp"

namespace expint {

namespace {

template <typename T, int BC, int KIND>
__global__ __launch_bounds__(kBlock) void k_batch(const BatchInst* __restrict__ insts,
                                                  const BatchOp* __restrict__ ops, int nops, int total) {
  __shared__ LdsCoef<T> s;
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    int lo = 0, hi = nops - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (ops[mid].block_start <= w) lo = mid;
      else hi = mid - 1;
    }
    const BatchOp& bo = ops[lo];
    const BatchInst& in = insts[bo.inst];
    __syncthreads();  // the previous item's readers are done with the table
    load_tables(s, in.coef, static_cast<int>(threadIdx.x), kBlock);
    __syncthreads();
    const int L = w - bo.block_start;
    const int bxi = L % in.gx;
    const int t = L / in.gx;
    const int byi = t % in.gy;
    const int i0 = (t / in.gy) * in.lp;
    const int j = byi * in.by + static_cast<int>(threadIdx.x) / in.bx;
    const int k = bxi * in.bx + static_cast<int>(threadIdx.x) % in.bx;
    if (j < in.g.ny && k < in.g.nz) {
      SweepArgs a{};
      if (KIND == kTerm) {
        a.op = bo.op;
      } else {
        a.x = bo.op.src;
        a.out = bo.op.y_out;
        a.rho = in.rho;
      }
      sweep_column<T, BC, 0, KIND, kRuntimeFlavor>(in.g, in.coef, s, a, i0, j, k, in.lp);
    }
  }
}

}  // namespace

hipError_t launch_batch(expint_dtype dt, expint_bc bc, bool rhs, const BatchInst* insts, const BatchOp* ops, int nops,
                        int total_blocks, int grid, hipStream_t st) {
  const dim3 g(grid), b(kBlock);
  if (dt == EXPINT_F64) {
    if (bc == EXPINT_NOFLUX) {
      if (rhs) k_batch<double, 0, kRhs><<<g, b, 0, st>>>(insts, ops, nops, total_blocks);
      else k_batch<double, 0, kTerm><<<g, b, 0, st>>>(insts, ops, nops, total_blocks);
    } else {
      if (rhs) k_batch<double, 1, kRhs><<<g, b, 0, st>>>(insts, ops, nops, total_blocks);
      else k_batch<double, 1, kTerm><<<g, b, 0, st>>>(insts, ops, nops, total_blocks);
    }
  } else {
    if (bc == EXPINT_NOFLUX) {
      if (rhs) k_batch<float, 0, kRhs><<<g, b, 0, st>>>(insts, ops, nops, total_blocks);
      else k_batch<float, 0, kTerm><<<g, b, 0, st>>>(insts, ops, nops, total_blocks);
    } else {
      if (rhs) k_batch<float, 1, kRhs><<<g, b, 0, st>>>(insts, ops, nops, total_blocks);
      else k_batch<float, 1, kTerm><<<g, b, 0, st>>>(insts, ops, nops, total_blocks);
    }
  }
  return hipGetLastError();
}

}  // namespace expint
