// Batched sweeps: one launch advances op t of every active instance of a
// batch of independent grids (different sizes, coefficients and plans).
//
// The launch's work list is the concatenation of each instance's tiles; each
// XCD takes a contiguous eighth of it and its workgroups walk that range
// with a stride; a workgroup finds the instance owning tile w by binary search over the per-op
// block offsets, loads that instance's class table into LDS and runs the same
// column sweep as the single-grid kernels (sweep_device.hpp) with the
// instance's own tile shape (bx x by threads of a 1-D workgroup, scalar or
// z-vectorised as the instance's autotuned tiling says).  The ops of one
// launch share the term flavour and the plane count lp, which are
// compile-time parameters as in the single-grid kernels.
// Every workgroup exits after its last work item: no inter-workgroup waits.

#include "batch.hpp"
#include "sweep_device.hpp"

namespace expint {

namespace {

template <typename T, int BC, int KIND, int FL, int LP>
__global__ __launch_bounds__(kBlock) void k_batch(const BatchItem* __restrict__ items, const T* __restrict__ tables,
                                                  int nitems, int total) {
  static_assert(sizeof(BatchItem) % 8 == 0, "BatchItem is staged as 32-bit words");
  __shared__ __align__(16) uint32_t si_words[kBatchMaxOps * sizeof(BatchItem) / 4];
  __shared__ LdsCoef<T> st[kBatchMaxOps];
  const BatchItem* si = reinterpret_cast<const BatchItem*>(si_words);
  // stage the launch's descriptors and class tables once per workgroup
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(items);
    uint32_t* dst = si_words;
    const int words = nitems * static_cast<int>(sizeof(BatchItem) / 4);
    for (int t = threadIdx.x; t < words; t += kBlock) dst[t] = src[t];
    const int vals = nitems * (kTab + kMaxClasses);
    for (int t = threadIdx.x; t < vals; t += kBlock) {
      const int it = t / (kTab + kMaxClasses), r = t % (kTab + kMaxClasses);
      if (r < kTab) st[it].tab[r] = tables[t];
      else st[it].wall[r - kTab] = tables[t];
    }
  }
  __syncthreads();
  // Workgroups are dealt to the 8 XCDs round-robin; give each XCD a contiguous
  // range of work items so that neighbouring tiles (and planes) share its L2.
  int w0 = blockIdx.x, w1 = total, dw = gridDim.x;
  if ((gridDim.x & 7) == 0) {
    const int per = gridDim.x >> 3, xcd = blockIdx.x & 7, chunk = (total + 7) >> 3;
    w0 = xcd * chunk + (blockIdx.x >> 3);
    w1 = min(total, (xcd + 1) * chunk);
    dw = per;
  }
  for (int w = w0; w < w1; w += dw) {
    int lo = 0, hi = nitems - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (si[mid].block_start <= w) lo = mid;
      else hi = mid - 1;
    }
    const BatchItem& it = si[lo];
    const int L = w - it.block_start;
    const int t = static_cast<int>(it.gx.div(static_cast<uint32_t>(L)));
    const int bxi = L - t * static_cast<int>(it.gx.d);
    const int xg = static_cast<int>(it.gy.div(static_cast<uint32_t>(t)));
    const int byi = t - xg * static_cast<int>(it.gy.d);
    const int i0 = xg * LP;
    const int j = byi * it.by + (static_cast<int>(threadIdx.x) >> it.bx_log2);
    const int kq = static_cast<int>(threadIdx.x) & (it.bx - 1);
    const int k = bxi * it.bx + kq;  // vec: the lane's 4-voxel vector index
    if (j < it.ny && k < (it.vec ? (it.nz >> 2) : it.nz)) {
      Geom g;
      g.nx = it.nx;
      g.ny = it.ny;
      g.nz = it.nz;
      g.n = static_cast<int64_t>(it.nx) * it.ny * it.nz;
      Coef cf{};
      cf.labels_form = true;
      cf.labels = it.labels;
      SweepArgs a{};
      if (is_term(KIND)) {
        a.op = it.op;
      } else {
        a.x = it.op.src;
        a.out = it.op.y_out;
        a.rho = it.rho;
      }
      if (it.vec) sweep_column4<T, BC, LP, KIND, FL>(g, it.labels, st[lo], a, i0, j, k, kq, it.bx, true);
      else sweep_column<T, BC, LP, KIND, FL>(g, cf, st[lo], a, i0, j, k, LP);
    }
  }
}

}  // namespace

template <typename T, int BC, int KIND, int FL>
static void batch_lp(int lp, const BatchItem* items, const void* tables, int n, int total, dim3 g, hipStream_t st) {
  const dim3 b(kBlock);
  const T* tb = static_cast<const T*>(tables);
  switch (lp) {
    case 1: k_batch<T, BC, KIND, FL, 1><<<g, b, 0, st>>>(items, tb, n, total); break;
    case 2: k_batch<T, BC, KIND, FL, 2><<<g, b, 0, st>>>(items, tb, n, total); break;
    default: k_batch<T, BC, KIND, FL, 4><<<g, b, 0, st>>>(items, tb, n, total); break;
  }
}

template <typename T, int BC, int KIND>
static void batch_terms(int flavor, int lp, const BatchItem* items, const void* tables, int n, int total, dim3 g,
                        hipStream_t st) {
  switch (flavor) {
    case kSkip: batch_lp<T, BC, KIND, kSkip>(lp, items, tables, n, total, g, st); break;
    case kFlushY: batch_lp<T, BC, KIND, kFlushY>(lp, items, tables, n, total, g, st); break;
    case kFlushNoY: batch_lp<T, BC, KIND, kFlushNoY>(lp, items, tables, n, total, g, st); break;
    case kFirst: batch_lp<T, BC, KIND, kFirst>(lp, items, tables, n, total, g, st); break;
    default: batch_lp<T, BC, KIND, kGeneric>(lp, items, tables, n, total, g, st); break;
  }
}

template <typename T, int BC>
static void batch_typed(bool rhs, bool lin, int flavor, int lp, const BatchItem* items, const void* tables, int n,
                        int total, dim3 g, hipStream_t st) {
  if (rhs) batch_lp<T, BC, kRhs, kGeneric>(lp, items, tables, n, total, g, st);
  else if (lin) batch_terms<T, BC, kTermJ>(flavor, lp, items, tables, n, total, g, st);
  else batch_terms<T, BC, kTerm>(flavor, lp, items, tables, n, total, g, st);
}

hipError_t launch_batch(expint_dtype dt, expint_bc bc, bool rhs, bool lin, int flavor, int lp,
                        const BatchItem* items, const void* tables, int nitems, int total_blocks, int grid,
                        hipStream_t st) {
  if (nitems < 1 || nitems > kBatchMaxOps) return hipErrorInvalidValue;
  const dim3 g(grid);
  if (dt == EXPINT_F64) {
    if (bc == EXPINT_NOFLUX) batch_typed<double, 0>(rhs, lin, flavor, lp, items, tables, nitems, total_blocks, g, st);
    else batch_typed<double, 1>(rhs, lin, flavor, lp, items, tables, nitems, total_blocks, g, st);
  } else {
    if (bc == EXPINT_NOFLUX) batch_typed<float, 0>(rhs, lin, flavor, lp, items, tables, nitems, total_blocks, g, st);
    else batch_typed<float, 1>(rhs, lin, flavor, lp, items, tables, nitems, total_blocks, g, st);
  }
  return hipGetLastError();
}

}  // namespace expint
