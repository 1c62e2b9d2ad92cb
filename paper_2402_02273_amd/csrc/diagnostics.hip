// Label ingestion and tumour diagnostics (sections 3.1, 3.2, 3.5).
//
//  * labels from an 8-bit scan: stencil point i of n along an axis of N scan
//    samples takes sample floor((2i + 1) N / (2n)) (the sample whose cell
//    holds the point's cell centre); its label is the number of thresholds
//    strictly below the intensity.  Integer arithmetic throughout.
//  * tumour size: the largest squared distance, in grid steps, between two
//    points with u > threshold.  A farthest pair of a finite set consists of
//    vertices of its convex hull, and a hull vertex that shares an axis line
//    with other points of the set is an end of the set's run on that line.
//    So only points that are first or last on their x-, y- and z-lines are
//    candidates: three line-extent passes, a candidate pass, then all pairs
//    of candidates (an integer maximum, then the smallest pair reaching it,
//    both by 64-bit atomics, so the result does not depend on the order of
//    the candidates).
//  * tumour volume per step: a deterministic reduction of sum u after every
//    step into one slot per step (host divides by the voxel count).

#include <cmath>
#include <cstdio>
#include <mutex>

#include "context.hpp"
#include "internal.hpp"

// The static workspace of expint_tumour_size_static: one copy per device,
// held until the process ends.  Host code never passes `scratch` itself to a
// kernel (that name is a host-side stand-in): it passes the device address
// that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[EXPINT_STATIC_SCRATCH_BYTES];

namespace expint {

namespace {

constexpr int kMaxThresholds = 7;

struct Thresholds {
  int n;
  int t[kMaxThresholds];
};

// Workgroup: 64 lanes along z by 4 rows along y; grid z covers x, so a lane
// knows (i, j, k) without divisions.  W = uint32_t when every (2i + 1) * N
// product fits in 32 bits (the host checks), else uint64_t.
constexpr int kLabZ = 64, kLabY = kBlock / kLabZ;

template <typename W>
__global__ __launch_bounds__(kBlock) void k_labels_from_intensity(const uint8_t* __restrict__ img, int NI, int NJ,
                                                                  int NK, int nx, int ny, int nz, Thresholds th,
                                                                  uint8_t* __restrict__ lab) {
  const int k = static_cast<int>(blockIdx.x) * kLabZ + static_cast<int>(threadIdx.x);
  const int j = static_cast<int>(blockIdx.y) * kLabY + static_cast<int>(threadIdx.y);
  const int i = static_cast<int>(blockIdx.z);
  if (k >= nz || j >= ny) return;
  const W I = ((2 * static_cast<W>(i) + 1) * static_cast<W>(NI)) / (2 * static_cast<W>(nx));
  const W J = ((2 * static_cast<W>(j) + 1) * static_cast<W>(NJ)) / (2 * static_cast<W>(ny));
  const W K = ((2 * static_cast<W>(k) + 1) * static_cast<W>(NK)) / (2 * static_cast<W>(nz));
  const int v = img[(static_cast<int64_t>(I) * NJ + static_cast<int64_t>(J)) * NK + static_cast<int64_t>(K)];
  int c = 0;
  for (int q = 0; q < th.n; ++q) c += v > th.t[q];
  lab[(static_cast<int64_t>(i) * ny + j) * nz + k] = static_cast<uint8_t>(c);
}

// First and last index along one axis line with u > thr (-1, -1 if none).
// Line l of `lines`; element e of the line sits at base(l) + e * stride.
template <typename T, int AXIS>
__global__ __launch_bounds__(kBlock) void k_line_extent(const T* __restrict__ u, int nx, int ny, int nz, double thr,
                                                        int* __restrict__ lo, int* __restrict__ hi) {
  const int64_t l = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  int64_t lines, base, stride;
  int len;
  if (AXIS == 0) {  // x-lines, indexed by (j, k)
    lines = static_cast<int64_t>(ny) * nz;
    base = l;
    stride = static_cast<int64_t>(ny) * nz;
    len = nx;
  } else if (AXIS == 1) {  // y-lines, indexed by (i, k)
    lines = static_cast<int64_t>(nx) * nz;
    base = (l / nz) * ny * nz + l % nz;
    stride = nz;
    len = ny;
  } else {  // z-lines, indexed by (i, j)
    lines = static_cast<int64_t>(nx) * ny;
    base = l * nz;
    stride = 1;
    len = nz;
  }
  if (l >= lines) return;
  int first = -1, last = -1;
  for (int e = 0; e < len; ++e) {
    if (static_cast<double>(u[base + e * stride]) > thr) {
      if (first < 0) first = e;
      last = e;
    }
  }
  lo[l] = first;
  hi[l] = last;
}

// Candidates: the ends of each x-line's run that are also ends of their y-
// and z-lines' runs; appended (in any order) as linear indices.
__global__ __launch_bounds__(kBlock) void k_candidates(int nx, int ny, int nz, const int* __restrict__ xlo,
                                                       const int* __restrict__ xhi, const int* __restrict__ ylo,
                                                       const int* __restrict__ yhi, const int* __restrict__ zlo,
                                                       const int* __restrict__ zhi, int* __restrict__ count,
                                                       int* __restrict__ cand) {
  const int64_t l = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (l >= static_cast<int64_t>(ny) * nz) return;
  const int j = static_cast<int>(l / nz), k = static_cast<int>(l % nz);
  const int a = xlo[l], b = xhi[l];
  if (a < 0) return;
  for (int w = 0; w < (a == b ? 1 : 2); ++w) {
    const int i = w == 0 ? a : b;
    const int64_t yl = static_cast<int64_t>(i) * nz + k, zl = static_cast<int64_t>(i) * ny + j;
    const bool ey = ylo[yl] == j || yhi[yl] == j;
    const bool ez = zlo[zl] == k || zhi[zl] == k;
    if (ey && ez) {
      const int pos = atomicAdd(count, 1);
      cand[pos] = static_cast<int>((static_cast<int64_t>(i) * ny + j) * nz + k);
    }
  }
}

constexpr int kPairChunk = 4096;  // candidates b per workgroup column

struct Coord {
  int i, j, k, lin;
};

__device__ __forceinline__ Coord decode(int lin, int ny, int nz) {
  Coord c;
  c.lin = lin;
  c.k = lin % nz;
  const int t = lin / nz;
  c.j = t % ny;
  c.i = t / ny;
  return c;
}

__device__ __forceinline__ unsigned long long dist2(const Coord& a, const Coord& b) {
  const long long di = a.i - b.i, dj = a.j - b.j, dk = a.k - b.k;
  return static_cast<unsigned long long>(di * di + dj * dj + dk * dk);
}

// PHASE 0: *best = max d2 over candidate pairs.  PHASE 1: *key = min over the
// pairs with d2 == *best of (lo << 32 | hi), lo < hi their linear indices.
// Grid: x covers the candidates a (one per lane), y the chunks of b.
template <int PHASE>
__global__ __launch_bounds__(kBlock) void k_pairs(const int* __restrict__ cand, const int* __restrict__ count,
                                                  int ny, int nz, unsigned long long* __restrict__ best,
                                                  unsigned long long* __restrict__ key) {
  __shared__ Coord sb[kBlock];
  const int C = *count;
  const int ia = blockIdx.x * kBlock + threadIdx.x;
  const int b0 = blockIdx.y * kPairChunk;
  if (blockIdx.x * kBlock >= C || b0 >= C) return;  // uniform per workgroup
  const bool has_a = ia < C;
  const Coord a = decode(has_a ? cand[ia] : 0, ny, nz);
  const unsigned long long target = PHASE == 1 ? *best : 0ull;
  unsigned long long mine = PHASE == 0 ? 0ull : ~0ull;
  const int b1 = min(C, b0 + kPairChunk);
  for (int t = b0; t < b1; t += kBlock) {
    __syncthreads();
    if (t + static_cast<int>(threadIdx.x) < b1) sb[threadIdx.x] = decode(cand[t + threadIdx.x], ny, nz);
    __syncthreads();
    const int nb = min(kBlock, b1 - t);
    if (has_a) {
      for (int q = 0; q < nb; ++q) {
        const unsigned long long d = dist2(a, sb[q]);
        if (PHASE == 0) {
          mine = d > mine ? d : mine;
        } else if (d == target) {
          const unsigned lo = static_cast<unsigned>(min(a.lin, sb[q].lin));
          const unsigned hi = static_cast<unsigned>(max(a.lin, sb[q].lin));
          const unsigned long long kk = (static_cast<unsigned long long>(lo) << 32) | hi;
          mine = kk < mine ? kk : mine;
        }
      }
    }
  }
  if (!has_a) return;
  if (PHASE == 0) atomicMax(best, mine);
  else if (mine != ~0ull) atomicMin(key, mine);
}

__global__ void k_pairs_init(int* count, unsigned long long* best, unsigned long long* key) {
  *count = 0;
  *best = 0ull;
  *key = ~0ull;
}

unsigned grid_of(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }

// Workspace of one tumour-size pass: line extents (two ints per line of each
// axis), candidates (up to two per x-line), the candidate count and the
// 64-bit best distance and pair key.
struct SizeWork {
  int* ext;
  int* cand;
  int* count;
  unsigned long long* best;  // best and key adjacent: one read-back copy
  unsigned long long* key;
};

struct SizeDims {
  int64_t lx, ly, lz, cmax, pgy;
};

// Line counts of the grid; EXPINT_EUNSUPPORTED when the pair pass cannot
// cover its cross-section.
int size_dims(int nx, int ny, int nz, SizeDims* d) {
  d->lx = static_cast<int64_t>(ny) * nz;
  d->ly = static_cast<int64_t>(nx) * nz;
  d->lz = static_cast<int64_t>(nx) * ny;
  d->cmax = 2 * d->lx;  // at most two candidates per x-line
  d->pgy = (d->cmax + kPairChunk - 1) / kPairChunk;
  if (d->cmax > INT32_MAX || d->pgy > 65535)
    return set_error(EXPINT_EUNSUPPORTED, "grid cross-section too large for the tumour size pass");
  return EXPINT_OK;
}

// Bytes of SizeWork laid out back to back from a 256-byte aligned base:
// extents, candidates, then 64 bytes of counters.
size_t size_work_bytes(const SizeDims& d) {
  const size_t ints = static_cast<size_t>(2 * (d.lx + d.ly + d.lz) + d.cmax);
  return ((ints * sizeof(int) + 255) / 256) * 256 + 64;
}

SizeWork size_work_at(void* base, const SizeDims& d) {
  SizeWork w;
  char* p = static_cast<char*>(base);
  w.ext = reinterpret_cast<int*>(p);
  w.cand = w.ext + 2 * (d.lx + d.ly + d.lz);
  const size_t ints = static_cast<size_t>(2 * (d.lx + d.ly + d.lz) + d.cmax);
  char* cnt = p + ((ints * sizeof(int) + 255) / 256) * 256;
  w.count = reinterpret_cast<int*>(cnt);
  w.best = reinterpret_cast<unsigned long long*>(cnt + 16);
  w.key = w.best + 1;
  return w;
}

// The kernels of one pass on stream st; every workspace word the pass reads
// is written by it first (the counters by k_pairs_init).
hipError_t enqueue_size_pass(expint_dtype dt, int nx, int ny, int nz, const void* u, double threshold,
                             const SizeDims& d, const SizeWork& w, hipStream_t st) {
  int* xlo = w.ext;
  int* xhi = xlo + d.lx;
  int* ylo = xhi + d.lx;
  int* yhi = ylo + d.ly;
  int* zlo = yhi + d.ly;
  int* zhi = zlo + d.lz;
  k_pairs_init<<<1, 1, 0, st>>>(w.count, w.best, w.key);
  if (dt == EXPINT_F64) {
    const double* f = static_cast<const double*>(u);
    k_line_extent<double, 0><<<grid_of(d.lx), kBlock, 0, st>>>(f, nx, ny, nz, threshold, xlo, xhi);
    k_line_extent<double, 1><<<grid_of(d.ly), kBlock, 0, st>>>(f, nx, ny, nz, threshold, ylo, yhi);
    k_line_extent<double, 2><<<grid_of(d.lz), kBlock, 0, st>>>(f, nx, ny, nz, threshold, zlo, zhi);
  } else {
    const float* f = static_cast<const float*>(u);
    k_line_extent<float, 0><<<grid_of(d.lx), kBlock, 0, st>>>(f, nx, ny, nz, threshold, xlo, xhi);
    k_line_extent<float, 1><<<grid_of(d.ly), kBlock, 0, st>>>(f, nx, ny, nz, threshold, ylo, yhi);
    k_line_extent<float, 2><<<grid_of(d.lz), kBlock, 0, st>>>(f, nx, ny, nz, threshold, zlo, zhi);
  }
  k_candidates<<<grid_of(d.lx), kBlock, 0, st>>>(nx, ny, nz, xlo, xhi, ylo, yhi, zlo, zhi, w.count, w.cand);
  // sized for the largest candidate count; workgroups past the actual count
  // return at once
  const dim3 pgrid(grid_of(d.cmax), static_cast<unsigned>(d.pgy));
  k_pairs<0><<<pgrid, kBlock, 0, st>>>(w.cand, w.count, ny, nz, w.best, w.key);
  k_pairs<1><<<pgrid, kBlock, 0, st>>>(w.cand, w.count, ny, nz, w.best, w.key);
  return hipGetLastError();
}

// Reads the pass's result back (synchronises st) into *d2 and pair.
hipError_t read_size_result(const SizeWork& w, hipStream_t st, int64_t* d2, int64_t* pair) {
  int count = 0;
  unsigned long long out[2] = {0, 0};
  int first = -1;
  hipError_t e;
  if ((e = hipMemcpyAsync(&count, w.count, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(out, w.best, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return e;
  if ((e = hipMemcpyAsync(&first, w.cand, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  if (count == 0) {
    *d2 = -1;
    if (pair) pair[0] = pair[1] = -1;
  } else if (count == 1) {
    *d2 = 0;
    if (pair) pair[0] = pair[1] = first;
  } else {
    *d2 = static_cast<int64_t>(out[0]);
    if (pair) {
      pair[0] = static_cast<int64_t>(out[1] >> 32);
      pair[1] = static_cast<int64_t>(out[1] & 0xffffffffull);
    }
  }
  return hipSuccess;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch`, looked up once per device.
int static_scratch(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return set_error(EXPINT_EUNSUPPORTED, "device index %d", device);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return set_error(EXPINT_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    }
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return EXPINT_OK;
}

}  // namespace

}  // namespace expint

using namespace expint;

extern "C" {

int expint_labels_from_intensity(const uint8_t* image, int32_t ni, int32_t nj, int32_t nk, const int32_t* thresholds,
                                 int32_t n_thresholds, int32_t nx, int32_t ny, int32_t nz, uint8_t* labels,
                                 void* stream) {
  if (!image || !labels || !thresholds) return set_error(EXPINT_EINVAL, "NULL argument");
  if (ni < 1 || nj < 1 || nk < 1 || nx < 1 || ny < 1 || nz < 1)
    return set_error(EXPINT_EINVAL, "image and grid dims must be >= 1");
  if (n_thresholds < 1 || n_thresholds > kMaxThresholds)
    return set_error(EXPINT_EINVAL, "n_thresholds must be in 1..%d", kMaxThresholds);
  Thresholds th{};
  th.n = n_thresholds;
  for (int q = 0; q < n_thresholds; ++q) {
    th.t[q] = thresholds[q];
    if (q > 0 && th.t[q] <= th.t[q - 1]) return set_error(EXPINT_EINVAL, "thresholds must increase");
  }
  const int64_t n = product_within(nx, ny, nz, (int64_t(1) << 31) * kBlock);
  const int64_t nimg = product_within(ni, nj, nk, INT64_MAX);
  if (n < 0) return set_error(EXPINT_EINVAL, "grid too large");
  if (nimg < 0) return set_error(EXPINT_EINVAL, "image too large");
  const char* a = reinterpret_cast<const char*>(image);
  const char* b = reinterpret_cast<const char*>(labels);
  if (a < b + n && b < a + nimg) return set_error(EXPINT_EINVAL, "image and labels overlap");
  if (ny > 65535 || nx > 65535) return set_error(EXPINT_EUNSUPPORTED, "nx and ny must be <= 65535");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const dim3 grid((nz + kLabZ - 1) / kLabZ, (ny + kLabY - 1) / kLabY, nx), block(kLabZ, kLabY);
  auto fits32 = [](int64_t npts, int64_t N) { return (2 * npts + 1) * N < (int64_t(1) << 32); };
  if (fits32(nx, ni) && fits32(ny, nj) && fits32(nz, nk))
    k_labels_from_intensity<uint32_t><<<grid, block, 0, st>>>(image, ni, nj, nk, nx, ny, nz, th, labels);
  else
    k_labels_from_intensity<uint64_t><<<grid, block, 0, st>>>(image, ni, nj, nk, nx, ny, nz, th, labels);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(EXPINT_EHIP, "label kernel launch failed: %s", hipGetErrorString(e));
  return EXPINT_OK;
}

int expint_tumour_size(expint_ctx* c, const void* u, double threshold, int64_t* d2, int64_t* pair) {
  CHECK_CTX(c);
  if (!u || !d2) return set_error(EXPINT_EINVAL, "NULL argument");
  if (std::isnan(threshold)) return set_error(EXPINT_EINVAL, "threshold is NaN");
  int rc = ensure_device(c);
  if (rc) return rc;
  const Geom& g = c->g;
  SizeDims d;
  if ((rc = size_dims(g.nx, g.ny, g.nz, &d))) return rc;
  auto& w = c->diag;
  if (!w.ext) {
    // allocated on first use; all or nothing
    void* base = nullptr;
    if ((rc = c->arena.alloc(&base, size_work_bytes(d)))) return rc;
    const SizeWork sw = size_work_at(base, d);
    w.ext = sw.ext;
    w.cand = sw.cand;
    w.count = sw.count;
    w.best = sw.best;
    w.key = sw.key;
  }
  const SizeWork sw{w.ext, w.cand, w.count, w.best, w.key};
  HIP_TRY(c, enqueue_size_pass(c->dtype, g.nx, g.ny, g.nz, u, threshold, d, sw, c->stream));
  HIP_TRY(c, read_size_result(sw, c->stream, d2, pair));
  return EXPINT_OK;
}

int expint_tumour_size_static(const void* u, int32_t dtype, int32_t nx, int32_t ny, int32_t nz, double threshold,
                              int64_t* d2, int64_t* pair, void* stream) {
  if (!u || !d2) return set_error(EXPINT_EINVAL, "NULL argument");
  if (dtype != EXPINT_F32 && dtype != EXPINT_F64) return set_error(EXPINT_EINVAL, "dtype must be F32 or F64");
  if (nx < 1 || ny < 1 || nz < 1) return set_error(EXPINT_EINVAL, "grid dims must be >= 1");
  if (std::isnan(threshold)) return set_error(EXPINT_EINVAL, "threshold is NaN");
  SizeDims d;
  int rc = size_dims(nx, ny, nz, &d);
  if (rc) return rc;
  const size_t need = size_work_bytes(d);
  if (need > static_cast<size_t>(EXPINT_STATIC_SCRATCH_BYTES))
    return set_error(EXPINT_EINVAL,
                     "grid %dx%dx%d needs %zu bytes of workspace, above the %d-byte static workspace of "
                     "expint_tumour_size_static",
                     nx, ny, nz, need, EXPINT_STATIC_SCRATCH_BYTES);
  int device = -1;
  if (hipGetDevice(&device) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(EXPINT_EHIP, "no HIP device");
  }
  void* base = nullptr;
  if ((rc = static_scratch(device, &base))) return rc;
  const SizeWork w = size_work_at(base, d);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = enqueue_size_pass(static_cast<expint_dtype>(dtype), nx, ny, nz, u, threshold, d, w, st);
  if (e == hipSuccess) e = read_size_result(w, st, d2, pair);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_error(EXPINT_EHIP, "tumour size pass failed: %s", hipGetErrorString(e));
  }
  return EXPINT_OK;
}

}  // extern "C"
