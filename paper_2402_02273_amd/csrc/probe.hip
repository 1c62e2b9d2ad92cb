// Peak probes: the attainable memory bandwidth and matrix-core rate of the
// device, measured with the same launch machinery as the library's kernels,
// so that rooflines can quote a fraction of the measured peak beside the
// datasheet one.
//
//   copy : dst = src, one 16-byte vector per lane and one launch-wide pass
//          (this shape, with non-temporal loads and stores, beat grid-stride
//          loops and several vectors per lane by 5-40% in sweeps of both);
//          bytes moved = 2 x size.  A buffer well above 256 MB streams from HBM;
//          one below it is served by the Infinity Cache after the first pass,
//          where ordinary (temporal) accesses are the ones to measure.
//   mfma : every wave runs a fixed number of independent v_mfma_f32_32x32x16
//          (bf16 or fp16) chains on register operands; flops = 2 * 32 * 32 * 16
//          per instruction.  The accumulators are written out once so nothing
//          is optimised away.

#include "context.hpp"
#include "internal.hpp"

namespace expint {

namespace {

constexpr int kProbeChains = 8;  // independent accumulators per wave

typedef unsigned int pu32x4 __attribute__((ext_vector_type(4)));

template <int NT>
__global__ __launch_bounds__(kBlock) void k_probe_copy(const pu32x4* __restrict__ src, pu32x4* __restrict__ dst,
                                                       int64_t n16) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n16) return;
  if (NT) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
  else dst[i] = src[i];
}

typedef __bf16 pbf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 pf16x8 __attribute__((ext_vector_type(8)));
typedef float pf32x16 __attribute__((ext_vector_type(16)));

template <int F16>
__global__ __launch_bounds__(kBlock) void k_probe_mfma(int iters, float seed, float* __restrict__ sink) {
  pf32x16 acc[kProbeChains];
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) acc[c] = pf32x16{};
  const float v = seed * static_cast<float>(threadIdx.x & 7);
  if (F16) {
    pf16x8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      a[e] = static_cast<_Float16>(v + e);
      b[e] = static_cast<_Float16>(v - e);
    }
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int c = 0; c < kProbeChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc[c], 0, 0, 0);
  } else {
    pbf16x8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      a[e] = static_cast<__bf16>(v + e);
      b[e] = static_cast<__bf16>(v - e);
    }
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int c = 0; c < kProbeChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c)
#pragma unroll
    for (int r = 0; r < 16; ++r) s += acc[c][r];
  sink[static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x] = s;
}

// Mean milliseconds per launch over reps launches after one warm-up launch.
template <typename F>
int time_ms(F&& launch, int reps, hipStream_t st, double* ms) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return set_error(EXPINT_EHIP, "hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return set_error(EXPINT_EHIP, "hipEventCreate failed");
  }
  hipError_t e = launch();
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_error(EXPINT_EHIP, "probe launch failed: %s", hipGetErrorString(e));
  }
  *ms = static_cast<double>(t) / reps;
  return EXPINT_OK;
}

}  // namespace

}  // namespace expint

using namespace expint;

extern "C" {

int expint_probe_copy(const void* src, void* dst, int64_t bytes, int32_t reps, int32_t nontemporal, void* stream,
                      double* ms) {
  if (!src || !dst || !ms || reps < 1) return set_error(EXPINT_EINVAL, "NULL argument or reps < 1");
  if (bytes < 16 || bytes % 16 != 0) return set_error(EXPINT_EINVAL, "bytes must be a positive multiple of 16");
  if (bytes / 16 > static_cast<int64_t>(kBlock) * 0x7fffffff)
    return set_error(EXPINT_EINVAL, "bytes exceeds one launch");
  if ((reinterpret_cast<uintptr_t>(src) & 15) || (reinterpret_cast<uintptr_t>(dst) & 15))
    return set_error(EXPINT_EINVAL, "buffers must be 16-byte aligned");
  const char* s = static_cast<const char*>(src);
  const char* d = static_cast<const char*>(dst);
  if (s < d + bytes && d < s + bytes) return set_error(EXPINT_EINVAL, "buffers overlap");
  const int64_t n16 = bytes / 16;
  const unsigned grid = static_cast<unsigned>((n16 + kBlock - 1) / kBlock);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const auto* in = static_cast<const pu32x4*>(src);
  auto* out = static_cast<pu32x4*>(dst);
  return time_ms(
      [&] {
        if (nontemporal) k_probe_copy<1><<<grid, kBlock, 0, st>>>(in, out, n16);
        else k_probe_copy<0><<<grid, kBlock, 0, st>>>(in, out, n16);
        return hipGetLastError();
      },
      reps, st, ms);
}

int expint_probe_mfma(int32_t f16, int32_t iters, int32_t blocks, void* sink, void* stream, double* tflops) {
  if (!sink || !tflops || iters < 1 || blocks < 1) return set_error(EXPINT_EINVAL, "bad probe arguments");
  hipStream_t st = static_cast<hipStream_t>(stream);
  float* out = static_cast<float*>(sink);
  double ms = 0.0;
  const int rc = time_ms(
      [&] {
        if (f16) k_probe_mfma<1><<<blocks, kBlock, 0, st>>>(iters, 1e-3f, out);
        else k_probe_mfma<0><<<blocks, kBlock, 0, st>>>(iters, 1e-3f, out);
        return hipGetLastError();
      },
      3, st, &ms);
  if (rc) return rc;
  const double waves = static_cast<double>(blocks) * (kBlock / 64);
  const double flops = waves * iters * kProbeChains * 2.0 * 32 * 32 * 16;
  *tflops = flops / (ms * 1e-3) / 1e12;
  return EXPINT_OK;
}

}  // extern "C"
