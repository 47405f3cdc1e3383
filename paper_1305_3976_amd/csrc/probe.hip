// probe.hip -- streaming-rate probe of libibgm.so (include/ibgm_probe.h):
// the HBM rate a plain hand-written elementwise kernel reaches on this GPU
// for a given mix of read and write streams, the practical ceiling that the
// step's bandwidth-bound kernels are measured against.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "errors.h"
#include "ibgm_probe.h"

using ibgm_err::fail;

namespace {

constexpr int kMaxStreams = 12;

struct StreamArgs {
  const float4 *src[kMaxStreams];
  float4 *dst[kMaxStreams];
  int nsrc, ndst;
  int64_t n4;  // float4 elements per stream
};

// Every thread reads element i of each source stream, adds them, and writes
// the sum (offset by the stream index) to each destination stream: one
// 16-byte load per source and one 16-byte store per destination per element,
// grid-stride.
__global__ void __launch_bounds__(256) k_stream(StreamArgs a) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n4;
       i += (int64_t)gridDim.x * blockDim.x) {
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int q = 0; q < a.nsrc; q++) {
      const float4 v = a.src[q][i];
      s.x += v.x, s.y += v.y, s.z += v.z, s.w += v.w;
    }
    for (int q = 0; q < a.ndst; q++) a.dst[q][i] = make_float4(s.x + q, s.y, s.z, s.w);
  }
}

}  // namespace

extern "C" ib_status ib_probe_stream_rate(const float *const *src, int32_t nsrc,
                                          float *const *dst, int32_t ndst, int64_t n,
                                          int32_t reps, void *hip_stream, double *bytes_per_s) {
  if (!bytes_per_s || nsrc < 0 || ndst < 0 || nsrc + ndst < 1 || nsrc > kMaxStreams ||
      ndst > kMaxStreams || n < 4 || n % 4 != 0 || reps < 1 || reps > 1000)
    return fail(IB_E_INVALID, "bad stream probe arguments");
  StreamArgs a{};
  for (int q = 0; q < nsrc; q++) {
    if (!src || !src[q] || ((uintptr_t)src[q] & 15)) return fail(IB_E_INVALID, "source %d", q);
    a.src[q] = (const float4 *)src[q];
  }
  for (int q = 0; q < ndst; q++) {
    if (!dst || !dst[q] || ((uintptr_t)dst[q] & 15)) return fail(IB_E_INVALID, "destination %d", q);
    a.dst[q] = (float4 *)dst[q];
  }
  a.nsrc = nsrc;
  a.ndst = ndst;
  a.n4 = n / 4;
  hipStream_t st = (hipStream_t)hip_stream;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    ncu = 256;
  // eight workgroups per compute unit, grid-stride over the rest
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((a.n4 + 255) / 256, 8 * ncu));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return fail(IB_E_DEVICE, "hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(IB_E_DEVICE, "hipEventCreate failed");
  }
  hipLaunchKernelGGL(k_stream, dim3(grid), dim3(256), 0, st, a);  // warm-up
  (void)hipEventRecord(e0, st);
  for (int r = 0; r < reps; r++) hipLaunchKernelGGL(k_stream, dim3(grid), dim3(256), 0, st, a);
  (void)hipEventRecord(e1, st);
  hipError_t e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess || hipGetLastError() != hipSuccess || ms <= 0.f)
    return fail(IB_E_DEVICE, "stream probe failed");
  *bytes_per_s = (double)(nsrc + ndst) * (double)n * 4.0 * reps / (ms * 1e-3);
  return IB_OK;
}
