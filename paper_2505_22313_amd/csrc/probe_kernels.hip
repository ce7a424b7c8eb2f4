// Plain HBM stream kernels: the bandwidth ceilings the propagation passes
// are measured against (dop_probe_bandwidth).  Every lane moves 16-byte
// vectors with non-temporal hints, four independent vectors per iteration,
// over a grid-stride loop of many resident blocks.
#include <hip/hip_runtime.h>

#include "../../include/dop.h"
#include "dop_internal.h"

namespace dop {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kProbeThreads = 256;
constexpr int kProbeUnroll = 4;
constexpr unsigned kProbeBlocks = 8192;  // 32 per CU

// Read every vector; the sum is stored only if it equals `never` (a NaN the
// host passes, which compares unequal to everything), so the loads stay but
// nothing is written.
__global__ __launch_bounds__(kProbeThreads) void k_probe_read(const v4f *__restrict__ src, size_t n,
                                                              float never, v4f *__restrict__ sink) {
  v4f acc = {0.f, 0.f, 0.f, 0.f};
  const size_t stride = (size_t)gridDim.x * kProbeThreads;
  size_t i = (size_t)blockIdx.x * kProbeThreads + threadIdx.x;
  for (; i + (kProbeUnroll - 1) * stride < n; i += kProbeUnroll * stride) {
    v4f r[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) r[u] = __builtin_nontemporal_load(&src[i + u * stride]);
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) acc += r[u];
  }
  for (; i < n; i += stride) acc += __builtin_nontemporal_load(&src[i]);
  if (acc.x + acc.y + acc.z + acc.w == never) sink[threadIdx.x] = acc;
}

__global__ __launch_bounds__(kProbeThreads) void k_probe_write(v4f *__restrict__ dst, size_t n,
                                                               float value) {
  const v4f v = {value, value, value, value};
  const size_t stride = (size_t)gridDim.x * kProbeThreads;
  for (size_t i = (size_t)blockIdx.x * kProbeThreads + threadIdx.x; i < n; i += stride)
    __builtin_nontemporal_store(v, &dst[i]);
}

__global__ __launch_bounds__(kProbeThreads) void k_probe_copy(const v4f *__restrict__ src,
                                                              v4f *__restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * kProbeThreads;
  size_t i = (size_t)blockIdx.x * kProbeThreads + threadIdx.x;
  for (; i + (kProbeUnroll - 1) * stride < n; i += kProbeUnroll * stride) {
    v4f r[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) r[u] = __builtin_nontemporal_load(&src[i + u * stride]);
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) __builtin_nontemporal_store(r[u], &dst[i + u * stride]);
  }
  for (; i < n; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(&src[i]), &dst[i]);
}

// In place: every vector read and written back times `scale` (a run-time
// value, so the store is not a no-op the compiler could drop).
__global__ __launch_bounds__(kProbeThreads) void k_probe_inplace(v4f *__restrict__ buf, size_t n,
                                                                 float scale) {
  const size_t stride = (size_t)gridDim.x * kProbeThreads;
  size_t i = (size_t)blockIdx.x * kProbeThreads + threadIdx.x;
  for (; i + (kProbeUnroll - 1) * stride < n; i += kProbeUnroll * stride) {
    v4f r[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) r[u] = __builtin_nontemporal_load(&buf[i + u * stride]);
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u)
      __builtin_nontemporal_store(r[u] * scale, &buf[i + u * stride]);
  }
  for (; i < n; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(&buf[i]) * scale, &buf[i]);
}

hipError_t launch_probe_stream(int kind, void *buf, size_t n16, float scale, hipStream_t s) {
  v4f *b = static_cast<v4f *>(buf);
  const dim3 grid(kProbeBlocks), block(kProbeThreads);
  switch (kind) {
    case DOP_PROBE_READ:
      // the sink is the buffer's first vectors (never written in practice)
      hipLaunchKernelGGL(k_probe_read, grid, block, 0, s, b, n16, __builtin_nanf(""), b);
      break;
    case DOP_PROBE_WRITE: hipLaunchKernelGGL(k_probe_write, grid, block, 0, s, b, n16, scale); break;
    case DOP_PROBE_COPY:
      hipLaunchKernelGGL(k_probe_copy, grid, block, 0, s, b, b + n16 / 2, n16 / 2);
      break;
    case DOP_PROBE_INPLACE: hipLaunchKernelGGL(k_probe_inplace, grid, block, 0, s, b, n16, scale); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace dop
