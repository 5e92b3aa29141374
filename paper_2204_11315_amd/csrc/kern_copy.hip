// kern_copy.hip -- copy-back of a slab from device memory into pinned host
// memory by a small kernel.
//
// The copy-back of a slab overlaps the kernels of the next one (Fig. 4: copies
// in, kernels, copies out on three streams).  A copy that the runtime turns
// into a full-machine blit kernel occupies every compute unit for the length
// of the PCIe transfer and so stalls the next slab's kernels; this kernel uses
// only a few workgroups and stores straight into the mapped host pages.
//
// Stores to host memory still share the chip's memory write path with the
// kernels that overlap them: while they are in flight, write-heavy kernels
// (decode, stencil) slow down roughly in proportion to the number of copy
// workgroups.  Each workgroup sustains about 10 GB/s to host memory, so four
// of them (about 40 GB/s, near the link's rate with traffic in both
// directions) balance the copy-back against the kernels it overlaps.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "oc_kernels.h"

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kDefaultBlocks = 4;

__global__ __launch_bounds__(kThreads) void k_copy16(u32x4 *__restrict__ dst,
                                                     const u32x4 *__restrict__ src, size_t n) {
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads)
    __builtin_nontemporal_store(src[i], &dst[i]);
}

__global__ __launch_bounds__(kThreads) void k_copy4(uint32_t *__restrict__ dst,
                                                    const uint32_t *__restrict__ src, size_t n) {
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads)
    __builtin_nontemporal_store(src[i], &dst[i]);
}

__global__ __launch_bounds__(kThreads) void k_copy1(uint8_t *__restrict__ dst,
                                                    const uint8_t *__restrict__ src, size_t n) {
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads)
    dst[i] = src[i];
}

// Start and end of the two probe kernels on the device's constant-rate clock.
__device__ unsigned long long g_probe_clock[4];

// One wave that runs for `ticks` of the constant-rate clock (at most 2^24
// clock reads) and records its start and end in slot `slot`: two of them on
// two streams show whether the streams run their kernels side by side.
__global__ __launch_bounds__(64) void k_busy(int slot, unsigned long long ticks) {
  const unsigned long long t0 = wall_clock64();
  unsigned long long t = t0;
  for (int i = 0; i < (1 << 24) && t - t0 < ticks; i++) t = wall_clock64();
  if (threadIdx.x == 0) {
    g_probe_clock[2 * slot] = t0;
    g_probe_clock[2 * slot + 1] = t;
  }
}

}  // namespace

namespace oc {

hipError_t probe_stream_overlap(hipStream_t a, hipStream_t b, double *overlap) {
  int dev = 0, khz = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
  if (e != hipSuccess) return e;
  if (khz <= 0) return hipErrorInvalidValue;
  const unsigned long long ticks = (unsigned long long)khz * 2;   // 2 ms
  // first launches on each stream carry one-time costs (code object, queue)
  for (int pass = 0; pass < 2; pass++) {
    hipLaunchKernelGGL(k_busy, dim3(1), dim3(64), 0, a, 0, pass ? ticks : ticks / 20);
    hipLaunchKernelGGL(k_busy, dim3(1), dim3(64), 0, b, 1, pass ? ticks : ticks / 20);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(a);
    if (e == hipSuccess) e = hipStreamSynchronize(b);
    if (e != hipSuccess) return e;
  }
  unsigned long long c[4] = {};
  e = hipMemcpyFromSymbolAsync(c, HIP_SYMBOL(g_probe_clock), sizeof(c), 0, hipMemcpyDeviceToHost, a);
  if (e == hipSuccess) e = hipStreamSynchronize(a);
  if (e != hipSuccess) return e;
  const double lo = (double)std::max(c[0], c[2]), hi = (double)std::min(c[1], c[3]);
  const double shorter = (double)std::min(c[1] - c[0], c[3] - c[2]);
  *overlap = shorter > 0 ? std::max(0.0, hi - lo) / shorter : 0.0;
  return hipSuccess;
}

hipError_t launch_copy_to_host(void *dst, const void *src, size_t bytes, int workgroups, hipStream_t s,
                               KernelTimer *kt) {
  if (!bytes) return hipSuccess;
  const int kBlocks = workgroups < 1 ? kDefaultBlocks : (workgroups > 1024 ? 1024 : workgroups);
  const uintptr_t a = (uintptr_t)dst | (uintptr_t)src;
  // widest aligned body, then a byte tail; the timer spans both
  const size_t unit = (a & 15) == 0 ? 16 : ((a & 3) == 0 ? 4 : 1);
  const size_t n = bytes / unit, done = n * unit;
  const bool tail = done < bytes;
  if (n) {
    hipEvent_t e0 = kt_start(kt), e1 = tail ? nullptr : kt_stop(kt);
    if (unit == 16)
      hipExtLaunchKernelGGL(k_copy16, dim3(kBlocks), dim3(kThreads), 0, s, e0, e1, 0, (u32x4 *)dst,
                            (const u32x4 *)src, n);
    else if (unit == 4)
      hipExtLaunchKernelGGL(k_copy4, dim3(kBlocks), dim3(kThreads), 0, s, e0, e1, 0, (uint32_t *)dst,
                            (const uint32_t *)src, n);
    else
      hipExtLaunchKernelGGL(k_copy1, dim3(kBlocks), dim3(kThreads), 0, s, e0, e1, 0, (uint8_t *)dst,
                            (const uint8_t *)src, n);
  }
  if (tail) {
    hipEvent_t e0 = n ? nullptr : kt_start(kt);
    hipExtLaunchKernelGGL(k_copy1, dim3(1), dim3(kThreads), 0, s, e0, kt_stop(kt), 0, (uint8_t *)dst + done,
                          (const uint8_t *)src + done, bytes - done);
  }
  return hipGetLastError();
}

}  // namespace oc
