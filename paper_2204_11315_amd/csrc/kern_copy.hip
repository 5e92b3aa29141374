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

}  // namespace

namespace oc {

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
