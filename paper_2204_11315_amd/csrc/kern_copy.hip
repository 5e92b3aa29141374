// kern_copy.hip -- copy-back of a slab from device memory into pinned host
// memory by a small kernel.
//
// The copy-back of a slab overlaps the kernels of the next one (Fig. 4: copies
// in, kernels, copies out on three streams).  A copy that the runtime turns
// into a full-machine blit kernel occupies every compute unit for the length
// of the PCIe transfer and so stalls the next slab's kernels; this kernel uses
// only a few workgroups (PCIe, not the GPU, limits its rate) and stores
// straight into the mapped host pages, leaving the rest of the chip to the
// decode / stencil / encode kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "oc_kernels.h"

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kBlocks = 32;

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

hipError_t launch_copy_to_host(void *dst, const void *src, size_t bytes, hipStream_t s) {
  if (!bytes) return hipSuccess;
  const uintptr_t a = (uintptr_t)dst | (uintptr_t)src;
  if ((a & 15) == 0) {
    const size_t n16 = bytes / 16;
    if (n16)
      hipLaunchKernelGGL(k_copy16, dim3(kBlocks), dim3(kThreads), 0, s, (u32x4 *)dst,
                         (const u32x4 *)src, n16);
    const size_t done = n16 * 16;
    if (done < bytes)
      hipLaunchKernelGGL(k_copy1, dim3(1), dim3(kThreads), 0, s, (uint8_t *)dst + done,
                         (const uint8_t *)src + done, bytes - done);
  } else if ((a & 3) == 0) {
    const size_t n4 = bytes / 4;
    if (n4)
      hipLaunchKernelGGL(k_copy4, dim3(kBlocks), dim3(kThreads), 0, s, (uint32_t *)dst,
                         (const uint32_t *)src, n4);
    const size_t done = n4 * 4;
    if (done < bytes)
      hipLaunchKernelGGL(k_copy1, dim3(1), dim3(kThreads), 0, s, (uint8_t *)dst + done,
                         (const uint8_t *)src + done, bytes - done);
  } else {
    hipLaunchKernelGGL(k_copy1, dim3(kBlocks), dim3(kThreads), 0, s, (uint8_t *)dst,
                       (const uint8_t *)src, bytes);
  }
  return hipGetLastError();
}

}  // namespace oc
