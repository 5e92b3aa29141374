// kern_wave25.hip -- 25-point (order-8 star) acoustic wave step on gfx950.
//
// The workload of Sec. 6 (Table 1): an acoustic wave propagation code with a
// 25-point stencil and a 4-cell halo.  One leapfrog step
//   p^{n+1} = 2 p^n - p^{n-1} + (v dt / h)^2 L8(p^n)   (+ Ricker source term)
// with L8 the eighth-order central second derivative summed over x, y, z.  The
// new level is written over p^{n-1} in place (each cell reads p^{n-1} only at
// its own position), so the three read-only / read-write datasets of the
// paper's accounting (Sec. 6.2: velocity, two pressure levels) need no fourth
// write-only buffer.  Zero outside the grid.
//
// Layout: a 64x4 workgroup owns a 64x4 column tile and marches a chunk of
// planes, keeping the nine z-values (z-4 .. z+4) of its column in registers;
// x- and y-neighbours are read from global memory (the neighbouring lanes'
// and rows' own loads, so cache hits).  Bandwidth bound: 16 bytes of HBM
// traffic per cell update (read p^n, p^{n-1}, v; write p^{n+1}).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "oc_kernels.h"

namespace {

constexpr int TX = 64, TY = 4, ZC = 16, RAD = 4;

// eighth-order central second-derivative weights (centre, then offsets 1..4)
constexpr float W0 = -205.0f / 72.0f, W1 = 8.0f / 5.0f, W2 = -1.0f / 5.0f, W3 = 8.0f / 315.0f,
                W4 = -1.0f / 560.0f;

__global__ __launch_bounds__(TX *TY) void k_wave25(const float *__restrict__ pn, float *__restrict__ pnm1,
                                                   const float *__restrict__ vel, int nx, int ny,
                                                   int z_lo, int z_hi, int gz0, int nz, float dt_h,
                                                   int sx, int sy, int sz, float src_amp) {
  const int x = blockIdx.x * TX + threadIdx.x;
  const int y = blockIdx.y * TY + threadIdx.y;
  if (x >= nx || y >= ny) return;
  const int zb = z_lo + blockIdx.z * ZC;
  const int ze = min(zb + ZC, z_hi);
  const size_t plane = (size_t)nx * (size_t)ny;
  const size_t col = (size_t)y * nx + x;
  // z window: w[j] = p^n at local plane z - 4 + j
  float w[2 * RAD + 1];
#pragma unroll
  for (int j = 0; j < 2 * RAD; j++) {
    const int z = zb - RAD + j;
    const bool in = gz0 + z >= 0 && gz0 + z < nz;
    w[j] = in ? pn[(ptrdiff_t)z * (ptrdiff_t)plane + (ptrdiff_t)col] : 0.0f;
  }
  for (int z = zb; z < ze; z++) {
    {
      const int zt = z + RAD;
      const bool in = gz0 + zt >= 0 && gz0 + zt < nz;
      w[2 * RAD] = in ? pn[(ptrdiff_t)zt * (ptrdiff_t)plane + (ptrdiff_t)col] : 0.0f;
    }
    const float *q = pn + (size_t)z * plane + col;
    float sx1 = 0.f, sx2 = 0.f, sx3 = 0.f, sx4 = 0.f;   // pairs at distance 1..4 in x
    float sy1 = 0.f, sy2 = 0.f, sy3 = 0.f, sy4 = 0.f;
    sx1 = (x >= 1 ? q[-1] : 0.f) + (x + 1 < nx ? q[1] : 0.f);
    sx2 = (x >= 2 ? q[-2] : 0.f) + (x + 2 < nx ? q[2] : 0.f);
    sx3 = (x >= 3 ? q[-3] : 0.f) + (x + 3 < nx ? q[3] : 0.f);
    sx4 = (x >= 4 ? q[-4] : 0.f) + (x + 4 < nx ? q[4] : 0.f);
    const ptrdiff_t sn = nx;
    sy1 = (y >= 1 ? q[-sn] : 0.f) + (y + 1 < ny ? q[sn] : 0.f);
    sy2 = (y >= 2 ? q[-2 * sn] : 0.f) + (y + 2 < ny ? q[2 * sn] : 0.f);
    sy3 = (y >= 3 ? q[-3 * sn] : 0.f) + (y + 3 < ny ? q[3 * sn] : 0.f);
    sy4 = (y >= 4 ? q[-4 * sn] : 0.f) + (y + 4 < ny ? q[4 * sn] : 0.f);
    const float c = w[RAD];
    const float lap = 3.0f * W0 * c + W1 * (sx1 + sy1 + (w[RAD - 1] + w[RAD + 1])) +
                      W2 * (sx2 + sy2 + (w[RAD - 2] + w[RAD + 2])) +
                      W3 * (sx3 + sy3 + (w[RAD - 3] + w[RAD + 3])) +
                      W4 * (sx4 + sy4 + (w[RAD - 4] + w[RAD + 4]));
    const size_t i = (size_t)z * plane + col;
    const float a = vel[i] * dt_h;
    const float a2 = a * a;
    float nv = 2.0f * c - pnm1[i] + a2 * lap;
    if (x == sx && y == sy && gz0 + z == sz) nv += a2 * src_amp;
    pnm1[i] = nv;
#pragma unroll
    for (int j = 0; j < 2 * RAD; j++) w[j] = w[j + 1];
  }
}

}  // namespace

namespace oc {

hipError_t launch_wave25(const float *pn, float *pnm1, const float *vel, int64_t nx, int64_t ny,
                         int64_t z_lo, int64_t z_hi, int64_t gz0, int64_t nz, float dt_h,
                         const int64_t *src, float src_amp, hipStream_t s, KernelTimer *kt) {
  if (z_hi <= z_lo) return hipSuccess;
  dim3 grid((unsigned)((nx + TX - 1) / TX), (unsigned)((ny + TY - 1) / TY),
            (unsigned)((z_hi - z_lo + ZC - 1) / ZC));
  const bool has_src = src && src[0] >= 0 && src[0] < nx && src[1] >= 0 && src[1] < ny &&
                       src[2] >= 0 && src[2] < nz;
  hipExtLaunchKernelGGL(k_wave25, grid, dim3(TX, TY), 0, s, kt_start(kt), kt_stop(kt), 0, pn, pnm1, vel,
                        (int)nx, (int)ny, (int)z_lo,
                     (int)z_hi, (int)gz0, (int)nz, dt_h, has_src ? (int)src[0] : -1,
                     has_src ? (int)src[1] : -1, has_src ? (int)src[2] : -1, src_amp);
  return hipGetLastError();
}

}  // namespace oc
