// kern_star7.hip -- 7-point star stencil step on gfx950.
//
// The stencil update of Sec. 3.1: every point is recomputed from itself and
// its six face neighbours, zero outside the grid.  Within a resident slab the
// same kernel is applied k times on a shrinking range of planes (temporal
// blocking, Sec. 3.1), so one launch updates local planes [z_lo, z_hi) of a
// slab buffer whose local plane 0 is global plane gz0.
//
// Layout: a 64x4 workgroup owns a 64x4 column tile and marches it through a
// chunk of planes.  Each lane keeps its (z-1, z, z+1) values in registers, so
// every input plane is loaded once per lane (plus the x/y neighbours, which
// hit the same cache lines as the neighbouring lanes' own loads).  A wave's
// 64 lanes cover 256 contiguous bytes of a row, so every load and store is one
// coalesced transaction.  Bandwidth bound: 8 bytes of HBM traffic per cell
// update (one read, one write) against 13 flops.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "oc_kernels.h"

namespace {

constexpr int TX = 64, TY = 4, ZC = 8;

template <bool FIELD>
__global__ __launch_bounds__(TX *TY) void k_star7(const float *__restrict__ in, float *__restrict__ out,
                                                  const float *__restrict__ c0f, int nx, int ny,
                                                  int z_lo, int z_hi, int gz0, int nz,
                                                  oc::Star7Coef c) {
  const int x = blockIdx.x * TX + threadIdx.x;
  const int y = blockIdx.y * TY + threadIdx.y;
  if (x >= nx || y >= ny) return;
  const int zb = z_lo + blockIdx.z * ZC;
  const int ze = min(zb + ZC, z_hi);
  const size_t plane = (size_t)nx * (size_t)ny;
  const size_t col = (size_t)y * nx + x;
  const float *p = in + col;
  float below = (gz0 + zb - 1 >= 0) ? p[(size_t)(zb - 1) * plane] : 0.0f;
  float cur = p[(size_t)zb * plane];
  for (int z = zb; z < ze; z++) {
    const size_t o = (size_t)z * plane;
    const float *q = p + o;
    const float above = (gz0 + z + 1 < nz) ? q[plane] : 0.0f;
    const float xm = x > 0 ? q[-1] : 0.0f;
    const float xp = x + 1 < nx ? q[1] : 0.0f;
    const float ym = y > 0 ? q[-(ptrdiff_t)nx] : 0.0f;
    const float yp = y + 1 < ny ? q[nx] : 0.0f;
    const float c0 = FIELD ? c0f[col + o] : c.c0;
    out[col + o] = c0 * cur + c.cmx * xm + c.cpx * xp + c.cmy * ym + c.cpy * yp + c.cmz * below +
                   c.cpz * above;
    below = cur;
    cur = above;
  }
}

}  // namespace

namespace oc {

hipError_t launch_star7(const float *in, float *out, const float *c0f, int64_t nx, int64_t ny,
                        int64_t z_lo, int64_t z_hi, int64_t gz0, int64_t nz, const Star7Coef &c,
                        hipStream_t s) {
  if (z_hi <= z_lo) return hipSuccess;
  dim3 grid((unsigned)((nx + TX - 1) / TX), (unsigned)((ny + TY - 1) / TY),
            (unsigned)((z_hi - z_lo + ZC - 1) / ZC));
  if (c0f)
    hipLaunchKernelGGL(k_star7<true>, grid, dim3(TX, TY), 0, s, in, out, c0f, (int)nx, (int)ny,
                       (int)z_lo, (int)z_hi, (int)gz0, (int)nz, c);
  else
    hipLaunchKernelGGL(k_star7<false>, grid, dim3(TX, TY), 0, s, in, out, c0f, (int)nx, (int)ny,
                       (int)z_lo, (int)z_hi, (int)gz0, (int)nz, c);
  return hipGetLastError();
}

}  // namespace oc
