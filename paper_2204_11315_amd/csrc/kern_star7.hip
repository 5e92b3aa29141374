// kern_star7.hip -- 7-point star stencil step on gfx950.
//
// The stencil update of Sec. 3.1: every point is recomputed from itself and
// its six face neighbours, zero outside the grid.  Within a resident slab the
// same kernel is applied k times on a shrinking range of planes (temporal
// blocking, Sec. 3.1), so one launch updates local planes [z_lo, z_hi) of a
// slab buffer whose local plane 0 is global plane gz0.
//
// Layout: a 64x4 workgroup owns a 64x4 column tile and marches a chunk of ZC
// planes.  Each lane keeps its (z-1, z, z+1) values in registers, so every
// input plane is loaded once per lane plus the x/y neighbours, which hit the
// cache lines of the neighbouring lanes' and rows' own loads.  A wave's 64
// lanes cover 256 contiguous bytes of a row (one coalesced transaction).
// Workgroups are numbered so that each XCD (and so each L2) receives a
// contiguous run of tiles in y, so halo rows shared by neighbouring tiles are
// fetched from HBM once per XCD rather than once per tile.
// Bandwidth bound: 8 bytes of HBM traffic per cell update against 13 flops.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "oc_kernels.h"

namespace {

constexpr int TX = 64, TY = 4, ZC = 16;
constexpr int NXCD = 8;    // XCDs on MI355X: workgroups are dealt to them round-robin

template <bool FIELD>
__global__ __launch_bounds__(TX *TY) void k_star7(const float *__restrict__ in, float *__restrict__ out,
                                                  const float *__restrict__ c0f, int nx, int ny,
                                                  int z_lo, int z_hi, int gz0, int nz, int nbx,
                                                  int nby, int nbz, oc::Star7Coef c) {
  // XCD-aware numbering: workgroup b runs on XCD b % 8; give each XCD a
  // contiguous range of tiles (tile order: x fastest, then y, then z-chunk).
  const int nb = nbx * nby * nbz;
  const int b = blockIdx.x;
  const int per = (nb + NXCD - 1) / NXCD;
  const int xcd = b % NXCD, slot = b / NXCD;
  // XCDs with id < nb % 8 (or all, when divisible) own `per` tiles, the rest per-1
  const int rem = nb % NXCD;
  const int base = rem == 0 || xcd < rem ? xcd * per : rem * per + (xcd - rem) * (per - 1);
  const int t = base + slot;
  if (t >= nb) return;
  const int tbx = t % nbx;
  const int tby = (t / nbx) % nby;
  const int tbz = t / (nbx * nby);

  const int x = tbx * TX + (int)threadIdx.x;
  const int y = tby * TY + (int)threadIdx.y;
  if (x >= nx || y >= ny) return;
  const int zb = z_lo + tbz * ZC;
  const int ze = min(zb + ZC, z_hi);
  const size_t plane = (size_t)nx * (size_t)ny;
  const size_t col = (size_t)y * nx + x;
  const float *p = in + col;
  float below = (gz0 + zb - 1 >= 0) ? p[(ptrdiff_t)(zb - 1) * (ptrdiff_t)plane] : 0.0f;
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

// g[i] += a[i] * b[i]: the per-cell coefficient-gradient accumulation of the
// adjoint, dL/dc0(x) += lambda_{n+1}(x) u_n(x).
__global__ __launch_bounds__(256) void k_axpy_prod(float *__restrict__ g, const float *__restrict__ a,
                                                   const float *__restrict__ b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    g[i] = fmaf(a[i], b[i], g[i]);
}

}  // namespace

namespace oc {

hipError_t launch_axpy_prod(float *g, const float *a, const float *b, size_t n, hipStream_t s) {
  if (!n) return hipSuccess;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_axpy_prod, dim3((unsigned)blocks), dim3(256), 0, s, g, a, b, n);
  return hipGetLastError();
}

hipError_t launch_star7(const float *in, float *out, const float *c0f, int64_t nx, int64_t ny,
                        int64_t z_lo, int64_t z_hi, int64_t gz0, int64_t nz, const Star7Coef &c,
                        hipStream_t s) {
  if (z_hi <= z_lo) return hipSuccess;
  const int nbx = (int)((nx + TX - 1) / TX);
  const int nby = (int)((ny + TY - 1) / TY);
  const int nbz = (int)((z_hi - z_lo + ZC - 1) / ZC);
  const int64_t nb = (int64_t)nbx * nby * nbz;
  if (nb > 0x7fffffff) return hipErrorInvalidValue;
  dim3 grid((unsigned)nb);
  if (c0f)
    hipLaunchKernelGGL(k_star7<true>, grid, dim3(TX, TY), 0, s, in, out, c0f, (int)nx, (int)ny,
                       (int)z_lo, (int)z_hi, (int)gz0, (int)nz, nbx, nby, nbz, c);
  else
    hipLaunchKernelGGL(k_star7<false>, grid, dim3(TX, TY), 0, s, in, out, c0f, (int)nx, (int)ny,
                       (int)z_lo, (int)z_hi, (int)gz0, (int)nz, nbx, nby, nbz, c);
  return hipGetLastError();
}

}  // namespace oc
