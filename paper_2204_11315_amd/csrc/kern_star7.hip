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

// One cell update in a fixed operation order, shared by every kernel here so
// that fused and single-step launches give bit-identical results.
__device__ __forceinline__ float star7_point(float c0, float cur, float xm, float xp, float ym,
                                             float yp, float zm, float zp, const oc::Star7Coef &c) {
  float r = c0 * cur;
  r = fmaf(c.cmx, xm, r);
  r = fmaf(c.cpx, xp, r);
  r = fmaf(c.cmy, ym, r);
  r = fmaf(c.cpy, yp, r);
  r = fmaf(c.cmz, zm, r);
  r = fmaf(c.cpz, zp, r);
  return r;
}

// XCD-aware tile number of workgroup b among nb tiles: workgroup b runs on
// XCD b % 8; each XCD gets a contiguous run of tiles.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int per = (nb + NXCD - 1) / NXCD;
  const int xcd = b % NXCD, slot = b / NXCD;
  const int rem = nb % NXCD;
  const int base = rem == 0 || xcd < rem ? xcd * per : rem * per + (xcd - rem) * (per - 1);
  return base + slot;
}

template <bool FIELD>
__global__ __launch_bounds__(TX *TY) void k_star7(const float *__restrict__ in, float *__restrict__ out,
                                                  const float *__restrict__ c0f, int nx, int ny,
                                                  int z_lo, int z_hi, int gz0, int nz, int nbx,
                                                  int nby, int nbz, oc::Star7Coef c) {
  // tile order: x fastest, then y, then z-chunk
  const int nb = nbx * nby * nbz;
  const int t = xcd_tile(blockIdx.x, nb);
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
    out[col + o] = star7_point(c0, cur, xm, xp, ym, yp, below, above, c);
    below = cur;
    cur = above;
  }
}

// ---- K fused time steps (temporal blocking inside one launch) --------------
// A 64x16 workgroup loads a 64x16 column region and marches z; level s
// (s = 1..K) of the region is computed one plane behind level s-1, from
// level s-1's three newest planes (registers) and its previous plane's xy
// neighbours (LDS, double-buffered by plane parity, one barrier per plane).
// The valid area shrinks by one column per level, so the (64-2K) x (16-2K)
// centre of the region is written at level K.  Only level 0 is read from and
// level K written to memory: 2 passes instead of 2K.
constexpr int FX = 64, FY = 16, FZC = 32;

template <int K, bool FIELD>
__global__ __launch_bounds__(FX *FY) void k_star7_multi(const float *__restrict__ in, float *__restrict__ out,
                                                       const float *__restrict__ c0f, int nx, int ny,
                                                       int zo_lo, int zo_hi, int gz0, int nz, int nbx,
                                                       int nby, int nbz, oc::Star7Coef c) {
  constexpr int OX = FX - 2 * K, OY = FY - 2 * K;
  __shared__ float lds[2][K][FY][FX];
  const int nb = nbx * nby * nbz;
  const int t = xcd_tile(blockIdx.x, nb);
  if (t >= nb) return;   // uniform across the workgroup
  const int tbx = t % nbx, tby = (t / nbx) % nby, tbz = t / (nbx * nby);
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int x = tbx * OX - K + tx;
  const int y = tby * OY - K + ty;
  const bool col_in = x >= 0 && x < nx && y >= 0 && y < ny;
  const bool col_out = tx >= K && tx < K + OX && ty >= K && ty < K + OY && col_in;
  const int zlo = zo_lo + tbz * FZC;
  const int zhi = min(zlo + FZC, zo_hi);
  const size_t plane = (size_t)nx * (size_t)ny;
  const ptrdiff_t col = (ptrdiff_t)y * nx + x;
  const int txm = max(tx - 1, 0), txp = min(tx + 1, FX - 1);
  const int tym = max(ty - 1, 0), typ = min(ty + 1, FY - 1);
  // w[s][0..2]: level s at planes (p-2, p-1, p), p = newest plane of level s
  float w[K + 1][3];
#pragma unroll
  for (int s = 0; s <= K; s++) w[s][0] = w[s][1] = w[s][2] = 0.0f;
  for (int z = zlo - K; z < zhi + K; z++) {
    const int par = z & 1;
    // level 0: plane z
    {
      const bool in_d = col_in && gz0 + z >= 0 && gz0 + z < nz;
      const float v = in_d ? in[(ptrdiff_t)z * (ptrdiff_t)plane + col] : 0.0f;
      w[0][0] = w[0][1];
      w[0][1] = w[0][2];
      w[0][2] = v;
    }
#pragma unroll
    for (int s = 1; s <= K; s++) {
      const int p = z - s;   // plane of level s computed now
      const bool in_d = col_in && gz0 + p >= 0 && gz0 + p < nz;
      float v = 0.0f;
      if (in_d) {
        const float (*L)[FX] = lds[par ^ 1][s - 1];   // level s-1 at plane p
        const float c0 = FIELD ? c0f[(ptrdiff_t)p * (ptrdiff_t)plane + col] : c.c0;
        v = star7_point(c0, w[s - 1][1], L[ty][txm], L[ty][txp], L[tym][tx], L[typ][tx],
                        w[s - 1][0], w[s - 1][2], c);
      }
      w[s][0] = w[s][1];
      w[s][1] = w[s][2];
      w[s][2] = v;
    }
    // publish this plane of levels 0..K-1 for the next plane's neighbours
#pragma unroll
    for (int s = 0; s < K; s++) lds[par][s][ty][tx] = w[s][2];
    const int po = z - K;
    if (col_out && po >= zlo && po < zhi)
      out[(ptrdiff_t)po * (ptrdiff_t)plane + col] = w[K][2];
    __syncthreads();
  }
}

template <int K>
hipError_t launch_multi(const float *in, float *out, const float *c0f, int64_t nx, int64_t ny,
                        int64_t zo_lo, int64_t zo_hi, int64_t gz0, int64_t nz, const oc::Star7Coef &c,
                        hipStream_t s, oc::KernelTimer *kt) {
  constexpr int OX = FX - 2 * K, OY = FY - 2 * K;
  const int nbx = (int)((nx + OX - 1) / OX);
  const int nby = (int)((ny + OY - 1) / OY);
  const int nbz = (int)((zo_hi - zo_lo + FZC - 1) / FZC);
  const int64_t nb = (int64_t)nbx * nby * nbz;
  if (nb > 0x7fffffff) return hipErrorInvalidValue;
  if (c0f)
    hipExtLaunchKernelGGL((k_star7_multi<K, true>), dim3((unsigned)nb), dim3(FX, FY), 0, s, oc::kt_start(kt),
                          oc::kt_stop(kt), 0, in, out, c0f,
                       (int)nx, (int)ny, (int)zo_lo, (int)zo_hi, (int)gz0, (int)nz, nbx, nby, nbz, c);
  else
    hipExtLaunchKernelGGL((k_star7_multi<K, false>), dim3((unsigned)nb), dim3(FX, FY), 0, s, oc::kt_start(kt),
                          oc::kt_stop(kt), 0, in, out, c0f,
                       (int)nx, (int)ny, (int)zo_lo, (int)zo_hi, (int)gz0, (int)nz, nbx, nby, nbz, c);
  return hipGetLastError();
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

hipError_t launch_star7_multi(const float *in, float *out, const float *c0f, int64_t nx, int64_t ny,
                              int64_t zo_lo, int64_t zo_hi, int64_t gz0, int64_t nz, int levels,
                              const Star7Coef &c, hipStream_t s, KernelTimer *kt) {
  if (zo_hi <= zo_lo) return hipSuccess;
  switch (levels) {
    case 1: return launch_multi<1>(in, out, c0f, nx, ny, zo_lo, zo_hi, gz0, nz, c, s, kt);
    case 2: return launch_multi<2>(in, out, c0f, nx, ny, zo_lo, zo_hi, gz0, nz, c, s, kt);
    case 3: return launch_multi<3>(in, out, c0f, nx, ny, zo_lo, zo_hi, gz0, nz, c, s, kt);
    case 4: return launch_multi<4>(in, out, c0f, nx, ny, zo_lo, zo_hi, gz0, nz, c, s, kt);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_axpy_prod(float *g, const float *a, const float *b, size_t n, hipStream_t s,
                            KernelTimer *kt) {
  if (!n) return hipSuccess;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
  hipExtLaunchKernelGGL(k_axpy_prod, dim3((unsigned)blocks), dim3(256), 0, s, kt_start(kt), kt_stop(kt), 0,
                        g, a, b, n);
  return hipGetLastError();
}

hipError_t launch_star7(const float *in, float *out, const float *c0f, int64_t nx, int64_t ny,
                        int64_t z_lo, int64_t z_hi, int64_t gz0, int64_t nz, const Star7Coef &c,
                        hipStream_t s, KernelTimer *kt) {
  if (z_hi <= z_lo) return hipSuccess;
  const int nbx = (int)((nx + TX - 1) / TX);
  const int nby = (int)((ny + TY - 1) / TY);
  const int nbz = (int)((z_hi - z_lo + ZC - 1) / ZC);
  const int64_t nb = (int64_t)nbx * nby * nbz;
  if (nb > 0x7fffffff) return hipErrorInvalidValue;
  dim3 grid((unsigned)nb);
  if (c0f)
    hipExtLaunchKernelGGL(k_star7<true>, grid, dim3(TX, TY), 0, s, kt_start(kt), kt_stop(kt), 0, in, out,
                          c0f, (int)nx, (int)ny,
                       (int)z_lo, (int)z_hi, (int)gz0, (int)nz, nbx, nby, nbz, c);
  else
    hipExtLaunchKernelGGL(k_star7<false>, grid, dim3(TX, TY), 0, s, kt_start(kt), kt_stop(kt), 0, in, out,
                          c0f, (int)nx, (int)ny,
                       (int)z_lo, (int)z_hi, (int)gz0, (int)nz, nbx, nby, nbz, c);
  return hipGetLastError();
}

}  // namespace oc
