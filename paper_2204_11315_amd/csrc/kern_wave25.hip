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

#ifndef OC_WAVE_TY
#define OC_WAVE_TY 4
#endif
#ifndef OC_WAVE_ZC
#define OC_WAVE_ZC 16
#endif
constexpr int TX = 64, TY = OC_WAVE_TY, ZC = OC_WAVE_ZC, RAD = 4;

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


// The same step with four consecutive x per lane, for rows of whole, 16-byte
// aligned float4s (nx % 4 == 0): a wave covers 256 contiguous x of a row, so
// every load and the store move 1 KiB per instruction, and the x neighbours at
// distance 1..4 come from the lane itself and its two neighbour lanes by DPP
// wave shifts (lane 0's left and lane 63's right four values, in the adjacent
// tiles, by one float4 load each).  The per-cell expression and its operand
// order are those of k_wave25, so the two kernels agree bit for bit.
constexpr int VX = 256;   // x per row of a workgroup (64 lanes x 4)

// DPP wave shifts by one lane; the lane with no source reads zero (bound_ctrl)
__device__ __forceinline__ float lane_from_left(float v) {    // value of lane - 1
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_from_right(float v) {   // value of lane + 1
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ float4 ld4(const float *p) { return *reinterpret_cast<const float4 *>(p); }
__device__ __forceinline__ void unpack(const float4 &v, float *a) {
  a[0] = v.x;
  a[1] = v.y;
  a[2] = v.z;
  a[3] = v.w;
}

__global__ __launch_bounds__(64 * TY) void k_wave25_x4(const float *__restrict__ pn, float *__restrict__ pnm1,
                                                      const float *__restrict__ vel, int nx, int ny,
                                                      int z_lo, int z_hi, int gz0, int nz, float dt_h,
                                                      int sx, int sy, int sz, float src_amp) {
  const int lane = (int)threadIdx.x;
  const int x0 = (int)blockIdx.x * VX + 4 * lane;
  const int y = (int)blockIdx.y * TY + (int)threadIdx.y;
  // a wave is one row: y is uniform across it; a lane's four x are all inside
  // or all outside the grid.  Every lane takes part in the shifts.
  const bool act = x0 < nx && y < ny;
  const int zb = z_lo + (int)blockIdx.z * ZC;
  const int ze = min(zb + ZC, z_hi);
  const ptrdiff_t plane = (ptrdiff_t)nx * (ptrdiff_t)ny;
  const ptrdiff_t col = (ptrdiff_t)y * nx + x0;
  const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
  // z window: w[j] = p^n at local plane z - 4 + j
  float4 w[2 * RAD + 1];
#pragma unroll
  for (int j = 0; j < 2 * RAD; j++) {
    const int z = zb - RAD + j;
    const bool in = act && gz0 + z >= 0 && gz0 + z < nz;
    w[j] = in ? ld4(pn + (ptrdiff_t)z * plane + col) : zero;
  }
  for (int z = zb; z < ze; z++) {
    {
      const int zt = z + RAD;
      const bool in = act && gz0 + zt >= 0 && gz0 + zt < nz;
      w[2 * RAD] = in ? ld4(pn + (ptrdiff_t)zt * plane + col) : zero;
    }
    const ptrdiff_t o = (ptrdiff_t)z * plane + col;
    const float4 c = w[RAD];
    float4 L, R;   // the four x before and the four x after this lane's
    L.x = lane_from_left(c.x);
    L.y = lane_from_left(c.y);
    L.z = lane_from_left(c.z);
    L.w = lane_from_left(c.w);
    R.x = lane_from_right(c.x);
    R.y = lane_from_right(c.y);
    R.z = lane_from_right(c.z);
    R.w = lane_from_right(c.w);
    if (lane == 0) L = (act && x0 > 0) ? ld4(pn + o - 4) : zero;
    if (lane == 63 || x0 + 4 >= nx) R = (act && x0 + 4 < nx) ? ld4(pn + o + 4) : zero;
    float xs[12], ym[RAD][4], yp[RAD][4], zm[RAD][4], zp[RAD][4], pm[4], vv[4];
    unpack(L, xs);
    unpack(c, xs + 4);
    unpack(R, xs + 8);
#pragma unroll
    for (int d = 1; d <= RAD; d++) {
      unpack((act && y >= d) ? ld4(pn + o - (ptrdiff_t)d * nx) : zero, ym[d - 1]);
      unpack((act && y + d < ny) ? ld4(pn + o + (ptrdiff_t)d * nx) : zero, yp[d - 1]);
      unpack(w[RAD - d], zm[d - 1]);
      unpack(w[RAD + d], zp[d - 1]);
    }
    unpack(act ? ld4(pnm1 + o) : zero, pm);
    unpack(act ? ld4(vel + o) : zero, vv);
    float res[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const float cc = xs[4 + i];
      float sxd[RAD], syd[RAD];
#pragma unroll
      for (int d = 1; d <= RAD; d++) {
        sxd[d - 1] = xs[4 + i - d] + xs[4 + i + d];
        syd[d - 1] = ym[d - 1][i] + yp[d - 1][i];
      }
      const float lap = 3.0f * W0 * cc + W1 * (sxd[0] + syd[0] + (zm[0][i] + zp[0][i])) +
                        W2 * (sxd[1] + syd[1] + (zm[1][i] + zp[1][i])) +
                        W3 * (sxd[2] + syd[2] + (zm[2][i] + zp[2][i])) +
                        W4 * (sxd[3] + syd[3] + (zm[3][i] + zp[3][i]));
      const float a = vv[i] * dt_h;
      const float a2 = a * a;
      float nv = 2.0f * cc - pm[i] + a2 * lap;
      if (x0 + i == sx && y == sy && gz0 + z == sz) nv += a2 * src_amp;
      res[i] = nv;
    }
    if (act) *reinterpret_cast<float4 *>(pnm1 + o) = make_float4(res[0], res[1], res[2], res[3]);
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
  const uintptr_t align = (uintptr_t)pn | (uintptr_t)pnm1 | (uintptr_t)vel;
  if (nx % 4 == 0 && align % 16 == 0) {   // rows of whole float4s
    dim3 grid4((unsigned)((nx + VX - 1) / VX), (unsigned)((ny + TY - 1) / TY),
               (unsigned)((z_hi - z_lo + ZC - 1) / ZC));
    hipExtLaunchKernelGGL(k_wave25_x4, grid4, dim3(64, TY), 0, s, kt_start(kt), kt_stop(kt), 0, pn, pnm1, vel,
                          (int)nx, (int)ny, (int)z_lo, (int)z_hi, (int)gz0, (int)nz, dt_h,
                          has_src ? (int)src[0] : -1, has_src ? (int)src[1] : -1,
                          has_src ? (int)src[2] : -1, src_amp);
    return hipGetLastError();
  }
  hipExtLaunchKernelGGL(k_wave25, grid, dim3(TX, TY), 0, s, kt_start(kt), kt_stop(kt), 0, pn, pnm1, vel,
                        (int)nx, (int)ny, (int)z_lo,
                     (int)z_hi, (int)gz0, (int)nz, dt_h, has_src ? (int)src[0] : -1,
                     has_src ? (int)src[1] : -1, has_src ? (int)src[2] : -1, src_amp);
  return hipGetLastError();
}

}  // namespace oc
