// kern_star7.hip -- 7-point star stencil step on gfx950.
//
// The stencil update of Sec. 3.1: every point is recomputed from itself and
// its six face neighbours, zero outside the grid.  Within a resident slab the
// same kernel is applied k times on a shrinking range of planes (temporal
// blocking, Sec. 3.1), so one launch updates local planes [z_lo, z_hi) of a
// slab buffer whose local plane 0 is global plane gz0.
//
// Layout (rows that are not whole float4s; otherwise k_star7_x4 below, four
// x per lane): a 64x4 workgroup owns a 64x4 column tile and marches a chunk of ZC
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
#include <atomic>

#include "oc_kernels.h"
#include "stencil_dev.h"

namespace {

constexpr int TX = 64, TY = 4, ZC = 16;
constexpr int NXCD = 8;    // XCDs on MI355X: workgroups are dealt to them round-robin

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
// A workgroup of FW waves owns a 64 x (FW*RY) column tile of the xy plane and
// marches z.  Lane l of every wave holds column x = x0 + l; wave w holds the
// RY consecutive rows y0 + w*RY + r in registers.  Level s (s = 1..K) is
// computed one plane behind level s-1: at input plane z, level s produces
// plane z - s from level s-1's planes z-s-1, z-s, z-s+1, which every thread
// keeps in a three-plane register window per level.  Neighbours of the centre
// plane come from:
//   x +- 1: the neighbouring lanes' registers (DPP wave shifts, no memory);
//   y +- 1: the thread's own rows, or, at the strip's first / last row, the
//           adjacent wave's edge row, published in LDS one plane earlier
//           (double-buffered by plane parity: one barrier per plane).
// Every level is valid one column / row further inside the tile than the
// level below it, so the (64 - 2K) x (FW*RY - 2K) centre is written at level
// K.  Cells outside the grid are held at zero at every level (the boundary
// condition).  The per-cell arithmetic is star7_point's, so the result is bit
// identical to K single steps.  The caller guarantees that input planes
// [zo_lo - K, zo_hi + K) lie inside the buffers; no plane outside that range
// is read.
// Five rows per wave: a 40-row tile writes 40 - 2K rows, 32 at K = 4, which
// tiles a 512-row plane exactly (16 tiles; 4 rows gave 24 of 32 and 22 tiles).
constexpr int FW = 8, RY = 5, FTY = FW * RY;

// One 7-point step with four consecutive x per lane, for rows of whole,
// 16-byte aligned float4s (nx % 4 == 0): a wave covers 256 contiguous x of a
// row, so the (z+1, y-1, y+1) loads and the store are 1 KiB per instruction,
// and the x neighbours come from the adjacent lanes by DPP shifts (lane 0's
// left and lane 63's right neighbour, in the adjacent tiles, by single
// loads).  Same per-cell operation order as every other 7-point kernel here.
constexpr int VX = 256;   // x per row of a workgroup (64 lanes x 4)

__device__ __forceinline__ float4 ld4(const float *p) { return *reinterpret_cast<const float4 *>(p); }

template <bool FIELD>
__global__ __launch_bounds__(64 * TY) void k_star7_x4(const float *__restrict__ in, float *__restrict__ out,
                                                      const float *__restrict__ c0f, int nx, int ny,
                                                      int z_lo, int z_hi, int gz0, int nz, int nbx,
                                                      int nby, int nbz, oc::Star7Coef c) {
  const int nb = nbx * nby * nbz;
  const int t = xcd_tile(blockIdx.x, nb);
  if (t >= nb) return;
  const int tbx = t % nbx;
  const int tby = (t / nbx) % nby;
  const int tbz = t / (nbx * nby);
  const int lane = (int)threadIdx.x;
  const int x0 = tbx * VX + 4 * lane;
  const int y = tby * TY + (int)threadIdx.y;
  // a wave is one row: y is uniform across it; a lane's four x are all
  // inside or all outside the grid.  Every lane takes part in the shifts.
  const bool act = x0 < nx && y < ny;
  const int zb = z_lo + tbz * ZC;
  const int ze = min(zb + ZC, z_hi);
  const ptrdiff_t plane = (ptrdiff_t)nx * (ptrdiff_t)ny;
  const ptrdiff_t col = (ptrdiff_t)y * nx + x0;
  const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
  float4 below = (act && gz0 + zb - 1 >= 0) ? ld4(in + col + (ptrdiff_t)(zb - 1) * plane) : zero;
  float4 cur = act ? ld4(in + col + (ptrdiff_t)zb * plane) : zero;
  for (int z = zb; z < ze; z++) {
    const ptrdiff_t o = col + (ptrdiff_t)z * plane;
    const float4 above = (act && gz0 + z + 1 < nz) ? ld4(in + o + plane) : zero;
    const float4 ym = (act && y > 0) ? ld4(in + o - nx) : zero;
    const float4 yp = (act && y + 1 < ny) ? ld4(in + o + nx) : zero;
    float l = lane_from_left(cur.w);
    float r = lane_from_right(cur.x);
    if (lane == 0) l = (act && x0 > 0) ? in[o - 1] : 0.0f;
    if (lane == 63 || x0 + 4 >= nx) r = (act && x0 + 4 < nx) ? in[o + 4] : 0.0f;
    const float4 c0 = FIELD ? (act ? ld4(c0f + o) : zero) : make_float4(c.c0, c.c0, c.c0, c.c0);
    float4 v;
    v.x = star7_point(c0.x, cur.x, l, cur.y, ym.x, yp.x, below.x, above.x, c);
    v.y = star7_point(c0.y, cur.y, cur.x, cur.z, ym.y, yp.y, below.y, above.y, c);
    v.z = star7_point(c0.z, cur.z, cur.y, cur.w, ym.z, yp.z, below.z, above.z, c);
    v.w = star7_point(c0.w, cur.w, cur.z, r, ym.w, yp.w, below.w, above.w, c);
    if (act) *reinterpret_cast<float4 *>(out + o) = v;
    below = cur;
    cur = above;
  }
}

// State of one thread of the fused kernel.  win[s][slot][r] holds level s of
// row r at three consecutive planes in rotating slots: in phase PH (the input
// plane index mod 3) the slot (PH + 2) % 3 holds the oldest plane, which the
// new plane replaces, so the window never moves in registers.
template <int K, bool FIELD>
struct FusedState {
  float win[K][3][RY];
  float cw[K][RY];   // c0 at planes z-1 .. z-K (FIELD)
  bool row_in[RY], row_out[RY];
};

// One input plane z of the fused kernel.  MASK = false is the interior form:
// the workgroup's whole column range and plane range lie inside the grid, so
// no cell needs the zero boundary value.
template <int K, bool FIELD, bool MASK, int PH>
__device__ __forceinline__ void fused_plane(FusedState<K, FIELD> &st, float (*edge)[K][FW][2][64], int z,
                                            const float *__restrict__ in, float *__restrict__ out,
                                            const float *__restrict__ c0f, ptrdiff_t plane, ptrdiff_t col0,
                                            int nx, int gz0, int nz, int zlo, int zhi, int lane, int w,
                                            const oc::Star7Coef &c) {
  // slots in this phase: the new plane goes to N, its two predecessors are in
  // C (one before) and O (two before)
  constexpr int N = (PH + 2) % 3, C = (PH + 1) % 3, O = PH % 3;
  const int par = z & 1;
  {
    // level 0: input plane z (the other resident waves hide its latency;
    // fetching a plane ahead costs registers and so occupancy, and measured
    // slower)
    const bool p_in = !MASK || (gz0 + z >= 0 && gz0 + z < nz);
#pragma unroll
    for (int r = 0; r < RY; r++)
      st.win[0][N][r] = (!MASK || (p_in && st.row_in[r])) ? in[(ptrdiff_t)z * plane + col0 + (ptrdiff_t)r * nx]
                                                          : 0.0f;
  }
  if (FIELD) {
    // c0 at plane z-1; planes below zlo-K+1 are needed by no level (and may
    // lie before the buffer), so they are not read
    const int p = z - 1;
    const bool p_use = p >= zlo - K + 1 && (!MASK || (gz0 + p >= 0 && gz0 + p < nz));
#pragma unroll
    for (int s = K - 1; s > 0; s--)
#pragma unroll
      for (int r = 0; r < RY; r++) st.cw[s][r] = st.cw[s - 1][r];
#pragma unroll
    for (int r = 0; r < RY; r++)
      st.cw[0][r] = (p_use && (!MASK || st.row_in[r])) ? c0f[(ptrdiff_t)p * plane + col0 + (ptrdiff_t)r * nx]
                                                       : 0.0f;
  }
  // the outermost waves read a clamped neighbour: their outer row lies in the
  // tile's invalid border, where any value may go
  const int wu = w > 0 ? w - 1 : 0, wd = w < FW - 1 ? w + 1 : FW - 1;
  // level s makes plane z - s from level s-1's planes z-s-1 (slot O),
  // z-s (slot C) and z-s+1 (slot N, made just now)
#pragma unroll
  for (int s = 1; s <= K; s++) {
    const int p = z - s;
    const bool p_in = !MASK || (gz0 + p >= 0 && gz0 + p < nz);
    const float up = edge[par ^ 1][s - 1][wu][1][lane];
    const float dn = edge[par ^ 1][s - 1][wd][0][lane];
    // star7_point's operation order, with the two x terms as FMAs that read
    // their first operand through a DPP wave shift (lane - 1, lane + 1; zero
    // at the wave's ends), for all RY rows in one block: each row's
    // accumulator is next read RY - 1 instructions after it is written, and
    // the leading s_nop covers the VALU-write-to-DPP-read distance for the
    // accumulators and row values written just before the block
    float v[RY];
#pragma unroll
    for (int r = 0; r < RY; r++) v[r] = (FIELD ? st.cw[s - 1][r] : c.c0) * st.win[s - 1][C][r];
    static_assert(RY == 5, "the DPP block below is written for five rows");
    asm("s_nop 4\n\t"
        "v_fmac_f32_dpp %0, %5, %10 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %6, %10 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %2, %7, %10 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %3, %8, %10 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %4, %9, %10 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %0, %5, %11 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %6, %11 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %2, %7, %11 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %3, %8, %11 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %4, %9, %11 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
        : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4])
        : "v"(st.win[s - 1][C][0]), "v"(st.win[s - 1][C][1]), "v"(st.win[s - 1][C][2]),
          "v"(st.win[s - 1][C][3]), "v"(st.win[s - 1][C][4]), "v"(c.cmx), "v"(c.cpx));
    float nv[RY];
#pragma unroll
    for (int r = 0; r < RY; r++) {
      const float ym = r > 0 ? st.win[s - 1][C][r - 1] : up;
      const float yp = r < RY - 1 ? st.win[s - 1][C][r + 1] : dn;
      float w = fmaf(c.cmy, ym, v[r]);
      w = fmaf(c.cpy, yp, w);
      w = fmaf(c.cmz, st.win[s - 1][O][r], w);
      w = fmaf(c.cpz, st.win[s - 1][N][r], w);
      nv[r] = (!MASK || (p_in && st.row_in[r])) ? w : 0.0f;
    }
    if (s < K) {
#pragma unroll
      for (int r = 0; r < RY; r++) st.win[s][N][r] = nv[r];
    } else if (p >= zlo && p < zhi) {
#pragma unroll
      for (int r = 0; r < RY; r++)
        if (st.row_out[r]) out[(ptrdiff_t)p * plane + col0 + (ptrdiff_t)r * nx] = nv[r];
    }
  }
  // publish the edge rows of the planes just made (levels 0..K-1)
#pragma unroll
  for (int s = 0; s < K; s++) {
    edge[par][s][w][0][lane] = st.win[s][N][0];
    edge[par][s][w][1][lane] = st.win[s][N][RY - 1];
  }
  __syncthreads();
}

// input planes z = zlo-K .. zhi+K-1, three per trip so that the window slots
// rotate at compile time
template <int K, bool FIELD, bool MASK>
__device__ __forceinline__ void fused_march(FusedState<K, FIELD> &st, float (*edge)[K][FW][2][64],
                                            const float *__restrict__ in, float *__restrict__ out,
                                            const float *__restrict__ c0f, ptrdiff_t plane, ptrdiff_t col0,
                                            int nx, int gz0, int nz, int zlo, int zhi, int lane, int w,
                                            const oc::Star7Coef &c) {
  int z = zlo - K;
  const int zend = zhi + K;
  for (; z + 3 <= zend; z += 3) {
    fused_plane<K, FIELD, MASK, 0>(st, edge, z, in, out, c0f, plane, col0, nx, gz0, nz, zlo, zhi, lane, w, c);
    fused_plane<K, FIELD, MASK, 1>(st, edge, z + 1, in, out, c0f, plane, col0, nx, gz0, nz, zlo, zhi, lane, w, c);
    fused_plane<K, FIELD, MASK, 2>(st, edge, z + 2, in, out, c0f, plane, col0, nx, gz0, nz, zlo, zhi, lane, w, c);
  }
  if (z < zend)
    fused_plane<K, FIELD, MASK, 0>(st, edge, z, in, out, c0f, plane, col0, nx, gz0, nz, zlo, zhi, lane, w, c);
  if (z + 1 < zend)
    fused_plane<K, FIELD, MASK, 1>(st, edge, z + 1, in, out, c0f, plane, col0, nx, gz0, nz, zlo, zhi, lane, w, c);
}

template <int K, bool FIELD>
__global__ __launch_bounds__(64 * FW) void k_star7_fused(const float *__restrict__ in, float *__restrict__ out,
                                                         const float *__restrict__ c0f, int nx, int ny,
                                                         int zo_lo, int zo_hi, int gz0, int nz, int nbx,
                                                         int nby, int nbz, int fz, oc::Star7Coef c) {
  constexpr int OX = 64 - 2 * K, OY = FTY - 2 * K;
  // edge rows of levels 0..K-1: [plane parity][level][wave][first/last row][lane]
  __shared__ float edge[2][K][FW][2][64];
  const int nb = nbx * nby * nbz;
  const int t = xcd_tile(blockIdx.x, nb);
  if (t >= nb) return;   // uniform across the workgroup
  const int tbx = t % nbx, tby = (t / nbx) % nby, tbz = t / (nbx * nby);
  const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
  const int xt = tbx * OX - K, yt = tby * OY - K;   // tile origin
  const int x = xt + lane;
  const int y0 = yt + w * RY;
  const bool x_in = x >= 0 && x < nx;
  const bool x_out = lane >= K && lane < K + OX && x_in;
  FusedState<K, FIELD> st;
#pragma unroll
  for (int r = 0; r < RY; r++) {
    const int y = y0 + r, ty = w * RY + r;
    st.row_in[r] = x_in && y >= 0 && y < ny;
    st.row_out[r] = x_out && y >= 0 && y < ny && ty >= K && ty < K + OY;
  }
  const int zlo = zo_lo + tbz * fz;
  const int zhi = min(zlo + fz, zo_hi);
  const ptrdiff_t plane = (ptrdiff_t)nx * (ptrdiff_t)ny;
  const ptrdiff_t col0 = (ptrdiff_t)y0 * nx + x;   // row 0 of this thread's strip
#pragma unroll
  for (int s = 0; s < K; s++)
#pragma unroll
    for (int r = 0; r < RY; r++) {
      st.win[s][0][r] = st.win[s][1][r] = st.win[s][2][r] = 0.0f;
      st.cw[s][r] = 0.0f;
    }
  for (int i = (int)threadIdx.x; i < 2 * K * FW * 2 * 64; i += 64 * FW) (&edge[0][0][0][0][0])[i] = 0.0f;
  __syncthreads();
  // the whole tile and its planes inside the grid: no boundary masking
  const bool interior = xt >= 0 && xt + 64 <= nx && yt >= 0 && yt + FTY <= ny && gz0 + zlo - K >= 0 &&
                        gz0 + zhi + K <= nz;
  if (interior)
    fused_march<K, FIELD, false>(st, edge, in, out, c0f, plane, col0, nx, gz0, nz, zlo, zhi, lane, w, c);
  else
    fused_march<K, FIELD, true>(st, edge, in, out, c0f, plane, col0, nx, gz0, nz, zlo, zhi, lane, w, c);
}

// Workgroups of k_star7_fused<K, FIELD> the device holds at once (occupancy x
// compute units), looked up once per kernel.
template <int K>
int64_t fused_resident_wgs(bool field) {
  static std::atomic<int> per_cu[2] = {{0}, {0}};
  int n = per_cu[field].load(std::memory_order_relaxed);
  if (n <= 0) {
    int blocks = 0;
    hipError_t e = field ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_star7_fused<K, true>, 64 * FW, 0)
                         : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_star7_fused<K, false>, 64 * FW, 0);
    n = (e == hipSuccess && blocks > 0) ? blocks : 1;
    per_cu[field].store(n, std::memory_order_relaxed);
  }
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    cus = 256;
  return (int64_t)n * cus;
}

template <int K>
hipError_t launch_fused(const float *in, float *out, const float *c0f, int64_t nx, int64_t ny,
                        int64_t zo_lo, int64_t zo_hi, int64_t gz0, int64_t nz, const oc::Star7Coef &c,
                        hipStream_t s, oc::KernelTimer *kt) {
  constexpr int OX = 64 - 2 * K, OY = FTY - 2 * K;
  const int nbx = (int)((nx + OX - 1) / OX);
  const int nby = (int)((ny + OY - 1) / OY);
  // z chunks: as many as keep every workgroup of the launch resident at once
  // (one round over the chip), since each chunk recomputes 2K planes of
  // halo; at least 2K output planes per chunk
  const int64_t nz_out = zo_hi - zo_lo;
  const int64_t xy = (int64_t)nbx * nby;
  const int64_t resident = fused_resident_wgs<K>(c0f != nullptr);
  int64_t nbz = std::max<int64_t>(1, std::min<int64_t>(nz_out / (2 * K), resident / xy));
  const int fz = (int)((nz_out + nbz - 1) / nbz);
  nbz = (nz_out + fz - 1) / fz;
  const int64_t nb = xy * nbz;
  if (nb > 0x7fffffff) return hipErrorInvalidValue;
  if (c0f)
    hipExtLaunchKernelGGL((k_star7_fused<K, true>), dim3((unsigned)nb), dim3(64 * FW), 0, s, oc::kt_start(kt),
                          oc::kt_stop(kt), 0, in, out, c0f, (int)nx, (int)ny, (int)zo_lo, (int)zo_hi,
                          (int)gz0, (int)nz, nbx, nby, (int)nbz, fz, c);
  else
    hipExtLaunchKernelGGL((k_star7_fused<K, false>), dim3((unsigned)nb), dim3(64 * FW), 0, s, oc::kt_start(kt),
                          oc::kt_stop(kt), 0, in, out, c0f, (int)nx, (int)ny, (int)zo_lo, (int)zo_hi,
                          (int)gz0, (int)nz, nbx, nby, (int)nbz, fz, c);
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
    case 1: return launch_fused<1>(in, out, c0f, nx, ny, zo_lo, zo_hi, gz0, nz, c, s, kt);
    case 2: return launch_fused<2>(in, out, c0f, nx, ny, zo_lo, zo_hi, gz0, nz, c, s, kt);
    case 3: return launch_fused<3>(in, out, c0f, nx, ny, zo_lo, zo_hi, gz0, nz, c, s, kt);
    case 4: return launch_fused<4>(in, out, c0f, nx, ny, zo_lo, zo_hi, gz0, nz, c, s, kt);
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
  const int nby = (int)((ny + TY - 1) / TY);
  const int nbz = (int)((z_hi - z_lo + ZC - 1) / ZC);
  const uintptr_t align = (uintptr_t)in | (uintptr_t)out | (uintptr_t)c0f;
  if (nx % 4 == 0 && align % 16 == 0) {   // rows of whole float4s
    const int nbx = (int)((nx + VX - 1) / VX);
    const int64_t nb = (int64_t)nbx * nby * nbz;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    dim3 grid((unsigned)nb);
    if (c0f)
      hipExtLaunchKernelGGL(k_star7_x4<true>, grid, dim3(64, TY), 0, s, kt_start(kt), kt_stop(kt), 0, in, out,
                            c0f, (int)nx, (int)ny, (int)z_lo, (int)z_hi, (int)gz0, (int)nz, nbx, nby, nbz, c);
    else
      hipExtLaunchKernelGGL(k_star7_x4<false>, grid, dim3(64, TY), 0, s, kt_start(kt), kt_stop(kt), 0, in, out,
                            c0f, (int)nx, (int)ny, (int)z_lo, (int)z_hi, (int)gz0, (int)nz, nbx, nby, nbz, c);
    return hipGetLastError();
  }
  const int nbx = (int)((nx + TX - 1) / TX);
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
