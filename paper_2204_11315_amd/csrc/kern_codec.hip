// kern_codec.hip -- fixed-rate block codec on gfx950 (encode and decode).
//
// The paper compresses each chunk on the GPU before it is copied back and
// decompresses it after it is copied in (Sec. 1, Sec. 4.2), at a fixed,
// user-specified rate (Sec. 5).  The format is this library's own fixed-rate
// block-transform code after the method of the compressor the paper runs
// (block floating point, the ZFP decorrelating transform in integer lifting
// steps, embedded bit-plane coding with group tests); every slot
// holds one 4x4x4 block in exactly 64*R bits, so a block's position in the
// stream is known without any index, and every group of four planes is one
// contiguous byte range.
//
// Kernel layout: one lane codes one block from start to finish.  A wave takes
// 64 consecutive blocks along x, so the 16 row loads/stores of a block are
// 64 x 16 B contiguous per instruction.  All per-block state lives in
// registers: 64 coefficients, turned by an in-register 32x32 bit-matrix
// transpose (twice) into 32 bit-plane words of 64 bits.  The embedded coder
// emits each plane in closed form: n verbatim bits, then one "group" token
// per newly significant coefficient (found with a count-trailing-zeros on the
// plane word shifted by n), then a closing 0 unless all 64 are significant.
// The decoder mirrors it, reading 64-bit windows of its slot; where the
// budget cut the stream, a coefficient with a 1 read gets the mean of its
// unread digits added (as the reference decoder does).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "oc_kernels.h"

// Sticky per-device error word: bit 0 = a non-finite value was met by the
// encoder.  Read and cleared by the host through its symbol address.
__device__ int g_oc_codec_err;

#include "codec_dev.h"
#include "stencil_dev.h"

namespace {

extern __shared__ uint32_t lds_slots[];

__global__ __launch_bounds__(256) void k_encode(const float *__restrict__ in, int64_t nx, int64_t ny,
                                                int64_t nbx, int64_t nby, int64_t nblocks, int R,
                                                uint32_t *__restrict__ out) {
  const int NW = 2 * R;        // dwords per slot
  const int64_t b0 = (int64_t)blockIdx.x * blockDim.x;
  const int64_t b = b0 + threadIdx.x;
  const int nslots = (int)min<int64_t>(blockDim.x, nblocks - b0);
  uint32_t *my = lds_slots + threadIdx.x * (NW + 1);
  for (int i = 0; i <= NW; i++) my[i] = 0u;   // own slot (+ pad); the writer only ORs in order
  if (b < nblocks) {
    const int64_t bx = b % nbx;
    const int64_t by = (b / nbx) % nby;
    const int64_t bz = b / (nbx * nby);
    if (encode_block(in + ((4 * bz) * ny + 4 * by) * nx + 4 * bx, nx, ny, R, my))
      atomicOr(&g_oc_codec_err, 1);
  }
  __syncthreads();
  // coalesced copy of the workgroup's slots to global memory, eight LDS
  // reads in flight per thread before their stores
  const uint32_t magic = div_magic(NW);
  uint32_t *dst = out + b0 * NW;
  const uint32_t total = (uint32_t)(nslots * NW);
  uint32_t i = threadIdx.x;
  for (; i + 7 * blockDim.x < total; i += 8 * blockDim.x) {
    uint32_t v[8];
#pragma unroll
    for (int j = 0; j < 8; j++) v[j] = lds_slots[lds_index(i + j * blockDim.x, NW, magic)];
#pragma unroll
    for (int j = 0; j < 8; j++) dst[i + j * blockDim.x] = v[j];
  }
  for (; i < total; i += blockDim.x) dst[i] = lds_slots[lds_index(i, NW, magic)];
}

// ---- workgroup sums of error statistics --------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
// Sums se and sr and takes the maximum of mx over the workgroup (at most 1024
// threads) in a fixed order; thread 0 writes the three results to dst.  Every
// thread of the workgroup must call it.
__device__ void block_sums(double se, double sr, double mx, double *dst) {
  __shared__ double red[3][16];
  se = wave_sum(se);
  sr = wave_sum(sr);
  mx = wave_max(mx);
  const int w = (int)threadIdx.x >> 6, l = (int)threadIdx.x & 63;
  if (l == 0) {
    red[0][w] = se;
    red[1][w] = sr;
    red[2][w] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0, m = 0.0;
    for (int i = 0; i < ((int)blockDim.x + 63) >> 6; i++) {
      a += red[0][i];
      c += red[1][i];
      m = fmax(m, red[2][i]);
    }
    dst[0] = a;
    dst[1] = c;
    dst[2] = m;
  }
}

// Error statistics of x against the reference r over n values: per workgroup
// (a fixed grid striding over the arrays) the sum of (x - r)^2, the sum of r^2
// and the largest |x - r|, in FP64.  Needs n % 4 == 0 and 16-byte alignment.
__global__ __launch_bounds__(256) void k_diff_err(const float4 *__restrict__ r, const float4 *__restrict__ x,
                                                  int64_t n4, double *__restrict__ parts) {
  double se = 0.0, sr = 0.0, mx = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x) {
    const float4 a = r[i], b = x[i];
    const float ra[4] = {a.x, a.y, a.z, a.w}, xb[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const double d = (double)xb[j] - (double)ra[j];
      se += d * d;
      sr += (double)ra[j] * (double)ra[j];
      mx = fmax(mx, fabs(d));
    }
  }
  block_sums(se, sr, mx, parts + 3 * (int64_t)blockIdx.x);
}

// One workgroup folds nparts triples (sum, sum, max) into out[3]: thread t
// takes triples t, t + 256, ... in order, then the fixed-order workgroup sum.
__global__ __launch_bounds__(256) void k_reduce_parts(const double *__restrict__ parts, int64_t nparts,
                                                      double *__restrict__ out) {
  double se = 0.0, sr = 0.0, mx = 0.0;
  for (int64_t i = threadIdx.x; i < nparts; i += blockDim.x) {
    se += parts[3 * i];
    sr += parts[3 * i + 1];
    mx = fmax(mx, parts[3 * i + 2]);
  }
  block_sums(se, sr, mx, out);
}

// ---- decoder ------------------------------------------------------------------
// Per-workgroup error sums of a codec round trip: sum of squared errors, sum
// of squared inputs (FP64) and the largest absolute error, of the blocks one
// workgroup coded.
struct ErrSums {
  double *parts;   // [gridDim.x][3]
};

// One kernel body for two modes (kept as one function so that the decoder's
// register allocation is that of a plain kernel; for the same reason the
// block decoder is written out here rather than called as decode_block(),
// which compiles to 97 VGPRs in this kernel against 91, one wave per SIMD
// fewer, and ran 37 % slower in the bench job; the fused kernel calls decode_block(), and
// its tests require the two to give the same codes' values bit for bit):
//  - decode (ROUNDTRIP = false): the workgroup's code slots are staged from
//    `in` into LDS, decoded, and the values stored to `out`;
//  - round trip (ROUNDTRIP = true): each lane encodes its block of the FP32
//    field `field` into its LDS slot, decodes that slot, and compares the
//    decoded values with the block's inputs; the workgroup's error sums go to
//    `err` (no codes and no decoded values are written).
template <bool ROUNDTRIP>
__global__ __launch_bounds__(256) void k_decode_t(const uint32_t *__restrict__ in, const float *__restrict__ field,
                                                  int64_t nx, int64_t ny, int64_t nbx, int64_t nby,
                                                  int64_t nblocks, int R, float *__restrict__ out,
                                                  ErrSums err, const uint32_t *__restrict__ in_lo,
                                                  int64_t lo_words) {
  const int NW = 2 * R;
  const int BITS = 64 * R;
  const int64_t b0 = (int64_t)blockIdx.x * blockDim.x;
  const int64_t b = b0 + threadIdx.x;
  if (!ROUNDTRIP) {
    // coalesced copy of the workgroup's slots into LDS, eight loads in flight
    // per thread before their LDS stores (every workgroup of a launch starts
    // with this copy, so its latency is not hidden by other waves' work).
    // Input words below lo_words come from in_lo.
    const int nslots = (int)min<int64_t>(blockDim.x, nblocks - b0);
    const uint32_t magic = div_magic(NW);
    const int64_t w0 = b0 * NW;
    const uint32_t total = (uint32_t)(nslots * NW);
    if (w0 < lo_words && w0 + total > lo_words) {
      // the workgroup straddles the two sources: word by word
      for (uint32_t i = threadIdx.x; i < total; i += blockDim.x) {
        const int64_t wi = w0 + i;
        lds_slots[lds_index(i, NW, magic)] = wi < lo_words ? in_lo[wi] : in[wi];
      }
    } else {
      const uint32_t *src = (w0 < lo_words ? in_lo : in) + w0;
      uint32_t i = threadIdx.x;
      for (; i + 7 * blockDim.x < total; i += 8 * blockDim.x) {
        uint32_t v[8];
#pragma unroll
        for (int j = 0; j < 8; j++) v[j] = src[i + j * blockDim.x];
#pragma unroll
        for (int j = 0; j < 8; j++) lds_slots[lds_index(i + j * blockDim.x, NW, magic)] = v[j];
      }
      for (; i < total; i += blockDim.x) lds_slots[lds_index(i, NW, magic)] = src[i];
    }
    __syncthreads();
    if (b >= nblocks) return;
  }
  const int64_t bx = b % nbx;
  const int64_t by = (b / nbx) % nby;
  const int64_t bz = b / (nbx * nby);
  if (ROUNDTRIP) {
    uint32_t *my = lds_slots + threadIdx.x * (NW + 1);
    for (int i = 0; i <= NW; i++) my[i] = 0u;
    if (b < nblocks &&
        encode_block(field + ((4 * bz) * ny + 4 * by) * nx + 4 * bx, nx, ny, R, my))
      atomicOr(&g_oc_codec_err, 1);
  }

  BitReader r;
  r.init(lds_slots + threadIdx.x * (NW + 1), NW);
  const int Eb = (int)r.get(8);
  uint32_t lo[32], hi[32];
  int n = 0;
  bool done = false;
  // where the budget ended the stream: plane cut_p, with the digits of
  // coefficients [0, cut_m) of that plane read (cut_p = -1: every plane read)
  int cut_p = -1, cut_m = 0;
#pragma unroll
  for (int p = 31; p >= 0; p--) {
    uint64_t x = 0;
    if (!done) {
      const int pos0 = r.pos();
      x = r.get64(n);
      int m = -1;   // -1: plane p complete
      if (pos0 + n > BITS) {
        m = BITS - pos0;   // cut inside the verbatim digits
      } else {
        while (n < 64) {
          if (r.pos() >= BITS) { m = n; break; }   // no room for the group bit
          const uint32_t w = r.peek();
          if (!(w & 1u)) {                         // closing group bit
            r.advance(1);
            break;
          }
          const uint32_t t = w >> 1;
          if (t) {
            // group bit, run and its closing 1 all lie in the window: one step
            const int run = __builtin_ctz(t);
            if (run >= 64 - n) { m = n + min(64 - n, BITS - (r.pos() + 1)); break; }
            const int used = run + 2;
            x |= 1ull << (n + run);
            n += run + 1;
            // the next token too, when it lies in the same window (fewer trips
            // for the lanes with the most new coefficients in this plane)
            if (n < 64 && used < 32 && r.pos() + used < BITS) {
              const uint32_t w2 = w >> used;
              if (!(w2 & 1u)) {                    // closing group bit
                r.advance(used + 1);
                break;
              }
              const uint32_t t2 = (w2 >> 1) & ((1u << (31 - used)) - 1u);
              if (t2) {
                const int run2 = __builtin_ctz(t2);
                if (run2 < 64 - n) {
                  r.advance(used + run2 + 2);
                  x |= 1ull << (n + run2);
                  n += run2 + 1;
                  continue;
                }
              }
            }
            r.advance(used);
            continue;
          }
          r.advance(1);
          const int rs = r.pos();
          const int run = r.zero_run(64 - n);
          if (run < 0) { m = n + min(64 - n, BITS - rs); break; }   // cut inside a run
          x |= 1ull << (n + run);
          n += run + 1;
        }
      }
      if (m >= 0) {
        done = true;
        cut_p = p;
        cut_m = m;
      } else if (r.pos() >= BITS) {
        done = true;
        cut_p = p - 1;
        cut_m = 0;
      }
    }
    lo[p] = (uint32_t)x;
    hi[p] = (uint32_t)(x >> 32);
  }
  bit_transpose32(lo);
  bit_transpose32(hi);
  // a coefficient with a 1 read gets the mean of its unread digits: its lowest
  // read plane is cut_p below position cut_m, cut_p + 1 from there on
  const int32_t mean_in = cut_p >= 0 ? unread_mean(cut_p) : 0;
  const int32_t mean_out = cut_p >= 0 ? unread_mean(cut_p + 1) : 0;
  int32_t q[64];
#pragma unroll
  for (int p = 0; p < 32; p++) {
    const int32_t a = (int32_t)((lo[p] ^ 0xAAAAAAAAu) - 0xAAAAAAAAu);
    const int32_t b = (int32_t)((hi[p] ^ 0xAAAAAAAAu) - 0xAAAAAAAAu);
    const int32_t ma = lo[p] ? (p < cut_m ? mean_in : mean_out) : 0;
    const int32_t mb = hi[p] ? (p + 32 < cut_m ? mean_in : mean_out) : 0;
    q[kSeq.at[p]] = (int32_t)((uint32_t)a + (uint32_t)ma);
    q[kSeq.at[p + 32]] = (int32_t)((uint32_t)b + (uint32_t)mb);
  }
  xform_inv(q);
  const int e = Eb - 153;
  if (!ROUNDTRIP) {
    float *base = out + ((4 * bz) * ny + 4 * by) * nx + 4 * bx;
#pragma unroll
    for (int k = 0; k < 4; k++)
#pragma unroll
      for (int j = 0; j < 4; j++) {
        float4 v;
        v.x = ldexpf((float)q[16 * k + 4 * j + 0], e);
        v.y = ldexpf((float)q[16 * k + 4 * j + 1], e);
        v.z = ldexpf((float)q[16 * k + 4 * j + 2], e);
        v.w = ldexpf((float)q[16 * k + 4 * j + 3], e);
        *reinterpret_cast<float4 *>(base + (k * ny + j) * nx) = v;
      }
  } else {
    double se = 0.0, sr = 0.0, mx = 0.0;
    if (b < nblocks) {
      const float *base = field + ((4 * bz) * ny + 4 * by) * nx + 4 * bx;
#pragma unroll
      for (int k = 0; k < 4; k++)
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const float4 v = *reinterpret_cast<const float4 *>(base + (k * ny + j) * nx);
          const float x[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
          for (int i = 0; i < 4; i++) {
            const double r = (double)x[i];
            const double d = (double)ldexpf((float)q[16 * k + 4 * j + i], e) - r;
            se += d * d;
            sr += r * r;
            mx = fmax(mx, fabs(d));
          }
        }
    }
    block_sums(se, sr, mx, err.parts + 3 * (int64_t)blockIdx.x);
  }
}

// 256 lanes per workgroup (128 above 16 bits/value, to keep the slot staging
// within 34 KiB of LDS per workgroup)
int codec_threads(int rate) { return rate > 16 ? 128 : 256; }
size_t codec_lds_bytes(int rate, int threads) { return (size_t)threads * (size_t)(2 * rate + 1) * 4u; }

// ---- fused decode -> K 7-point steps -> encode, one launch per slab --------
// The three kernels of a coded residency (decode after the copy-in, k stencil
// steps, encode before the copy-back; Sec. 1, Sec. 3.1, Sec. 4.2) in one
// kernel with no full-size working buffer: a workgroup owns an xy tile of the
// slab and marches its block layers in z, holding decoded planes and finished
// output planes only in LDS.  Its eight waves take fixed roles for the whole
// launch, one step per block layer, one workgroup barrier per step:
//   waves 0-1  decode block layer t of the input tile (16 x 8 blocks, one lane
//              per block) into a two-layer LDS ring of FP32 planes;
//   waves 4-7  run the K-level wavefront over layer t-1's four planes: level s
//              makes plane z - s from level s-1's planes z-s-1 .. z-s+1, kept
//              in a three-plane register window per level; x neighbours by DPP
//              lane shifts, and each wave carries K extra rows on either side
//              of its 6 output rows so that no row crosses between waves
//              within a step; level K goes to a three-layer LDS output ring;
//   waves 2-3  encode the output layer the stencil finished in an earlier step
//              (14 x 6 blocks: the tile minus its one-block halo).
// Codes move between global memory and LDS with per-wave coalesced copies.
// The output tile is block aligned, so its codes are bit-identical to those of
// the decode / stencil / encode kernels on the same slab: same decoder and
// encoder, same per-cell operation order (star7_point), zero outside the grid.
constexpr int FZ_IBX = 16, FZ_IBY = 8;                    // input tile, blocks
constexpr int FZ_OBX = FZ_IBX - 2, FZ_OBY = FZ_IBY - 2;   // output tile, blocks
constexpr int FZ_ICX = 4 * FZ_IBX, FZ_ICY = 4 * FZ_IBY;   // 64 x 32 cells
constexpr int FZ_OCX = 4 * FZ_OBX, FZ_OCY = 4 * FZ_OBY;   // 56 x 24 cells
constexpr int FZ_DEC = 2, FZ_ENC = 2, FZ_ST = 4, FZ_WAVES = FZ_DEC + FZ_ENC + FZ_ST;
constexpr int FZ_SROWS = FZ_OCY / FZ_ST;                   // output rows per stencil wave
constexpr int FZ_EROWS = FZ_OBY / FZ_ENC;                  // output block rows per encode wave
constexpr int FZ_RING = 3;                                 // output layers held in LDS
constexpr int FZ_L0 = 2 * 4 * FZ_ICY * FZ_ICX;             // floats: two decoded layers
constexpr int FZ_OUT = FZ_RING * 4 * FZ_OCY * FZ_OCX;      // floats: the output ring
constexpr int FZ_DSLOTS = FZ_DEC * 64;
constexpr int FZ_ESLOTS = FZ_OBX * FZ_OBY;
static_assert(FZ_DEC * 64 == FZ_IBX * FZ_IBY, "one decode lane per input block");
static_assert(FZ_EROWS * FZ_OBX <= 64, "one encode lane per output block");

size_t fused_lds_bytes(int R) {
  return 4u * (size_t)(FZ_L0 + FZ_OUT) + 4u * (size_t)(FZ_DSLOTS + FZ_ESLOTS) * (size_t)(2 * R + 1);
}

struct FusedArgs {
  const uint32_t *in;   // slot codes: local block layer l at in + l * lw
  uint32_t *out;        // output codes: layer m at out + m * lw
  int64_t lw;           // dwords per coded layer (nbx * nby * 2R)
  int nx, ny, nbx, nby, R;
  int lay_lo, lay_hi;   // slot layers holding codes; the others lie outside the grid (zero)
  int nl;               // slot layers (S + 2h) / 4
  int out_l0, out_nl;   // local layer of output layer 0 (h / 4); output layers (S / 4)
  int gz0, nz;          // global z of local plane 0; grid depth
  int ntx, nty;         // tiles
  oc::Star7Coef c;
};

// LDS accesses of one wave take effect in issue order; this only keeps the
// compiler from moving the wave's later LDS reads above its earlier writes
// (another lane's slot data written by the same wave).
__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// dwords of one block row's slots per lane (16 blocks x 2R dwords / 64 lanes,
// R <= kCodecStar7MaxRate)
constexpr int FZ_CPL = (FZ_IBX * 2 * oc::kCodecStar7MaxRate + 63) / 64;
// the same for one output block row (14 blocks)
constexpr int FZ_EPL = (FZ_OBX * 2 * oc::kCodecStar7MaxRate + 63) / 64;

__device__ __forceinline__ void fz_decode_role(const FusedArgs &a, int tx, int ty, int w, int lane, int T,
                                               float *L0, uint32_t *DSL) {
  const int NW = 2 * a.R;
  const uint32_t magic = div_magic(NW);
  const int bx0 = tx * FZ_OBX - 1, by0 = ty * FZ_OBY - 1;   // the tile's first input block
  const int bxl = lane & 15, byl = 4 * w + (lane >> 4);
  const int bx = bx0 + bxl, by = by0 + byl;
  const bool xy_in = bx >= 0 && bx < a.nbx && by >= 0 && by < a.nby;
  const int cx_lo = max(bx0, 0), cx_hi = min(bx0 + FZ_IBX, a.nbx);
  const int n = max(cx_hi - cx_lo, 0) * NW;   // dwords of one block row's slots
  uint32_t *my = DSL + (64 * w + lane) * (NW + 1);
  // This wave's four block rows of a layer are four contiguous runs of
  // slots.  The codes of layer t + 1 are loaded into registers while layer t
  // is decoded (coalesced dwords, all loads in flight together) and moved
  // into the lanes' LDS slots at the start of the next step.
  uint32_t buf[4][FZ_CPL];
  auto row_ok = [&](int r) {
    const int gby = by0 + 4 * w + r;
    return gby >= 0 && gby < a.nby && n > 0;
  };
  auto lay_in = [&](int t) { return t >= a.lay_lo && t < a.lay_hi; };
  auto load_layer = [&](int t) {
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const uint32_t *src = a.in + (int64_t)t * a.lw + ((int64_t)(by0 + 4 * w + r) * a.nbx + cx_lo) * NW;
      const bool ok = row_ok(r);
#pragma unroll
      for (int j = 0; j < FZ_CPL; j++) {
        const int i = lane + 64 * j;
        buf[r][j] = (ok && i < n) ? src[i] : 0u;
      }
    }
  };
  auto store_layer = [&]() {
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const bool ok = row_ok(r);
      const int s0 = 64 * w + 16 * r + (cx_lo - bx0);
#pragma unroll
      for (int j = 0; j < FZ_CPL; j++) {
        const int i = lane + 64 * j;
        if (ok && i < n) {
          const int sl = (int)__umulhi((uint32_t)i, magic);   // i / NW
          DSL[(s0 + sl) * (NW + 1) + (i - sl * NW)] = buf[r][j];
        }
      }
    }
  };
  if (a.nl > 0 && lay_in(0)) load_layer(0);
  for (int t = 0; t < T; t++) {
    if (t < a.nl) {
      if (lay_in(t)) {
        store_layer();
        wave_lds_order();
      }
      if (t + 1 < a.nl && lay_in(t + 1)) load_layer(t + 1);
      const bool have = lay_in(t) && xy_in;
      float *dst = L0 + (t & 1) * (4 * FZ_ICY * FZ_ICX) + (4 * byl) * FZ_ICX + 4 * bxl;
      if (have) {
        int32_t q[64];
        const int e = decode_block(my, a.R, q) - 153;
#pragma unroll
        for (int k = 0; k < 4; k++)
#pragma unroll
          for (int j = 0; j < 4; j++) {
            float4 v;
            v.x = ldexpf((float)q[16 * k + 4 * j + 0], e);
            v.y = ldexpf((float)q[16 * k + 4 * j + 1], e);
            v.z = ldexpf((float)q[16 * k + 4 * j + 2], e);
            v.w = ldexpf((float)q[16 * k + 4 * j + 3], e);
            *reinterpret_cast<float4 *>(dst + (k * FZ_ICY + j) * FZ_ICX) = v;
          }
      } else {
        const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int k = 0; k < 4; k++)
#pragma unroll
          for (int j = 0; j < 4; j++) *reinterpret_cast<float4 *>(dst + (k * FZ_ICY + j) * FZ_ICX) = z4;
      }
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void fz_encode_role(const FusedArgs &a, int tx, int ty, int ew, int lane, int T,
                                               const float *OUT, uint32_t *ESL) {
  const int NW = 2 * a.R;
  const uint32_t magic = div_magic(NW);
  const bool act = lane < FZ_EROWS * FZ_OBX;
  const int la = act ? lane : 0;
  const int oxl = la % FZ_OBX, oyl = FZ_EROWS * ew + la / FZ_OBX;
  const int bx = tx * FZ_OBX + oxl, by = ty * FZ_OBY + oyl;
  const bool mine = act && bx < a.nbx && by < a.nby;
  uint32_t *my = ESL + (FZ_EROWS * FZ_OBX * ew + la) * (NW + 1);
  const int ncols = min(FZ_OBX, a.nbx - tx * FZ_OBX);
  for (int t = 0; t < T; t++) {
    const int m = t - (a.out_l0 + 3);   // the output layer the stencil finished a step ago
    if (m >= 0 && m < a.out_nl) {
      if (mine) {
        for (int i = 0; i <= NW; i++) my[i] = 0u;
        const float *base = OUT + (m % FZ_RING) * (4 * FZ_OCY * FZ_OCX) + (4 * oyl) * FZ_OCX + 4 * oxl;
        if (encode_block<true>(base, FZ_OCX, FZ_OCY, a.R, my)) atomicOr(&g_oc_codec_err, 1);
      }
      wave_lds_order();
      // this wave's block rows of the output layer: contiguous runs of
      // slots, copied out coalesced (every LDS read of a row issued first)
      const int n = ncols * NW;
#pragma unroll
      for (int r = 0; r < FZ_EROWS; r++) {
        const int gby = ty * FZ_OBY + FZ_EROWS * ew + r;
        if (gby >= a.nby) continue;
        uint32_t *dst = a.out + (int64_t)m * a.lw + ((int64_t)gby * a.nbx + tx * FZ_OBX) * NW;
        const int s0 = FZ_EROWS * FZ_OBX * ew + FZ_OBX * r;
        uint32_t v[FZ_EPL];
#pragma unroll
        for (int j = 0; j < FZ_EPL; j++) {
          const int i = lane + 64 * j;
          const int sl = (int)__umulhi((uint32_t)i, magic);
          v[j] = i < n ? ESL[(s0 + sl) * (NW + 1) + (i - sl * NW)] : 0u;
        }
#pragma unroll
        for (int j = 0; j < FZ_EPL; j++)
          if (lane + 64 * j < n) dst[lane + 64 * j] = v[j];
      }
    }
    __syncthreads();
  }
}

template <int K>
__device__ __forceinline__ void fz_stencil_role(const FusedArgs &a, int tx, int ty, int sw, int lane, int T,
                                                const float *L0, float *OUT) {
  constexpr int NR0 = FZ_SROWS + 2 * K;   // rows of level 0; level s has NR0 - 2s
  const int X = lane;
  const int gx = tx * FZ_OCX - 4 + X;
  const bool x_in = gx >= 0 && gx < a.nx;
  const bool x_out = X >= 4 && X < 4 + FZ_OCX;
  const int y0 = 4 + FZ_SROWS * sw;            // first output row of this wave (tile rows)
  const int gy0 = ty * FZ_OCY - 4 + y0;
  const int out_z0 = 4 * a.out_l0, out_z1 = out_z0 + 4 * a.out_nl;
  // win[s][i][r]: level s, planes (oldest, middle, newest), row y0 - (K - s) + r
  float win[K][3][NR0];
#pragma unroll
  for (int s = 0; s < K; s++)
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int r = 0; r < NR0; r++) win[s][i][r] = 0.0f;
  for (int t = 0; t < T; t++) {
    if (t >= 1 && t <= a.nl) {
      const int l = t - 1;
      const float *src = L0 + (l & 1) * (4 * FZ_ICY * FZ_ICX) + (y0 - K) * FZ_ICX + X;
      // one loop body for the layer's four planes (the windows move by
      // register copies): the three roles' code together must stay small
#pragma unroll 1
      for (int c = 0; c < 4; c++) {
        const int z = 4 * l + c;
#pragma unroll
        for (int r = 0; r < NR0; r++) {
          win[0][0][r] = win[0][1][r];
          win[0][1][r] = win[0][2][r];
          win[0][2][r] = src[(c * FZ_ICY + r) * FZ_ICX];
        }
#pragma unroll
        for (int s = 1; s <= K; s++) {
          const int nr = NR0 - 2 * s;
          const int gq = a.gz0 + z - s;
          const bool p_in = x_in && gq >= 0 && gq < a.nz;
          float nv[NR0];
#pragma unroll
          for (int r = 0; r < nr; r++) {
            const float cur = win[s - 1][1][r + 1];
            const float v = star7_point(a.c.c0, cur, lane_from_left(cur), lane_from_right(cur),
                                        win[s - 1][1][r], win[s - 1][1][r + 2], win[s - 1][0][r + 1],
                                        win[s - 1][2][r + 1], a.c);
            const int gy = gy0 - (K - s) + r;
            nv[r] = (p_in && gy >= 0 && gy < a.ny) ? v : 0.0f;
          }
          if (s < K) {
#pragma unroll
            for (int r = 0; r < nr; r++) {
              win[s][0][r] = win[s][1][r];
              win[s][1][r] = win[s][2][r];
              win[s][2][r] = nv[r];
            }
          } else {
            const int q = z - K;
            if (q >= out_z0 && q < out_z1 && x_out) {
              const int m = (q - out_z0) >> 2, pl = (q - out_z0) & 3;
              float *o = OUT + ((m % FZ_RING) * 4 + pl) * (FZ_OCY * FZ_OCX) + (FZ_SROWS * sw) * FZ_OCX + (X - 4);
#pragma unroll
              for (int r = 0; r < FZ_SROWS; r++) o[r * FZ_OCX] = nv[r];
            }
          }
        }
      }
    }
    __syncthreads();
  }
}

template <int K>
__global__ __launch_bounds__(64 * FZ_WAVES) void k_codec_star7(FusedArgs a) {
  const int tile = (int)blockIdx.x;
  if (tile >= a.ntx * a.nty) return;   // uniform over the workgroup
  const int tx = tile % a.ntx, ty = tile / a.ntx;
  const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int lane = (int)threadIdx.x & 63;
  float *L0 = reinterpret_cast<float *>(lds_slots);
  float *OUT = L0 + FZ_L0;
  uint32_t *DSL = reinterpret_cast<uint32_t *>(OUT + FZ_OUT);
  uint32_t *ESL = DSL + FZ_DSLOTS * (2 * a.R + 1);
  // steps: layer t is decoded in step t, stepped in step t + 1; output layer
  // m is finished in step out_l0 + m + 2 and encoded in the next one.  Every
  // wave runs all T steps, each ending in the one workgroup barrier.
  const int T = max(a.nl + 1, a.out_l0 + a.out_nl + 3);
  if (w < FZ_DEC)
    fz_decode_role(a, tx, ty, w, lane, T, L0, DSL);
  else if (w < FZ_DEC + FZ_ENC)
    fz_encode_role(a, tx, ty, w - FZ_DEC, lane, T, OUT, ESL);
  else
    fz_stencil_role<K>(a, tx, ty, w - FZ_DEC - FZ_ENC, lane, T, L0, OUT);
}

}  // namespace

namespace oc {

hipError_t launch_encode(const float *d_in, int64_t nx, int64_t ny, int64_t nlayers, int rate,
                         void *d_out, hipStream_t s, KernelTimer *kt) {
  if (rate < 1 || rate > 32) return hipErrorInvalidValue;
  const int64_t nbx = nx / 4, nby = ny / 4, nb = nbx * nby * nlayers;
  if (nb <= 0) return hipSuccess;
  const int threads = codec_threads(rate);
  dim3 grid((unsigned)((nb + threads - 1) / threads));
  hipExtLaunchKernelGGL(k_encode, grid, dim3(threads), codec_lds_bytes(rate, threads), s, kt_start(kt),
                        kt_stop(kt), 0, d_in, nx, ny,
                     nbx, nby, nb, rate, (uint32_t *)d_out);
  return hipGetLastError();
}

hipError_t launch_decode(const void *d_in, int64_t nx, int64_t ny, int64_t nlayers, int rate,
                         float *d_out, hipStream_t s, KernelTimer *kt, const void *d_in_lo,
                         int64_t lo_bytes) {
  if (rate < 1 || rate > 32) return hipErrorInvalidValue;
  const int64_t nbx = nx / 4, nby = ny / 4, nb = nbx * nby * nlayers;
  if (lo_bytes < 0 || lo_bytes % 4 || (lo_bytes > 0 && !d_in_lo) || lo_bytes > nb * 8 * rate)
    return hipErrorInvalidValue;
  if (nb <= 0) return hipSuccess;
  const int threads = codec_threads(rate);
  dim3 grid((unsigned)((nb + threads - 1) / threads));
  hipExtLaunchKernelGGL(k_decode_t<false>, grid, dim3(threads), codec_lds_bytes(rate, threads), s,
                        kt_start(kt), kt_stop(kt), 0, (const uint32_t *)d_in, (const float *)nullptr,
                        nx, ny, nbx, nby, nb, rate, d_out, ErrSums{nullptr},
                        (const uint32_t *)d_in_lo, lo_bytes / 4);
  return hipGetLastError();
}

int64_t codec_error_parts(int64_t nx, int64_t ny, int64_t nlayers, int rate) {
  if (rate < 1 || rate > 32) return 0;
  const int64_t nb = (nx / 4) * (ny / 4) * nlayers;
  const int threads = codec_threads(rate);
  return (nb + threads - 1) / threads;
}

hipError_t launch_codec_error(const float *d_in, int64_t nx, int64_t ny, int64_t nlayers, int rate,
                              double *parts, double *d_out3, hipStream_t s) {
  if (rate < 1 || rate > 32) return hipErrorInvalidValue;
  const int64_t nbx = nx / 4, nby = ny / 4, nb = nbx * nby * nlayers;
  if (nb <= 0) return hipErrorInvalidValue;
  const int threads = codec_threads(rate);
  const int64_t nparts = codec_error_parts(nx, ny, nlayers, rate);
  hipLaunchKernelGGL(k_decode_t<true>, dim3((unsigned)nparts), dim3(threads),
                     codec_lds_bytes(rate, threads), s, (const uint32_t *)nullptr, d_in, nx, ny, nbx,
                     nby, nb, rate, (float *)nullptr, ErrSums{parts}, (const uint32_t *)nullptr,
                     (int64_t)0);
  hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(256), 0, s, (const double *)parts, nparts, d_out3);
  return hipGetLastError();
}

hipError_t launch_diff_error(const float *ref, const float *x, int64_t n, double *parts, double *d_out3,
                             hipStream_t s) {
  if (n <= 0 || n % 4 || (((uintptr_t)ref | (uintptr_t)x) & 15)) return hipErrorInvalidValue;
  const int64_t n4 = n / 4;
  const int64_t nparts = std::min<int64_t>(kDiffErrParts, (n4 + 255) / 256);
  hipLaunchKernelGGL(k_diff_err, dim3((unsigned)nparts), dim3(256), 0, s, (const float4 *)ref,
                     (const float4 *)x, n4, parts);
  hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(256), 0, s, (const double *)parts, nparts, d_out3);
  return hipGetLastError();
}

size_t codec_star7_lds_bytes(int rate) { return fused_lds_bytes(rate); }

hipError_t launch_codec_star7(const void *in, void *out, int64_t nx, int64_t ny, int rate, int64_t lay_lo,
                              int64_t lay_hi, int64_t nl, int64_t out_l0, int64_t out_nl, int64_t gz0,
                              int64_t nz, int levels, const Star7Coef &c, hipStream_t s, KernelTimer *kt) {
  if (rate < 1 || rate > kCodecStar7MaxRate || levels < 1 || levels > 4) return hipErrorInvalidValue;
  if (nx <= 0 || ny <= 0 || nx % 4 || ny % 4 || out_l0 < 1 || 4 * out_l0 < levels || out_nl < 1 ||
      nl != out_nl + 2 * out_l0 || lay_lo < 0 || lay_hi > nl || lay_lo > lay_hi)
    return hipErrorInvalidValue;
  if (nx > (1 << 28) || ny > (1 << 28) || nl > (1 << 24) || gz0 < -(1 << 28) || gz0 > (1 << 28) ||
      nz > (1 << 28))
    return hipErrorInvalidValue;
  const int64_t nbx = nx / 4, nby = ny / 4;
  const int64_t ntx = (nbx + FZ_OBX - 1) / FZ_OBX, nty = (nby + FZ_OBY - 1) / FZ_OBY;
  if (ntx * nty > 0x7fffffff) return hipErrorInvalidValue;
  FusedArgs a;
  a.in = (const uint32_t *)in;
  a.out = (uint32_t *)out;
  a.lw = nbx * nby * 2 * rate;
  a.nx = (int)nx;
  a.ny = (int)ny;
  a.nbx = (int)nbx;
  a.nby = (int)nby;
  a.R = rate;
  a.lay_lo = (int)lay_lo;
  a.lay_hi = (int)lay_hi;
  a.nl = (int)nl;
  a.out_l0 = (int)out_l0;
  a.out_nl = (int)out_nl;
  a.gz0 = (int)gz0;
  a.nz = (int)nz;
  a.ntx = (int)ntx;
  a.nty = (int)nty;
  a.c = c;
  const size_t lds = fused_lds_bytes(rate);
  const dim3 grid((unsigned)(ntx * nty)), block(64 * FZ_WAVES);
  switch (levels) {
    case 1:
      hipExtLaunchKernelGGL(k_codec_star7<1>, grid, block, lds, s, kt_start(kt), kt_stop(kt), 0, a);
      break;
    case 2:
      hipExtLaunchKernelGGL(k_codec_star7<2>, grid, block, lds, s, kt_start(kt), kt_stop(kt), 0, a);
      break;
    case 3:
      hipExtLaunchKernelGGL(k_codec_star7<3>, grid, block, lds, s, kt_start(kt), kt_stop(kt), 0, a);
      break;
    default:
      hipExtLaunchKernelGGL(k_codec_star7<4>, grid, block, lds, s, kt_start(kt), kt_stop(kt), 0, a);
      break;
  }
  return hipGetLastError();
}

hipError_t codec_error_word(int **dev_ptr) {
  return hipGetSymbolAddress((void **)dev_ptr, HIP_SYMBOL(g_oc_codec_err));
}

}  // namespace oc

// ---- allocation-free round trip ----------------------------------------------
// The per-workgroup partial sums of the codec round trip live in this
// file-scope array when the caller brings no workspace: one copy per device,
// held until the process ends.  On the host the array's name only stands for
// the symbol; kernels get the device address that hipGetSymbolAddress returns
// for the current device, looked up once per device and kept.
static __device__ __align__(256) double scratch[3 * oc::kCodecErrStaticParts];

namespace oc {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_addr[kMaxDevices] = {};
}  // namespace

hipError_t codec_error_scratch(double **dev_ptr) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_addr[dev] = (double *)p;
  }
  *dev_ptr = g_scratch_addr[dev];
  return hipSuccess;
}

}  // namespace oc
