// codec_dev.h -- device-side pieces of the fixed-rate block codec (gfx950),
// shared by the codec kernels and the fused decode / stencil / encode kernel.
//
// One lane codes one 4x4x4 block from start to finish, with all per-block
// state in registers; the slot a lane reads or writes (2R dwords, R bits per
// value) lives in LDS.  Format: 8-bit block exponent, quantisation to 27-bit
// integers, the ZFP method's decorrelating transform along x, y and z (lifting
// steps, wrapping arithmetic, floor shifts), sequency order, negabinary,
// embedded group-test bit-plane coding (the budget may end the stream inside
// any plane), reconstruction ldexp((float)q, Eb - 153).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

// ---- coefficient order: ascending (i+j+k, i^2+j^2+k^2, t) ------------------
struct SeqOrder {
  int at[64];
};
constexpr SeqOrder make_seq_order() {
  SeqOrder o{};
  int key1[64] = {}, key2[64] = {};
  for (int t = 0; t < 64; t++) {
    int i = t & 3, j = (t >> 2) & 3, k = t >> 4;
    key1[t] = i + j + k;
    key2[t] = i * i + j * j + k * k;
    o.at[t] = t;
  }
  // selection sort, compile time
  for (int a = 0; a < 64; a++) {
    int best = a;
    for (int b = a + 1; b < 64; b++) {
      int x = o.at[b], y = o.at[best];
      bool less = key1[x] != key1[y] ? key1[x] < key1[y]
                  : key2[x] != key2[y] ? key2[x] < key2[y] : x < y;
      if (less) best = b;
    }
    int tmp = o.at[a];
    o.at[a] = o.at[best];
    o.at[best] = tmp;
  }
  return o;
}
constexpr SeqOrder kSeq = make_seq_order();

// ---- decorrelating transform of one line (wrapping, floor shifts) ----------
// The published matrix of the ZFP method, (1/16) [[4 4 4 4] [5 1 -1 -5]
// [-4 4 4 -4] [-2 6 -6 2]], as five lifting steps: halve-and-difference of the
// outer pair, of the inner pair, of the two means and of the two differences,
// then a shear of the differences.  The halvings drop low bits, so the inverse
// (the steps undone in reverse order) is exact only to a few units of the
// 27-bit integers.
__device__ __forceinline__ int32_t wadd(int32_t u, int32_t v) { return (int32_t)((uint32_t)u + (uint32_t)v); }
__device__ __forceinline__ int32_t wsub(int32_t u, int32_t v) { return (int32_t)((uint32_t)u - (uint32_t)v); }
__device__ __forceinline__ void lift_fwd(int32_t &a, int32_t &b, int32_t &c, int32_t &d) {
  int32_t x0 = a, x1 = b, x2 = c, x3 = d;
  x0 = wadd(x0, x3) >> 1;  x3 = wsub(x3, x0);
  x2 = wadd(x2, x1) >> 1;  x1 = wsub(x1, x2);
  x0 = wadd(x0, x2) >> 1;  x2 = wsub(x2, x0);
  x3 = wadd(x3, x1) >> 1;  x1 = wsub(x1, x3);
  x3 = wadd(x3, x1 >> 1);  x1 = wsub(x1, x3 >> 1);
  a = x0;
  b = x1;
  c = x2;
  d = x3;
}
__device__ __forceinline__ void lift_inv(int32_t &a, int32_t &b, int32_t &c, int32_t &d) {
  int32_t x0 = a, x1 = b, x2 = c, x3 = d;
  x1 = wadd(x1, x3 >> 1);  x3 = wsub(x3, x1 >> 1);
  x1 = wadd(x1, x3);       x3 = wsub(wadd(x3, x3), x1);
  x2 = wadd(x2, x0);       x0 = wsub(wadd(x0, x0), x2);
  x1 = wadd(x1, x2);       x2 = wsub(wadd(x2, x2), x1);
  x3 = wadd(x3, x0);       x0 = wsub(wadd(x0, x0), x3);
  a = x0;
  b = x1;
  c = x2;
  d = x3;
}

__device__ __forceinline__ void xform_fwd(int32_t *q) {
#pragma unroll
  for (int k = 0; k < 4; k++)
#pragma unroll
    for (int j = 0; j < 4; j++) lift_fwd(q[16 * k + 4 * j], q[16 * k + 4 * j + 1], q[16 * k + 4 * j + 2], q[16 * k + 4 * j + 3]);
#pragma unroll
  for (int k = 0; k < 4; k++)
#pragma unroll
    for (int i = 0; i < 4; i++) lift_fwd(q[16 * k + i], q[16 * k + 4 + i], q[16 * k + 8 + i], q[16 * k + 12 + i]);
#pragma unroll
  for (int j = 0; j < 4; j++)
#pragma unroll
    for (int i = 0; i < 4; i++) lift_fwd(q[4 * j + i], q[16 + 4 * j + i], q[32 + 4 * j + i], q[48 + 4 * j + i]);
}
__device__ __forceinline__ void xform_inv(int32_t *q) {
#pragma unroll
  for (int j = 0; j < 4; j++)
#pragma unroll
    for (int i = 0; i < 4; i++) lift_inv(q[4 * j + i], q[16 + 4 * j + i], q[32 + 4 * j + i], q[48 + 4 * j + i]);
#pragma unroll
  for (int k = 0; k < 4; k++)
#pragma unroll
    for (int i = 0; i < 4; i++) lift_inv(q[16 * k + i], q[16 * k + 4 + i], q[16 * k + 8 + i], q[16 * k + 12 + i]);
#pragma unroll
  for (int k = 0; k < 4; k++)
#pragma unroll
    for (int j = 0; j < 4; j++) lift_inv(q[16 * k + 4 * j], q[16 * k + 4 * j + 1], q[16 * k + 4 * j + 2], q[16 * k + 4 * j + 3]);
}

// ---- 32x32 bit-matrix transpose, in place: bit c of A[r] <-> bit r of A[c] --
__device__ __forceinline__ void bit_transpose32(uint32_t *A) {
#pragma unroll
  for (int r = 0; r < 16; r++) {
    // halves: bytes {A.b0, A.b1, B.b0, B.b1} and {A.b2, A.b3, B.b2, B.b3}
    uint32_t a = A[r], b = A[r + 16];
    A[r] = __builtin_amdgcn_perm(b, a, 0x05040100u);
    A[r + 16] = __builtin_amdgcn_perm(b, a, 0x07060302u);
  }
#pragma unroll
  for (int r = 0; r < 32; r++) {
    if (r & 8) continue;
    uint32_t a = A[r], b = A[r + 8];
    A[r] = __builtin_amdgcn_perm(b, a, 0x06020400u);
    A[r + 8] = __builtin_amdgcn_perm(b, a, 0x07030501u);
  }
#pragma unroll
  for (int r = 0; r < 32; r++) {
    if (r & 4) continue;
    uint32_t t = ((A[r] >> 4) ^ A[r + 4]) & 0x0F0F0F0Fu;
    A[r] ^= t << 4;
    A[r + 4] ^= t;
  }
#pragma unroll
  for (int r = 0; r < 32; r++) {
    if (r & 2) continue;
    uint32_t t = ((A[r] >> 2) ^ A[r + 2]) & 0x33333333u;
    A[r] ^= t << 2;
    A[r + 2] ^= t;
  }
#pragma unroll
  for (int r = 0; r < 32; r++) {
    if (r & 1) continue;
    uint32_t t = ((A[r] >> 1) ^ A[r + 1]) & 0x55555555u;
    A[r] ^= t << 1;
    A[r + 1] ^= t;
  }
}

// floor((1 - (-2)^d) / 6): the mean of d unread negabinary digits, rounded
// down.  d = 0 (nothing unread) and d = 32 (nothing read, so no 1 read either)
// add nothing.
__device__ __forceinline__ int32_t unread_mean(int d) {
  if (d <= 0 || d >= 32) return 0;
  const int64_t pw = (int64_t)1 << d;
  const int64_t num = 1 - ((d & 1) ? -pw : pw);
  return (int32_t)(num >= 0 ? num / 6 : -((-num + 5) / 6));
}

__device__ __forceinline__ uint64_t lowmask64(int n) {
  return n >= 64 ? ~0ull : ((1ull << n) - 1ull);
}

// ---- bit writer over one slot of NW dwords ----------------------------------
// Branch-free: every put stores the current (possibly partial) dword, so a
// later put simply overwrites it; once the budget is spent the index is
// clamped onto the slot's padding dword (index NW), which is never copied out.
// The slot must start zeroed, and flush() ends the stream.
struct BitWriter {
  uint32_t *slot;
  int NW;    // dwords in the slot
  uint64_t acc;
  int nacc;  // valid bits in acc (< 32 between calls)
  int widx;  // dwords completed
  __device__ __forceinline__ int pos() const { return 32 * widx + nacc; }
  __device__ __forceinline__ void put(uint32_t v, int len) {  // len <= 32, v < 2^len
    acc |= (uint64_t)v << nacc;
    nacc += len;
    slot[min(widx, NW)] = (uint32_t)acc;
    const bool full = nacc >= 32;
    widx += full ? 1 : 0;
    acc = full ? (acc >> 32) : acc;
    nacc -= full ? 32 : 0;
  }
  __device__ __forceinline__ void put64(uint64_t v, int len) {  // len <= 64
    const int lo = min(len, 32);
    put((uint32_t)v & (lo >= 32 ? 0xFFFFFFFFu : ((1u << lo) - 1u)), lo);
    put((uint32_t)(v >> 32), len - lo);
  }
  // Stores the bits still held in acc (a put that completes a dword leaves the
  // carry in acc until the next put).
  __device__ __forceinline__ void flush() { slot[min(widx, NW)] = (uint32_t)acc; }
};

// ---- bit reader over one slot of NW dwords ----------------------------------
struct BitReader {
  const uint32_t *slot;
  int NW;
  uint64_t win;  // dwords wi, wi+1
  int wi, off;   // bit position = 32*wi + off, 0 <= off < 32
  __device__ __forceinline__ uint32_t fetch(int i) const {   // 0 past the slot, branch-free
    const uint32_t v = slot[min(i, NW - 1)];
    return i < NW ? v : 0u;
  }
  __device__ __forceinline__ void init(const uint32_t *s, int nw) {
    slot = s;
    NW = nw;
    wi = 0;
    off = 0;
    win = (uint64_t)fetch(0) | ((uint64_t)fetch(1) << 32);
  }
  __device__ __forceinline__ int pos() const { return 32 * wi + off; }
  // the next 32 bits of the stream (lowest = next bit)
  __device__ __forceinline__ uint32_t peek() const { return (uint32_t)(win >> off); }
  __device__ __forceinline__ void advance(int len) {  // off + len < 64
    off += len;
    const bool f = off >= 32;
    const uint32_t nxt = fetch(wi + 2);
    off -= f ? 32 : 0;
    wi += f ? 1 : 0;
    win = f ? ((win >> 32) | ((uint64_t)nxt << 32)) : win;
  }
  __device__ __forceinline__ uint32_t get(int len) {  // 1 <= len <= 32
    uint32_t v = (uint32_t)(win >> off) & (uint32_t)(len >= 32 ? 0xFFFFFFFFu : ((1u << len) - 1u));
    advance(len);
    return v;
  }
  __device__ __forceinline__ uint64_t get64(int len) {  // 0 <= len <= 64
    if (len == 0) return 0;
    if (len > 32) {
      uint64_t lo = get(32);
      return lo | ((uint64_t)get(len - 32) << 32);
    }
    return get(len);
  }
  // Consumes a run of zeros and the 1 ending it; returns the run length, or
  // -1 if no 1 appears within `limit` bits (the stream was cut by the budget).
  __device__ __forceinline__ int zero_run(int limit) {
    int run = 0;
    for (;;) {
      uint32_t w = (uint32_t)(win >> off);
      if (w) {
        int c = __builtin_ctz(w);
        if (run + c >= limit) return -1;
        advance(c + 1);
        return run + c;
      }
      run += 32;
      advance(32);
      if (run >= limit) return -1;
    }
  }
};

// ---- slot staging through LDS ----------------------------------------------------
// A workgroup's slots are one contiguous range of global memory; they move
// between global memory and LDS with coalesced dword accesses, and each lane
// reads / writes its own slot in LDS at a padded stride of NW + 1 dwords so
// that the per-lane sequential accesses spread over the LDS banks.
__device__ __forceinline__ uint32_t div_magic(int nw) {  // floor(2^32 / nw) + 1
  return (uint32_t)(0xFFFFFFFFu / (uint32_t)nw) + 1u;
}
__device__ __forceinline__ uint32_t lds_index(uint32_t i, int nw, uint32_t magic) {
  const uint32_t slot = __umulhi(i, magic);   // exact floor(i / nw) for i * nw < 2^32
  return i + slot;                            // slot * (nw + 1) + (i - slot * nw)
}

// ---- encoder ------------------------------------------------------------------
// Codes the block whose first value is at `base` (rows of 4 floats, row pitch
// nx, plane pitch nx*ny) into the lane's own LDS slot `my` of 2R + 1 zeroed
// dwords; returns true if the block holds an infinity or NaN.
template <bool ROLLED = false>
__device__ __forceinline__ bool encode_block(const float *__restrict__ base, int64_t nx, int64_t ny,
                                             int R, uint32_t *my) {
  const int NW = 2 * R;        // dwords per slot
  const int BITS = 64 * R;     // slot bits

  // load and take the block apart into sign / exponent / mantissa
  uint32_t raw[64];
#pragma unroll
  for (int k = 0; k < 4; k++)
#pragma unroll
    for (int j = 0; j < 4; j++) {
      float4 v = *reinterpret_cast<const float4 *>(base + (k * ny + j) * nx);
      raw[16 * k + 4 * j + 0] = __float_as_uint(v.x);
      raw[16 * k + 4 * j + 1] = __float_as_uint(v.y);
      raw[16 * k + 4 * j + 2] = __float_as_uint(v.z);
      raw[16 * k + 4 * j + 3] = __float_as_uint(v.w);
    }
  // block exponent: the largest exponent field, taken in place (bits 23..30)
  // so that no per-value exponent stays live until the quantisation below
  uint32_t emax = 0;
#pragma unroll
  for (int t = 0; t < 64; t++) emax = max(emax, raw[t] & 0x7F800000u);
  const bool bad = emax == 0x7F800000u;   // an infinity or NaN in the block
  const uint32_t Eb = max(emax >> 23, 1u);
  int32_t q[64];
#pragma unroll
  for (int t = 0; t < 64; t++) {
    uint32_t E = (raw[t] >> 23) & 255u;
    uint32_t M = E ? ((raw[t] & 0x7FFFFFu) | 0x800000u) : (raw[t] & 0x7FFFFFu);
    uint32_t sh = Eb - max(E, 1u);
    uint32_t mag = sh >= 27u ? 0u : ((M << 3) >> sh);
    q[t] = (raw[t] >> 31) ? -(int32_t)mag : (int32_t)mag;
  }
  xform_fwd(q);
  // reorder + negabinary, split in halves for the plane transpose
  uint32_t lo[32], hi[32];
#pragma unroll
  for (int p = 0; p < 32; p++) {
    lo[p] = ((uint32_t)q[kSeq.at[p]] + 0xAAAAAAAAu) ^ 0xAAAAAAAAu;
    hi[p] = ((uint32_t)q[kSeq.at[p + 32]] + 0xAAAAAAAAu) ^ 0xAAAAAAAAu;
  }
  bit_transpose32(lo);
  bit_transpose32(hi);
  // finish the transposes here: left to itself the compiler sinks their last
  // stages into the plane loop, which keeps more intermediate words live than
  // the 64 plane words (155 VGPRs, three waves per SIMD instead of four)
#pragma unroll
  for (int p = 0; p < 32; p++) {
    asm volatile("" : "+v"(lo[p]));
    asm volatile("" : "+v"(hi[p]));
  }

  BitWriter w;
  w.NW = NW;
  w.slot = my;
  w.acc = 0;
  w.nacc = 0;
  w.widx = 0;
  w.put(Eb, 8);
  int n = 0;
  // one bit plane; `plane` is the plane index
  auto code_plane = [&](int plane) __attribute__((always_inline)) {
    const int p = plane;
    if (w.pos() < BITS) {
      const uint64_t x = (uint64_t)lo[p] | ((uint64_t)hi[p] << 32);
      w.put64(x & lowmask64(n), n);
      if (n < 64) {
        uint64_t rest = x >> n;
        while (rest && w.pos() < BITS) {
          int tz = __builtin_ctzll(rest);
          // group test 1, then tz zeros and the set bit
          if (tz < 31) {
            uint32_t v = 1u | (2u << tz);
            int len = tz + 2;
            n += tz + 1;
            rest >>= tz + 1;
            // the next token in the same 32-bit put when it fits (bits past
            // the budget only ever reach the slot's padding dword)
            if (rest) {
              const int tz2 = __builtin_ctzll(rest);
              if (len + tz2 + 2 <= 32) {
                v |= (1u | (2u << tz2)) << len;
                len += tz2 + 2;
                n += tz2 + 1;
                rest >>= tz2 + 1;
              }
            }
            w.put(v, len);
            continue;
          } else if (tz < 62) {
            w.put64(1ull | (2ull << tz), tz + 2);
          } else {
            w.put(1u, 1);
            w.put64(1ull << tz, tz + 1);
          }
          n += tz + 1;
          rest = (tz + 1 < 64) ? (rest >> (tz + 1)) : 0ull;
        }
        if (n < 64) w.put(0u, 1);            // group test: nothing left
      }
    }
  };
  if constexpr (ROLLED) {
    // one loop body (the plane words indexed by the uniform plane number):
    // small code, for kernels whose waves run other code beside the coder
#pragma unroll 1
    for (int p = 31; p >= 0; p--) code_plane(p);
  } else {
#pragma unroll
    for (int p = 31; p >= 0; p--) code_plane(p);
  }
  w.flush();
  return bad;
}

// Decodes one slot (NW = 2R dwords, the bit stream LSB first) into the
// block's 64 integers q in value order t = i + 4j + 16k and returns the
// block exponent Eb: the values are ldexp(q[t], Eb - 153).  Where the budget
// cut the stream, a coefficient with a 1 among its read digits gets the mean
// of its unread digits added.
__device__ __forceinline__ int decode_block(const uint32_t *slot, int R, int32_t (&q)[64]) {
  const int NW = 2 * R;
  const int BITS = 64 * R;
  BitReader r;
  r.init(slot, NW);
  const int Eb = (int)r.get(8);
  uint32_t lo[32], hi[32];
  int n = 0;
  bool done = false;
  // where the budget ended the stream: plane cut_p, with the digits of
  // coefficients [0, cut_m) of that plane read (cut_p = -1: every plane read)
  int cut_p = -1, cut_m = 0;
  // one loop body (plane words indexed by the uniform plane number): the
  // fused kernel's decode waves run beside encode and stencil waves, and a
  // fully unrolled decoder alone is larger than the instruction cache
#pragma unroll 1
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
  return Eb;
}

}  // namespace
