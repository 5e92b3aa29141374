/*
 * codec_ref.c -- scalar, bit-serial reference of the fixed-rate block codec.
 *
 * TEST INFRASTRUCTURE ONLY (see ocref.h).  Independent of the HIP codec.
 *
 * The paper compresses each chunk on the GPU before the device-to-host copy and
 * decompresses it after the host-to-device copy (Sec. 1 and Sec. 4.2), at a
 * user-specified fixed rate (Sec. 5: 32 bits per 64-bit value).  It uses a
 * third-party compressor (cuZFP, Sec. 4) and does not restate its format.  This
 * file defines our own fixed-rate format after that compressor's published
 * method (Lindstrom, "Fixed-Rate Compressed Floating-Point Arrays", IEEE TVCG
 * 2014): block floating point, its non-orthogonal integer decorrelating
 * transform, embedded bit-plane coding with group tests.  Each step below is
 * numbered as in the format definition; nothing is blocked, fused or
 * reordered.
 *
 * Format, per 4x4x4 block at R bits per value (1 <= R <= 32):
 *  1. The block owns a slot of B = 64*R bits.  Stream bit j lives in slot byte
 *     j>>3, bit j&7 (LSB first).  Values: t = i + 4j + 16k.
 *  2. Exponent: per value, sign s, biased exponent E, fraction F.  E == 255 is
 *     an error.  Ee = max(E,1); M = F | 2^23 when E > 0, else F.  Eb = max Ee.
 *     The first 8 stream bits hold Eb.
 *  3. Quantise (integers only): q = (-1)^s ((M << 3) >> (Eb - Ee)), a shift of
 *     27 or more giving 0.  |q| < 2^27.
 *  4. Transform: along x, then y, then z, every line of four integers is taken
 *     through the published decorrelating transform, the 4x4 matrix
 *     A = (1/16) [[4 4 4 4] [5 1 -1 -5] [-4 4 4 -4] [-2 6 -6 2]], computed as
 *     five lifting steps with floor halvings (see lift_fwd).  The halvings drop
 *     low bits, so the inverse (lift_inv, the steps undone in reverse order)
 *     returns the input to within a few units in the last place of the 27-bit
 *     integers.  Arithmetic wraps mod 2^32 and >> is a floor (arithmetic) shift.
 *  5. Reorder: output position p holds the coefficient whose (i,j,k) sorts p-th
 *     by the key (i+j+k, i^2+j^2+k^2, t).
 *  6. Negabinary: u = (c + 0xAAAAAAAA) ^ 0xAAAAAAAA as 32-bit unsigned.
 *  7. Embedded coding of the 64 words, bit plane 31 down to 0, into the
 *     remaining B-8 bits (see encode_planes).  Coding stops the moment the
 *     budget is spent; unused slot bits are 0.
 *  7'. Decoding reads the stream back.  Where the budget ended it before plane
 *     0, a coefficient whose digits of planes d-1 .. 0 were never read but
 *     which has a 1 among the digits that were read is reconstructed at the
 *     mean of its unread digits: it gets floor((1 - (-2)^d) / 6) added, the
 *     mean of sum_{j<d} b_j (-2)^j over equally likely digits b_j (the paper
 *     fixes only the rate, Sec. 5; filling the unread digits with zeros
 *     instead leaves a bias that piles up over repeated re-encodes).
 *     Coefficients with no 1 read stay 0.
 *  8. Reconstruction: v = ldexp((float)q, Eb - 153), (float) rounding to
 *     nearest even, IEEE gradual underflow.
 */
#include "ocref.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* floor shift of a signed 32-bit value, written so it does not rely on the
 * implementation-defined behaviour of >> on negative operands */
static int32_t asr(int32_t x, int s) { return x >= 0 ? (x >> s) : ~((~x) >> s); }
/* wrapping add / subtract mod 2^32 */
static int32_t wadd(int32_t a, int32_t b) { return (int32_t)((uint32_t)a + (uint32_t)b); }
static int32_t wsub(int32_t a, int32_t b) { return (int32_t)((uint32_t)a - (uint32_t)b); }

/* ---- step 4: transform ------------------------------------------------- */
/* Forward transform of one line (a, b, c, d) = (x0, x1, x2, x3).  Without the
 * floors the five steps compute, with s = x0 + x1 + x2 + x3:
 *   after 1: a = (x0 + x3)/2, d = (x3 - x0)/2
 *   after 2: c = (x1 + x2)/2, b = (x1 - x2)/2
 *   after 3: a = s/4,         c = (x1 + x2 - x0 - x3)/4
 *   after 4: d = (x3 - x0 + x1 - x2)/4, b = (x0 + x1 - x2 - x3)/4
 *   after 5: d = d + b/2 = (-2x0 + 6x1 - 6x2 + 2x3)/16,
 *            b = b - d/2 = (5x0 + x1 - x2 - 5x3)/16
 * so (a, b, c, d) are rows 1, 2, 3 and 4 of A applied to the line. */
static void lift_fwd(int32_t *a, int32_t *b, int32_t *c, int32_t *d) {
  int32_t x0 = *a, x1 = *b, x2 = *c, x3 = *d;
  x0 = asr(wadd(x0, x3), 1); x3 = wsub(x3, x0);        /* 1: outer pair */
  x2 = asr(wadd(x2, x1), 1); x1 = wsub(x1, x2);        /* 2: inner pair */
  x0 = asr(wadd(x0, x2), 1); x2 = wsub(x2, x0);        /* 3: the two means */
  x3 = asr(wadd(x3, x1), 1); x1 = wsub(x1, x3);        /* 4: the two differences */
  x3 = wadd(x3, asr(x1, 1)); x1 = wsub(x1, asr(x3, 1)); /* 5: shear of the differences */
  *a = x0; *b = x1; *c = x2; *d = x3;
}
/* Inverse: each step undone, in reverse order.  Step 5 is a pair of shears and
 * is undone exactly; steps 1-4 replace (u, v) by (m, v - m) with m = (u + v) >> 1,
 * undone as v = (v - m) + m, u = 2m - v (exact when u + v is even). */
static void lift_inv(int32_t *a, int32_t *b, int32_t *c, int32_t *d) {
  int32_t x0 = *a, x1 = *b, x2 = *c, x3 = *d;
  x1 = wadd(x1, asr(x3, 1)); x3 = wsub(x3, asr(x1, 1)); /* 5 */
  x1 = wadd(x1, x3); x3 = wsub(wadd(x3, x3), x1);       /* 4 */
  x2 = wadd(x2, x0); x0 = wsub(wadd(x0, x0), x2);       /* 3 */
  x1 = wadd(x1, x2); x2 = wsub(wadd(x2, x2), x1);       /* 2 */
  x3 = wadd(x3, x0); x0 = wsub(wadd(x0, x0), x3);       /* 1 */
  *a = x0; *b = x1; *c = x2; *d = x3;
}
static int tix(int i, int j, int k) { return i + 4 * j + 16 * k; }

void ocref_fwd_lift_line(int32_t *x) { lift_fwd(&x[0], &x[1], &x[2], &x[3]); }
void ocref_inv_lift_line(int32_t *x) { lift_inv(&x[0], &x[1], &x[2], &x[3]); }

void ocref_fwd_xform(int32_t *q) {
  for (int k = 0; k < 4; k++)           /* along x */
    for (int j = 0; j < 4; j++)
      lift_fwd(&q[tix(0, j, k)], &q[tix(1, j, k)], &q[tix(2, j, k)], &q[tix(3, j, k)]);
  for (int k = 0; k < 4; k++)           /* along y */
    for (int i = 0; i < 4; i++)
      lift_fwd(&q[tix(i, 0, k)], &q[tix(i, 1, k)], &q[tix(i, 2, k)], &q[tix(i, 3, k)]);
  for (int j = 0; j < 4; j++)           /* along z */
    for (int i = 0; i < 4; i++)
      lift_fwd(&q[tix(i, j, 0)], &q[tix(i, j, 1)], &q[tix(i, j, 2)], &q[tix(i, j, 3)]);
}
void ocref_inv_xform(int32_t *q) {
  for (int j = 0; j < 4; j++)           /* z first: reverse order of the forward */
    for (int i = 0; i < 4; i++)
      lift_inv(&q[tix(i, j, 0)], &q[tix(i, j, 1)], &q[tix(i, j, 2)], &q[tix(i, j, 3)]);
  for (int k = 0; k < 4; k++)
    for (int i = 0; i < 4; i++)
      lift_inv(&q[tix(i, 0, k)], &q[tix(i, 1, k)], &q[tix(i, 2, k)], &q[tix(i, 3, k)]);
  for (int k = 0; k < 4; k++)
    for (int j = 0; j < 4; j++)
      lift_inv(&q[tix(0, j, k)], &q[tix(1, j, k)], &q[tix(2, j, k)], &q[tix(3, j, k)]);
}

/* ---- step 5: sequency order (plain insertion sort on the key) ----------- */
static long seq_key(int t) {
  int i = t & 3, j = (t >> 2) & 3, k = t >> 4;
  return (long)(i + j + k) * 100000 + (long)(i * i + j * j + k * k) * 100 + t;
}
void ocref_sequency_order(int *perm) {
  for (int t = 0; t < 64; t++) perm[t] = t;
  for (int a = 1; a < 64; a++) {
    int v = perm[a], b = a - 1;
    while (b >= 0 && seq_key(perm[b]) > seq_key(v)) { perm[b + 1] = perm[b]; b--; }
    perm[b + 1] = v;
  }
}

/* ---- step 6: negabinary ------------------------------------------------ */
uint32_t ocref_to_negabinary(int32_t c) { return ((uint32_t)c + 0xAAAAAAAAu) ^ 0xAAAAAAAAu; }
int32_t ocref_from_negabinary(uint32_t u) { return (int32_t)((u ^ 0xAAAAAAAAu) - 0xAAAAAAAAu); }

/* ---- steps 2 and 3: block floating point ------------------------------- */
int ocref_quantize(const float *v, int32_t *q, int *Eb_out) {
  uint32_t sgn[64], Ee[64], M[64];
  uint32_t Eb = 0;
  for (int t = 0; t < 64; t++) {
    uint32_t bits;
    memcpy(&bits, &v[t], 4);
    uint32_t E = (bits >> 23) & 255u, F = bits & 0x7FFFFFu;
    if (E == 255u) return OCREF_ERR_NONFINITE;
    sgn[t] = bits >> 31;
    Ee[t] = E > 1u ? E : 1u;
    M[t] = E > 0u ? (F | 0x800000u) : F;
    if (Ee[t] > Eb) Eb = Ee[t];
  }
  for (int t = 0; t < 64; t++) {
    uint32_t sh = Eb - Ee[t];
    uint32_t mag = sh >= 27u ? 0u : ((M[t] << 3) >> sh);
    q[t] = sgn[t] ? -(int32_t)mag : (int32_t)mag;
  }
  *Eb_out = (int)Eb;
  return OCREF_OK;
}

/* ---- bit I/O ----------------------------------------------------------- */
typedef struct { uint8_t *buf; int64_t pos, cap; } bitw_t;
static void put_bit(bitw_t *w, unsigned b) {
  if (w->pos < w->cap && b) w->buf[w->pos >> 3] |= (uint8_t)(1u << (w->pos & 7));
  w->pos++;   /* keeps counting past the budget so callers learn the full length */
}
typedef struct { const uint8_t *buf; int64_t pos, cap; } bitr_t;
/* returns 0/1, or -1 when the budget is spent */
static int get_bit(bitr_t *r) {
  if (r->pos >= r->cap) return -1;
  int b = (r->buf[r->pos >> 3] >> (r->pos & 7)) & 1;
  r->pos++;
  return b;
}

/* ---- step 7: embedded coding ------------------------------------------- */
/* For plane p the plane word x has bit q = bit p of u[q].  With n = number of
 * coefficients already known to be significant (initially 0):
 *   (i)  the first n bits of x are sent verbatim;
 *   (ii) while n < 64: send g = (some bit of x at position >= n is set); stop
 *        the plane if g is 0; otherwise send bits of x from position n upward,
 *        advancing n after each, until a 1 has been sent.
 * There is no implied final bit. */
static void encode_planes(const uint32_t *u, bitw_t *w) {
  int n = 0;
  for (int p = 31; p >= 0; p--) {
    for (int q = 0; q < n; q++) put_bit(w, (u[q] >> p) & 1u);
    while (n < 64) {
      int g = 0;
      for (int q = n; q < 64; q++) g |= (int)((u[q] >> p) & 1u);
      put_bit(w, (unsigned)g);
      if (!g) break;
      for (;;) {
        unsigned b = (u[n] >> p) & 1u;
        put_bit(w, b);
        n++;
        if (b) break;
      }
    }
  }
}
/* mirror of encode_planes; stops at the budget, leaving unread bits 0 */
/* Decodes the planes into u; low[q] receives the lowest plane whose digit of
 * coefficient q is known (32 = none): read verbatim or in a run, or known to
 * be 0 from a closing group bit. */
static void decode_planes(uint32_t *u, int *low, bitr_t *r) {
  int n = 0;
  memset(u, 0, 64 * sizeof(uint32_t));
  for (int q = 0; q < 64; q++) low[q] = 32;
  for (int p = 31; p >= 0; p--) {
    for (int q = 0; q < n; q++) {
      int b = get_bit(r);
      if (b < 0) return;
      u[q] |= (uint32_t)b << p;
      low[q] = p;
    }
    while (n < 64) {
      int g = get_bit(r);
      if (g < 0) return;
      if (!g) break;
      for (;;) {
        int b = get_bit(r);
        if (b < 0) return;
        u[n] |= (uint32_t)b << p;
        low[n] = p;
        n++;
        if (b) break;
        /* a run that passes the last coefficient without its closing 1 is
         * never written by the encoder; such a stream ends here, as if the
         * budget had cut it */
        if (n == 64) return;
      }
    }
    for (int q = n; q < 64; q++) low[q] = p;   /* closed by a group bit 0 (or n == 64) */
  }
}

/* floor((1 - (-2)^d) / 6): the mean of d unread negabinary digits, rounded down */
int32_t ocref_unread_mean(int d) {
  const int64_t pw = (int64_t)1 << d;
  const int64_t num = 1 - ((d & 1) ? -pw : pw);
  return (int32_t)(num >= 0 ? num / 6 : -((-num + 5) / 6));
}

/* ---- whole block -------------------------------------------------------- */
int ocref_block_encode(const float *v, int R, uint8_t *slot, int64_t *full_bits) {
  if (R < 1 || R > 32) return OCREF_ERR_ARG;
  int32_t q[64];
  int Eb;
  int st = ocref_quantize(v, q, &Eb);                  /* steps 2-3 */
  if (st) return st;
  ocref_fwd_xform(q);                                  /* step 4 */
  int perm[64];
  ocref_sequency_order(perm);                          /* step 5 */
  uint32_t u[64];
  for (int p = 0; p < 64; p++) u[p] = ocref_to_negabinary(q[perm[p]]);   /* step 6 */
  memset(slot, 0, (size_t)8 * R);
  bitw_t w = {slot, 0, (int64_t)64 * R};
  for (int b = 0; b < 8; b++) put_bit(&w, ((unsigned)Eb >> b) & 1u);     /* header */
  encode_planes(u, &w);                                /* step 7 */
  if (full_bits) *full_bits = w.pos;
  return OCREF_OK;
}

int ocref_block_decode(const uint8_t *slot, int R, float *v) {
  if (R < 1 || R > 32) return OCREF_ERR_ARG;
  bitr_t r = {slot, 0, (int64_t)64 * R};
  int Eb = 0;
  for (int b = 0; b < 8; b++) Eb |= get_bit(&r) << b;
  uint32_t u[64];
  int low[64];
  decode_planes(u, low, &r);
  int perm[64];
  ocref_sequency_order(perm);
  int32_t q[64];
  for (int p = 0; p < 64; p++) {
    int32_t c = ocref_from_negabinary(u[p]);
    if (u[p] != 0 && low[p] > 0 && low[p] < 32)   /* step 7' */
      c = (int32_t)((uint32_t)c + (uint32_t)ocref_unread_mean(low[p]));
    q[perm[p]] = c;
  }
  ocref_inv_xform(q);
  for (int t = 0; t < 64; t++) v[t] = ldexpf((float)q[t], Eb - 153);   /* step 8 */
  return OCREF_OK;
}

/* ---- whole field: block (bx,by,bz) -> slot (bz*(ny/4) + by)*(nx/4) + bx -- */
static int field_ok(int64_t nx, int64_t ny, int64_t nz, int R) {
  if (nx <= 0 || ny <= 0 || nz <= 0 || R < 1 || R > 32) return OCREF_ERR_ARG;
  if (nx % 4 || ny % 4 || nz % 4) return OCREF_ERR_SHAPE;
  return OCREF_OK;
}
int ocref_compress(const float *f, int64_t nx, int64_t ny, int64_t nz, int R, uint8_t *out) {
  int st = field_ok(nx, ny, nz, R);
  if (st) return st;
  int64_t bx_n = nx / 4, by_n = ny / 4, bz_n = nz / 4;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t bz = 0; bz < bz_n; bz++)
    for (int64_t by = 0; by < by_n; by++)
      for (int64_t bx = 0; bx < bx_n; bx++) {
        float v[64];
        for (int k = 0; k < 4; k++)
          for (int j = 0; j < 4; j++)
            for (int i = 0; i < 4; i++)
              v[tix(i, j, k)] = f[((4 * bz + k) * ny + 4 * by + j) * nx + 4 * bx + i];
        int64_t b = (bz * by_n + by) * bx_n + bx;
        if (ocref_block_encode(v, R, out + b * 8 * R, NULL)) bad = 1;
      }
  return bad ? OCREF_ERR_NONFINITE : OCREF_OK;
}
int ocref_decompress(const uint8_t *in, int64_t nx, int64_t ny, int64_t nz, int R, float *f) {
  int st = field_ok(nx, ny, nz, R);
  if (st) return st;
  int64_t bx_n = nx / 4, by_n = ny / 4, bz_n = nz / 4;
#pragma omp parallel for schedule(static)
  for (int64_t bz = 0; bz < bz_n; bz++)
    for (int64_t by = 0; by < by_n; by++)
      for (int64_t bx = 0; bx < bx_n; bx++) {
        float v[64];
        int64_t b = (bz * by_n + by) * bx_n + bx;
        ocref_block_decode(in + b * 8 * R, R, v);
        for (int k = 0; k < 4; k++)
          for (int j = 0; j < 4; j++)
            for (int i = 0; i < 4; i++)
              f[((4 * bz + k) * ny + 4 * by + j) * nx + 4 * bx + i] = v[tix(i, j, k)];
      }
  return OCREF_OK;
}
