/* Drives the oracle's C code over the inputs its tests use and over edge
 * cases (every rate, special blocks, arbitrary byte strings, tiny and
 * ragged grids), for a build with AddressSanitizer and UndefinedBehavior-
 * Sanitizer: the codec's shift guards and wrapping integer arithmetic, and the
 * stencils' index arithmetic, must stay defined.  Exit status 0 = clean. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ocref.h"

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t next_u64(void) {   /* splitmix64 */
  uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static double uniform(void) { return (double)(next_u64() >> 11) * (1.0 / 9007199254740992.0); }

static int fail(const char *what) {
  fprintf(stderr, "oracle_drive: %s\n", what);
  return 1;
}

static void block_kinds(int kind, float *v) {
  for (int t = 0; t < 64; t++) {
    switch (kind) {
      case 0: v[t] = 0.0f; break;                                  /* zero */
      case 1: v[t] = 1.5f; break;                                  /* constant */
      case 2: v[t] = 1e-40f; break;                                /* subnormal constant */
      case 3: v[t] = (float)(2.0 * uniform() - 1.0); break;        /* random */
      case 4: v[t] = (t & 1) ? 3.0e38f : -3.0e38f; break;          /* extremes */
      case 5: v[t] = (float)ldexp(2.0 * uniform() - 1.0, (int)(next_u64() % 250) - 125); break;
      case 6: v[t] = (t == 17) ? 1.0f : 1e-30f; break;             /* wide exponent range */
      default: v[t] = (float)sin(0.3 * t) + 5.0f; break;           /* smooth, offset */
    }
  }
}

int main(void) {
  /* codec: every rate, every block kind, round trips and byte strings */
  for (int R = 1; R <= 32; R++) {
    uint8_t slot[8 * 32 + 8];
    float v[64], w[64];
    for (int kind = 0; kind < 8; kind++) {
      block_kinds(kind, v);
      int64_t full = 0;
      if (ocref_block_encode(v, R, slot, &full) != OCREF_OK) return fail("encode");
      if (ocref_block_decode(slot, R, w) != OCREF_OK) return fail("decode");
    }
    for (int rep = 0; rep < 200; rep++) {
      for (int b = 0; b < 8 * R; b++) slot[b] = (uint8_t)next_u64();
      (void)ocref_block_decode(slot, R, w);
    }
  }
  int32_t q[64];
  for (int rep = 0; rep < 100; rep++) {
    for (int t = 0; t < 64; t++) q[t] = (int32_t)(uint32_t)next_u64();   /* full-range words */
    ocref_fwd_xform(q);
    ocref_inv_xform(q);
    for (int t = 0; t < 64; t++) (void)ocref_from_negabinary(ocref_to_negabinary(q[t]));
  }
  for (int d = 0; d <= 31; d++) (void)ocref_unread_mean(d);
  int perm[64];
  ocref_sequency_order(perm);
  {
    float v[64];
    int Eb = 0;
    for (int kind = 0; kind < 8; kind++) {
      block_kinds(kind, v);
      (void)ocref_quantize(v, q, &Eb);
    }
  }
  /* compress / decompress of ragged small fields */
  const int64_t dims[][3] = {{4, 4, 4}, {8, 12, 16}, {20, 8, 4}};
  for (size_t di = 0; di < sizeof dims / sizeof dims[0]; di++) {
    const int64_t nx = dims[di][0], ny = dims[di][1], nz = dims[di][2], n = nx * ny * nz;
    float *f = malloc((size_t)n * 4), *g = malloc((size_t)n * 4);
    uint8_t *c = malloc((size_t)(n / 64) * 8 * 32);
    for (int64_t i = 0; i < n; i++) f[i] = (float)(2.0 * uniform() - 1.0);
    for (int R = 1; R <= 32; R += 5) {
      if (ocref_compress(f, nx, ny, nz, R, c) != OCREF_OK) return fail("compress");
      if (ocref_decompress(c, nx, ny, nz, R, g) != OCREF_OK) return fail("decompress");
    }
    f[n / 2] = NAN;
    if (ocref_compress(f, nx, ny, nz, 8, c) != OCREF_ERR_NONFINITE) return fail("nonfinite flag");
    if (ocref_compress(f, nx + 1, ny, nz, 8, c) == OCREF_OK) return fail("shape check");
    free(f);
    free(g);
    free(c);
  }
  /* stencils and gradients on tiny and ragged grids */
  const int64_t sg[][3] = {{1, 1, 1}, {3, 5, 7}, {8, 8, 8}, {9, 4, 2}};
  const double cs[7] = {0.4, 0.1, 0.1, 0.1, 0.1, 0.1, 0.1};
  for (size_t gi = 0; gi < sizeof sg / sizeof sg[0]; gi++) {
    const int64_t nx = sg[gi][0], ny = sg[gi][1], nz = sg[gi][2], n = nx * ny * nz;
    double *u = malloc((size_t)n * 8), *o = malloc((size_t)n * 8), *c0 = malloc((size_t)n * 8);
    double *uT = malloc((size_t)n * 8), *gu = malloc((size_t)n * 8), *gc = malloc((size_t)n * 8);
    double L = 0.0;
    for (int64_t i = 0; i < n; i++) {
      u[i] = uniform();
      c0[i] = 0.3 + 0.2 * uniform();
    }
    ocref_star7_step(u, o, nx, ny, nz, cs, NULL);
    ocref_star7_step_T(u, o, nx, ny, nz, cs, c0);
    if (ocref_star7_run(u, nx, ny, nz, cs, c0, 3) != OCREF_OK) return fail("star7_run");
    if (ocref_star7_grad(u, nx, ny, nz, cs, c0, 4, uT, gu, gc, &L) != OCREF_OK) return fail("grad");
    double *pp = malloc((size_t)n * 8), *pc = malloc((size_t)n * 8), *vel = malloc((size_t)n * 8);
    for (int64_t i = 0; i < n; i++) {
      pp[i] = 0.0;
      pc[i] = 1e-3 * uniform();
      vel[i] = 1500.0 + 3000.0 * uniform();
    }
    const int64_t src[3] = {nx / 2, ny / 2, nz / 2};
    if (ocref_wave25_run(pp, pc, vel, nx, ny, nz, 10.0, 8e-4, src, 15.0, 1.0 / 15.0, 0, 5) != OCREF_OK)
      return fail("wave25_run");
    free(u); free(o); free(c0); free(uT); free(gu); free(gc); free(pp); free(pc); free(vel);
  }
  puts("oracle_drive: clean");
  return 0;
}
