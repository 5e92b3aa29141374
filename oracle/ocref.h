/*
 * ocref.h -- the CPU oracle for compressed out-of-core stencil sweeps.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this code; only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It shares no source, header, table or helper with
 * the HIP path.
 *
 * Everything here is a plain, slow, obviously-correct restatement of what the
 * method computes (Shen et al., "Compression-Based Optimizations for Out-of-Core
 * GPU Stencil Computation"):
 *   - the stencil update of Sec. 3.1 (a point updated from itself and its halo),
 *     as a 7-point star and as the 25-point order-8 acoustic-wave update used in
 *     the experiments of Sec. 6;
 *   - the adjoint (transpose) of the 7-point update and the gradients of a
 *     quadratic loss, for the differentiation extension;
 *   - a fixed-rate block-transform codec (the paper uses a fixed-rate GPU
 *     compressor at a user-specified rate, Sec. 4.2 and Sec. 5, but does not
 *     define its format; this codec is our own reading, stated step by step in
 *     codec_ref.c).
 * Floating point is FP64 throughout, except the codec which by definition maps
 * FP32 values to bits and back.
 *
 * All arrays are C order [nz][ny][nx] (x fastest).  Ghost cells outside the
 * grid are zero (zero Dirichlet boundary).
 */
#ifndef OCREF_H
#define OCREF_H
#include <stdint.h>

#define OCREF_OK            0
#define OCREF_ERR_ARG      -1
#define OCREF_ERR_SHAPE    -2
#define OCREF_ERR_NONFINITE -5

/* ---- 7-point star stencil (Sec. 3.1) ---------------------------------- */
/* c[7] = c0, c_-x, c_+x, c_-y, c_+y, c_-z, c_+z.  c0f (nullable) overrides c0
 * per cell.  out = A u. */
void ocref_star7_step(const double *u, double *out, int64_t nx, int64_t ny, int64_t nz,
                      const double *c, const double *c0f);
/* out = A^T lam  (the transpose swaps the -/+ neighbour coefficients). */
void ocref_star7_step_T(const double *lam, double *out, int64_t nx, int64_t ny, int64_t nz,
                        const double *c, const double *c0f);
/* u <- A^steps u, in place. */
int ocref_star7_run(double *u, int64_t nx, int64_t ny, int64_t nz, const double *c,
                    const double *c0f, int64_t steps);
/* Loss L = 1/2 sum over the top plane z = nz-1 of u_T^2 with u_T = A^steps u0.
 * Writes u_T, dL/du0, dL/dc0 (per cell) and L.  Stores every u_n. */
int ocref_star7_grad(const double *u0, int64_t nx, int64_t ny, int64_t nz, const double *c,
                     const double *c0f, int64_t steps, double *uT, double *g_u0,
                     double *g_c0, double *loss);

/* ---- 25-point order-8 acoustic wave (Sec. 6 workload) ------------------ */
/* Advances (p_prev, p_cur) = (p^{n0-1}, p^{n0}) by `steps` leapfrog steps.
 * vel in m/s, h grid spacing (m), dt (s); Ricker source of peak frequency
 * f_peak (Hz) delayed by t0 (s) at cell src = (x, y, z). */
int ocref_wave25_run(double *p_prev, double *p_cur, const double *vel, int64_t nx,
                     int64_t ny, int64_t nz, double h, double dt, const int64_t *src,
                     double f_peak, double t0, int64_t n0, int64_t steps);
double ocref_ricker(double t, double f_peak, double t0);

/* ---- fixed-rate block codec ------------------------------------------- */
/* One 4x4x4 block, values v[t], t = i + 4j + 16k.  slot = 8*R bytes.
 * *full_bits (nullable) receives the length the stream would have without a
 * budget (header included). */
int ocref_block_encode(const float *v, int R, uint8_t *slot, int64_t *full_bits);
int ocref_block_decode(const uint8_t *slot, int R, float *v);
int ocref_compress(const float *f, int64_t nx, int64_t ny, int64_t nz, int R, uint8_t *out);
int ocref_decompress(const uint8_t *in, int64_t nx, int64_t ny, int64_t nz, int R, float *f);
/* sub-steps, exported so that tests can pin each one */
void ocref_fwd_xform(int32_t *q);
void ocref_inv_xform(int32_t *q);
/* the transform of one line of four integers, forward and inverse */
void ocref_fwd_lift_line(int32_t *x);
void ocref_inv_lift_line(int32_t *x);
uint32_t ocref_to_negabinary(int32_t c);
int32_t ocref_from_negabinary(uint32_t u);
/* floor((1 - (-2)^d) / 6), 0 <= d <= 31: the value added at decode to a
 * significant coefficient whose d lowest digits were not read (step 7') */
int32_t ocref_unread_mean(int d);
void ocref_sequency_order(int *perm);
int ocref_quantize(const float *v, int32_t *q, int *Eb);

/* Host threads the OpenMP loops use from the calling thread on; n <= 0 leaves
 * the count as it is.  Returns the previous count.  (Timing only.) */
int ocref_set_threads(int n);

#endif
