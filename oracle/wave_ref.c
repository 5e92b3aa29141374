/*
 * wave_ref.c -- FP64 reference of the 25-point order-8 acoustic wave update.
 *
 * TEST INFRASTRUCTURE ONLY (see ocref.h).  Independent of the HIP path.
 *
 * The experiments (Sec. 6, Table 1) run an acoustic wave propagation code with
 * a 25-point stencil whose halo is 4 cells: the star of radius 4 in 3-D.  The
 * paper gives neither the scheme nor the source; the reading used here is the
 * standard second-order-in-time leapfrog with eighth-order central second
 * derivatives:
 *   p^{n+1} = 2 p^n - p^{n-1} + (v dt / h)^2 L8(p^n),
 *   L8(p)[x] = sum over the three axes of sum_{j=-4..4} w_|j| p[x + j e_axis],
 *   w = (-205/72, 8/5, -1/5, 8/315, -1/560)   (centre weight counted per axis),
 * then a Ricker wavelet is added at the source cell:
 *   p^{n+1}[src] += (v_src dt / h)^2 rho(n dt),
 *   rho(t) = (1 - 2 pi^2 f^2 tau^2) exp(-pi^2 f^2 tau^2),  tau = t - t0.
 * Zero ghosts outside the grid; p^0 = p^{-1} = 0 unless the caller says otherwise.
 */
#include "ocref.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

static const double W8[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};

double ocref_ricker(double t, double f_peak, double t0) {
  const double pi = 3.14159265358979323846;
  double a = pi * f_peak * (t - t0);
  a = a * a;
  return (1.0 - 2.0 * a) * exp(-a);
}

static double at(const double *u, int64_t nx, int64_t ny, int64_t nz, int64_t x, int64_t y,
                 int64_t z) {
  if (x < 0 || y < 0 || z < 0 || x >= nx || y >= ny || z >= nz) return 0.0;
  return u[(z * ny + y) * nx + x];
}

int ocref_wave25_run(double *p_prev, double *p_cur, const double *vel, int64_t nx,
                     int64_t ny, int64_t nz, double h, double dt, const int64_t *src,
                     double f_peak, double t0, int64_t n0, int64_t steps) {
  if (nx <= 0 || ny <= 0 || nz <= 0 || steps < 0 || h <= 0 || dt <= 0) return OCREF_ERR_ARG;
  int64_t n = nx * ny * nz;
  double *nxt = (double *)malloc((size_t)n * sizeof(double));
  if (!nxt) return OCREF_ERR_ARG;
  for (int64_t s = 0; s < steps; s++) {
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; z++)
      for (int64_t y = 0; y < ny; y++)
        for (int64_t x = 0; x < nx; x++) {
          int64_t i = (z * ny + y) * nx + x;
          double lap = 3.0 * W8[0] * p_cur[i];
          for (int j = 1; j <= 4; j++)
            lap += W8[j] * (at(p_cur, nx, ny, nz, x - j, y, z) + at(p_cur, nx, ny, nz, x + j, y, z) +
                            at(p_cur, nx, ny, nz, x, y - j, z) + at(p_cur, nx, ny, nz, x, y + j, z) +
                            at(p_cur, nx, ny, nz, x, y, z - j) + at(p_cur, nx, ny, nz, x, y, z + j));
          double a = vel[i] * dt / h;
          nxt[i] = 2.0 * p_cur[i] - p_prev[i] + a * a * lap;
        }
    if (src && src[0] >= 0 && src[0] < nx && src[1] >= 0 && src[1] < ny && src[2] >= 0 &&
        src[2] < nz) {
      int64_t i = (src[2] * ny + src[1]) * nx + src[0];
      double a = vel[i] * dt / h;
      nxt[i] += a * a * ocref_ricker((double)(n0 + s) * dt, f_peak, t0);
    }
    memcpy(p_prev, p_cur, (size_t)n * sizeof(double));
    memcpy(p_cur, nxt, (size_t)n * sizeof(double));
  }
  free(nxt);
  return OCREF_OK;
}
