/*
 * stencil_ref.c -- FP64 reference of the 7-point star stencil, its transpose
 * and the gradients of a quadratic loss.
 *
 * TEST INFRASTRUCTURE ONLY (see ocref.h).  Independent of the HIP path.
 *
 * The stencil update (Sec. 3.1): the new value of a point is computed from the
 * point itself and its halo neighbours, once per time step, over the whole grid.
 * Here, with zero ghosts outside the grid:
 *   (A u)[z,y,x] = c0(x) u[z,y,x] + c_-x u[z,y,x-1] + c_+x u[z,y,x+1]
 *                + c_-y u[z,y-1,x] + c_+y u[z,y+1,x] + c_-z u[z-1,y,x] + c_+z u[z+1,y,x]
 * Out-of-core decomposition and temporal blocking (Sec. 3.1) change where this
 * is evaluated, not what it evaluates, so the oracle is the plain definition.
 *
 * Transpose: (A^T l)[x] = c0(x) l[x] + sum_d c_d l[x - e_d], i.e. the -/+
 * coefficients swap and the diagonal stays.
 *
 * Gradients of L = 1/2 sum_{y,x} u_T[nz-1,y,x]^2, u_{n+1} = A u_n:
 *   lambda_T = u_T on the top plane, 0 elsewhere; lambda_n = A^T lambda_{n+1};
 *   dL/du0 = lambda_0;  dL/dc0(x) = sum_{n=0}^{T-1} lambda_{n+1}[x] u_n[x].
 */
#include "ocref.h"
#include <omp.h>
#include <stdlib.h>
#include <string.h>

int ocref_set_threads(int n) {
  const int prev = omp_get_max_threads();
  if (n > 0) omp_set_num_threads(n);
  return prev;
}

static double at(const double *u, int64_t nx, int64_t ny, int64_t nz, int64_t x, int64_t y,
                 int64_t z) {
  if (x < 0 || y < 0 || z < 0 || x >= nx || y >= ny || z >= nz) return 0.0;
  return u[(z * ny + y) * nx + x];
}

void ocref_star7_step(const double *u, double *out, int64_t nx, int64_t ny, int64_t nz,
                      const double *c, const double *c0f) {
#pragma omp parallel for schedule(static)
  for (int64_t z = 0; z < nz; z++)
    for (int64_t y = 0; y < ny; y++)
      for (int64_t x = 0; x < nx; x++) {
        int64_t i = (z * ny + y) * nx + x;
        double c0 = c0f ? c0f[i] : c[0];
        out[i] = c0 * u[i] + c[1] * at(u, nx, ny, nz, x - 1, y, z) +
                 c[2] * at(u, nx, ny, nz, x + 1, y, z) + c[3] * at(u, nx, ny, nz, x, y - 1, z) +
                 c[4] * at(u, nx, ny, nz, x, y + 1, z) + c[5] * at(u, nx, ny, nz, x, y, z - 1) +
                 c[6] * at(u, nx, ny, nz, x, y, z + 1);
      }
}

void ocref_star7_step_T(const double *l, double *out, int64_t nx, int64_t ny, int64_t nz,
                        const double *c, const double *c0f) {
#pragma omp parallel for schedule(static)
  for (int64_t z = 0; z < nz; z++)
    for (int64_t y = 0; y < ny; y++)
      for (int64_t x = 0; x < nx; x++) {
        int64_t i = (z * ny + y) * nx + x;
        double c0 = c0f ? c0f[i] : c[0];
        /* entry A[x', x] with x' = x - e_d carries c_{+d}: the neighbour at -d
         * received this cell's value through its +d coefficient */
        out[i] = c0 * l[i] + c[2] * at(l, nx, ny, nz, x - 1, y, z) +
                 c[1] * at(l, nx, ny, nz, x + 1, y, z) + c[4] * at(l, nx, ny, nz, x, y - 1, z) +
                 c[3] * at(l, nx, ny, nz, x, y + 1, z) + c[6] * at(l, nx, ny, nz, x, y, z - 1) +
                 c[5] * at(l, nx, ny, nz, x, y, z + 1);
      }
}

int ocref_star7_run(double *u, int64_t nx, int64_t ny, int64_t nz, const double *c,
                    const double *c0f, int64_t steps) {
  if (nx <= 0 || ny <= 0 || nz <= 0 || steps < 0) return OCREF_ERR_ARG;
  int64_t n = nx * ny * nz;
  double *tmp = (double *)malloc((size_t)n * sizeof(double));
  if (!tmp) return OCREF_ERR_ARG;
  for (int64_t s = 0; s < steps; s++) {
    ocref_star7_step(u, tmp, nx, ny, nz, c, c0f);
    memcpy(u, tmp, (size_t)n * sizeof(double));
  }
  free(tmp);
  return OCREF_OK;
}

int ocref_star7_grad(const double *u0, int64_t nx, int64_t ny, int64_t nz, const double *c,
                     const double *c0f, int64_t steps, double *uT, double *g_u0,
                     double *g_c0, double *loss) {
  if (nx <= 0 || ny <= 0 || nz <= 0 || steps < 0) return OCREF_ERR_ARG;
  int64_t n = nx * ny * nz;
  /* every state u_0 .. u_T */
  double *us = (double *)malloc((size_t)(steps + 1) * n * sizeof(double));
  double *lam = (double *)malloc((size_t)n * sizeof(double));
  double *tmp = (double *)malloc((size_t)n * sizeof(double));
  if (!us || !lam || !tmp) { free(us); free(lam); free(tmp); return OCREF_ERR_ARG; }
  memcpy(us, u0, (size_t)n * sizeof(double));
  for (int64_t s = 0; s < steps; s++)
    ocref_star7_step(us + s * n, us + (s + 1) * n, nx, ny, nz, c, c0f);
  const double *ut = us + steps * n;
  memcpy(uT, ut, (size_t)n * sizeof(double));
  double L = 0.0;
  memset(lam, 0, (size_t)n * sizeof(double));
  for (int64_t y = 0; y < ny; y++)
    for (int64_t x = 0; x < nx; x++) {
      int64_t i = ((nz - 1) * ny + y) * nx + x;
      L += 0.5 * ut[i] * ut[i];
      lam[i] = ut[i];
    }
  *loss = L;
  memset(g_c0, 0, (size_t)n * sizeof(double));
  for (int64_t s = steps - 1; s >= 0; s--) {
    /* lam holds lambda_{s+1}; accumulate its product with u_s, then step back */
    const double *us_s = us + s * n;
    for (int64_t i = 0; i < n; i++) g_c0[i] += lam[i] * us_s[i];
    ocref_star7_step_T(lam, tmp, nx, ny, nz, c, c0f);
    memcpy(lam, tmp, (size_t)n * sizeof(double));
  }
  memcpy(g_u0, lam, (size_t)n * sizeof(double));
  free(us); free(lam); free(tmp);
  return OCREF_OK;
}
