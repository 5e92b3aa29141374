"""Dense-matrix brute force for tiny grids (TEST INFRASTRUCTURE ONLY).

Builds the 7-point stencil operator of Sec. 3.1 as an explicit n x n matrix by
enumerating, for every cell, its neighbours inside the grid (zero ghosts are
simply absent entries).  Used to pin the C oracle: powers of the matrix, its
transpose, and gradients by the product rule, all in FP64 numpy.
"""
from __future__ import annotations

import numpy as np

# neighbour offsets (dx, dy, dz) in coefficient order c-x, c+x, c-y, c+y, c-z, c+z
_OFFS = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]


def dense_star7(nx: int, ny: int, nz: int, c, c0f=None) -> np.ndarray:
    n = nx * ny * nz
    A = np.zeros((n, n))
    c = np.asarray(c, dtype=np.float64)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                row = (z * ny + y) * nx + x
                A[row, row] = c[0] if c0f is None else float(np.asarray(c0f)[z, y, x])
                for d, (dx, dy, dz) in enumerate(_OFFS):
                    xx, yy, zz = x + dx, y + dy, z + dz
                    if 0 <= xx < nx and 0 <= yy < ny and 0 <= zz < nz:
                        A[row, (zz * ny + yy) * nx + xx] = c[1 + d]
    return A


def top_plane_mask(nx: int, ny: int, nz: int) -> np.ndarray:
    m = np.zeros((nz, ny, nx))
    m[nz - 1] = 1.0
    return m.reshape(-1)


def grad_brute(u0, c, steps: int, c0f):
    """L, dL/du0, dL/dc0 for L = 1/2 |P A^s u0|^2 with explicit matrices.

    dL/du0 = (A^s)^T P A^s u0.  For c0 at cell x, dA/dc0(x) = E_xx, so
    d(A^s)/dc0(x) = sum_{n} A^{s-1-n} E_xx A^n and
    dL/dc0(x) = sum_n (A^{s-1-n})^T P u_T)[x] * (A^n u0)[x].
    """
    nz, ny, nx = np.asarray(u0).shape
    A = dense_star7(nx, ny, nz, c, c0f)
    u = np.asarray(u0, dtype=np.float64).reshape(-1)
    P = top_plane_mask(nx, ny, nz)
    pows = [np.eye(A.shape[0])]
    for _ in range(steps):
        pows.append(A @ pows[-1])
    uT = pows[steps] @ u
    r = P * uT
    L = 0.5 * float(r @ r)
    g_u0 = pows[steps].T @ r
    g_c0 = np.zeros_like(u)
    for n in range(steps):
        g_c0 += (pows[steps - 1 - n].T @ r) * (pows[n] @ u)
    return L, uT.reshape(nz, ny, nx), g_u0.reshape(nz, ny, nx), g_c0.reshape(nz, ny, nx)
