"""Seeded synthetic inputs (shared by the tests, the benchmark and the smoke check).

This module holds no arithmetic of the method itself: it only draws fields with
the shapes and value distributions of the workloads.  The paper's own data (an
acoustic-wave velocity model of (1152+8)^3 doubles, Sec. 6, Table 1) is not
available, so these stand in for it.

Recipes:
* `modes_field`     -- sum of products of sines sin(pi m (i+1)/(N+1)) with integer
  wavenumbers m in 1..4 and amplitudes U(0.5, 1), plus uniform noise; built in
  FP64, returned FP32.
* `grf_field`       -- Gaussian random field with 3-D power spectral density
  P(|k|) ~ |k|^-3 (amplitude ~ |k|^-1.5) on the periodic box, k = 0 removed,
  normalised to zero mean and unit standard deviation.  FP32 white noise is
  filtered with single-precision real FFTs (scipy.fft, multithreaded).
* `c0_field`        -- 0.4 + 0.1 g/max|g|, g a sum of 8 seeded separable sines
  with wavenumbers 1..3: a smooth field in [0.3, 0.5].
* `layered_velocity` -- 5 layers (1500, 2250, 3000, 3750, 4500 m/s) with depth,
  interfaces at nz*l/5 perturbed by 3 smooth seeded sines of amplitude nz/40.
"""
from __future__ import annotations

import os

import numpy as np


def modes_field(shape, n_modes: int = 4, seed: int = 1, noise: float = 1e-3,
                return_modes: bool = False):
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    f = np.zeros((nz, ny, nx))
    modes = []
    for _ in range(n_modes):
        mx, my, mz = (int(v) for v in rng.integers(1, 5, size=3))
        a = float(rng.uniform(0.5, 1.0))
        modes.append(((mx, my, mz), a))
        f += a * (np.sin(np.pi * mx * (x + 1) / (nx + 1)) * np.sin(np.pi * my * (y + 1) / (ny + 1))
                  * np.sin(np.pi * mz * (z + 1) / (nz + 1)))
    if noise:
        f += rng.uniform(-noise, noise, size=(nz, ny, nx))
    out = f.astype(np.float32)
    return (out, modes) if return_modes else out


def single_mode(shape, m, amp: float = 1.0) -> np.ndarray:
    """One product-of-sines mode in FP64 (an eigenvector of the zero-ghost star)."""
    nz, ny, nx = shape
    mx, my, mz = m
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    return amp * (np.sin(np.pi * mx * (x + 1) / (nx + 1)) * np.sin(np.pi * my * (y + 1) / (ny + 1))
                  * np.sin(np.pi * mz * (z + 1) / (nz + 1)))


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def grf_field(shape, seed: int = 2, slope: float = -3.0) -> np.ndarray:
    import scipy.fft as sfft

    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((nz, ny, nx), dtype=np.float32)
    W = sfft.rfftn(w, workers=_workers())
    del w
    kz = (np.fft.fftfreq(nz) * nz).astype(np.float32)[:, None, None]
    ky = (np.fft.fftfreq(ny) * ny).astype(np.float32)[None, :, None]
    kx = (np.fft.rfftfreq(nx) * nx).astype(np.float32)[None, None, :]
    # amplitude |k|^(slope/2) applied plane by plane to bound temporary memory
    for iz in range(nz):
        k2 = kz[iz] ** 2 + ky[0] ** 2 + kx[0] ** 2
        k2[k2 == 0] = np.inf
        W[iz] *= (k2 ** np.float32(slope / 4.0)).astype(np.float32)
    f = sfft.irfftn(W, s=(nz, ny, nx), workers=_workers())
    del W
    f = f.astype(np.float32, copy=False)
    m = float(f.mean(dtype=np.float64))
    s = float(f.std(dtype=np.float64))
    f -= np.float32(m)
    f *= np.float32(1.0 / s)
    return f


def c0_field(shape, seed: int = 5, lo: float = 0.3, hi: float = 0.5) -> np.ndarray:
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    z = np.arange(nz, dtype=np.float64)[:, None, None] / nz
    y = np.arange(ny, dtype=np.float64)[None, :, None] / ny
    x = np.arange(nx, dtype=np.float64)[None, None, :] / nx
    g = np.zeros((nz, ny, nx))
    for _ in range(8):
        kx, ky, kz = (int(v) for v in rng.integers(1, 4, size=3))
        ph = rng.uniform(0, 2 * np.pi, size=3)
        a = rng.uniform(0.5, 1.0)
        g += a * (np.sin(2 * np.pi * kx * x + ph[0]) * np.sin(2 * np.pi * ky * y + ph[1])
                  * np.sin(2 * np.pi * kz * z + ph[2]))
    mid, half = 0.5 * (lo + hi), 0.5 * (hi - lo)
    return (mid + half * g / np.abs(g).max()).astype(np.float32)


def smooth_direction(shape, rng) -> np.ndarray:
    """A smooth random perturbation direction (same construction as c0_field's g)."""
    nz, ny, nx = shape
    z = np.arange(nz, dtype=np.float64)[:, None, None] / nz
    y = np.arange(ny, dtype=np.float64)[None, :, None] / ny
    x = np.arange(nx, dtype=np.float64)[None, None, :] / nx
    g = np.zeros((nz, ny, nx))
    for _ in range(8):
        kx, ky, kz = (int(v) for v in rng.integers(1, 4, size=3))
        ph = rng.uniform(0, 2 * np.pi, size=3)
        g += (np.sin(2 * np.pi * kx * x + ph[0]) * np.sin(2 * np.pi * ky * y + ph[1])
              * np.sin(2 * np.pi * kz * z + ph[2]))
    return g


def layered_velocity(shape, seed: int = 4, speeds=(1500.0, 2250.0, 3000.0, 3750.0, 4500.0)):
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    y = np.arange(ny, dtype=np.float64)[:, None] / ny
    x = np.arange(nx, dtype=np.float64)[None, :] / nx
    pert = np.zeros((ny, nx))
    for _ in range(3):
        kx, ky = (int(v) for v in rng.integers(1, 4, size=2))
        ph = rng.uniform(0, 2 * np.pi, size=2)
        pert += np.sin(2 * np.pi * kx * x + ph[0]) * np.sin(2 * np.pi * ky * y + ph[1])
    pert *= (nz / 40.0) / max(np.abs(pert).max(), 1e-30)
    nl = len(speeds)
    v = np.empty((nz, ny, nx), dtype=np.float32)
    zc = np.arange(nz, dtype=np.float64)
    for iz in range(nz):
        # layer index = number of interfaces (nz*l/nl + pert) at or above this depth
        layer = np.zeros((ny, nx), dtype=np.int64)
        for l in range(1, nl):
            layer += (zc[iz] >= nz * l / nl + pert).astype(np.int64)
        v[iz] = np.asarray(speeds, dtype=np.float32)[layer]
    return v
