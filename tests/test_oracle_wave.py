"""Pins of the FP64 25-point acoustic-wave oracle (CPU only).

The eighth-order second-derivative weights are tied to exact polynomial
reproduction (L8 x^m = m(m-1) x^(m-2) for m <= 9) at cells far enough from the
faces; the time stepping to the scalar leapfrog recurrence of a Fourier mode
inside the light cone; the source to the Ricker wavelet's closed form.
"""
from fractions import Fraction

import numpy as np

import oracle

W = [Fraction(-205, 72), Fraction(8, 5), Fraction(-1, 5), Fraction(8, 315), Fraction(-1, 560)]


def test_fd8_weights_moment_conditions_exact():
    def moment(m):
        return sum(W[abs(j)] * Fraction(j) ** m for j in range(-4, 5))
    assert moment(0) == 0
    assert moment(2) == 2
    for m in (4, 6, 8):
        assert moment(m) == 0


def test_cfl_limit_from_symbol():
    sym_pi = float(W[0] + 2 * sum(W[j] * (-1) ** j for j in range(1, 5)))
    assert abs(sym_pi - (-6.5016)) < 1e-4
    courant_max = np.sqrt(4.0 / (3 * -sym_pi))
    assert abs(courant_max - 0.4529) < 1e-4
    assert 0.4 < courant_max


def _one_step(p, vel, h, dt):
    pp, pc = oracle.wave25_run(p, p, vel, h, dt, [-1, -1, -1], 15.0, 0.0, 0, 1)
    return pc


def test_polynomial_reproduction_pins_every_weight():
    n = 20
    z, y, x = np.meshgrid(*(np.arange(n, dtype=np.float64) - 9.5,) * 3, indexing="ij")
    vel = np.full((n, n, n), 1000.0)
    h, dt = 10.0, 1e-3          # a = v dt / h = 0.1
    a2 = (1000.0 * dt / h) ** 2
    for field, lap in [(x ** 2, 2.0 + 0 * x), (y ** 4 / 100, 12 * y ** 2 / 100),
                       (z ** 6 / 1e4, 30 * z ** 4 / 1e4), (x ** 8 / 1e6, 56 * x ** 6 / 1e6),
                       (x ** 3 * y ** 2, 6 * x * y ** 2 + 2 * x ** 3)]:
        # p^{n-1} = p^n = field  =>  p^{n+1} = field + a^2 L8(field)
        got = _one_step(field, vel, h, dt)
        core = (slice(4, -4),) * 3
        want = field + a2 * lap
        scale = np.abs(want[core]).max()
        assert np.abs(got[core] - want[core]).max() < 1e-12 * scale


def test_fourier_mode_follows_leapfrog_recurrence_inside_light_cone():
    n, steps = 40, 4
    kx, ky, kz = 0.7, 1.1, 0.4
    z, y, x = np.meshgrid(*(np.arange(n, dtype=np.float64),) * 3, indexing="ij")
    phi = np.cos(kx * x + ky * y + kz * z)
    v, h, dt = 2000.0, 10.0, 1.5e-3
    a2 = (v * dt / h) ** 2
    lam = sum(float(W[0]) + 2 * sum(float(W[j]) * np.cos(j * k) for j in range(1, 5))
              for k in (kx, ky, kz))
    pp, pc = oracle.wave25_run(phi, phi, np.full(phi.shape, v), h, dt, [-1, -1, -1], 10.0,
                               0.0, 0, steps)
    a_prev, a_cur = 1.0, 1.0
    for _ in range(steps):
        a_prev, a_cur = a_cur, (2 + a2 * lam) * a_cur - a_prev
    r = 4 * steps
    core = (slice(r, n - r),) * 3
    assert np.abs(pc[core] - a_cur * phi[core]).max() < 1e-11
    # closed form of the recurrence: a_n = cos((n + 1/2) w) / cos(w / 2)
    w = np.arccos(1 + a2 * lam / 2)
    assert abs(a_cur - np.cos((steps + 0.5) * w) / np.cos(w / 2)) < 1e-12


def test_ricker_closed_form():
    f, t0 = 15.0, 1.0 / 15.0
    assert abs(oracle.ricker(t0, f, t0) - 1.0) < 1e-15
    tz = t0 + 1.0 / (np.pi * f * np.sqrt(2.0))
    assert abs(oracle.ricker(tz, f, t0)) < 1e-14
    t = 0.05
    a = (np.pi * f * (t - t0)) ** 2
    assert abs(oracle.ricker(t, f, t0) - (1 - 2 * a) * np.exp(-a)) < 1e-15


def test_source_injection_single_step_and_symmetry():
    n = 21
    vel = np.full((n, n, n), 1500.0)
    h, dt, f = 10.0, 1e-3, 15.0
    t0 = 1.0 / f
    src = [10, 10, 10]
    z0 = np.zeros((n, n, n))
    pp, pc = oracle.wave25_run(z0, z0, vel, h, dt, src, f, t0, 0, 1)
    a2 = (1500.0 * dt / h) ** 2
    want = np.zeros_like(z0)
    want[10, 10, 10] = a2 * oracle.ricker(0.0, f, t0)
    assert np.array_equal(pc, want)
    pp, pc = oracle.wave25_run(z0, z0, vel, h, dt, src, f, t0, 0, 3)
    # homogeneous medium, centred source: mirror symmetric in every axis
    assert np.abs(pc - pc[::-1]).max() == 0
    assert np.abs(pc - pc[:, ::-1]).max() == 0
    assert np.abs(pc - pc.transpose(2, 1, 0)).max() < 1e-18


def test_time_index_offset_composes():
    n = 16
    rng = np.random.default_rng(3)
    vel = rng.uniform(1500, 4500, size=(n, n, n))
    p0 = rng.standard_normal((n, n, n)) * 1e-3
    args = (10.0, 8.8e-4, [8, 7, 6], 15.0, 1.0 / 15.0)
    pa, pb = oracle.wave25_run(p0, p0, vel, *args, 0, 5)
    qa, qb = oracle.wave25_run(p0, p0, vel, *args, 0, 2)
    qa, qb = oracle.wave25_run(qa, qb, vel, *args, 2, 3)
    assert np.array_equal(pa, qa) and np.array_equal(pb, qb)
