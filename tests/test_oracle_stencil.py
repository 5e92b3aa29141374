"""Pins of the FP64 stencil oracle against mathematics (CPU only).

The stencil update is the plain definition of Sec. 3.1; these tests tie the C
oracle to facts that do not come from it: the closed-form decay of a sine mode
(zero ghosts make products of sines exact eigenvectors), constant-field
invariance inside the light cone, linearity, norm contraction for convex
weights, and an explicit dense matrix built cell by cell.
"""
import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2204_11315_amd import inputs

C_CFG = [0.4, 0.1, 0.1, 0.1, 0.1, 0.1, 0.1]


def mode_eigenvalue(shape, m, c0=0.4, c1=0.1):
    nz, ny, nx = shape
    mx, my, mz = m
    return c0 + 2 * c1 * (np.cos(np.pi * mx / (nx + 1)) + np.cos(np.pi * my / (ny + 1))
                          + np.cos(np.pi * mz / (nz + 1)))


@pytest.mark.parametrize("m", [(1, 1, 1), (4, 4, 4), (1, 2, 3), (3, 1, 4)])
def test_sine_mode_decays_by_closed_form(m):
    shape = (64, 64, 64)
    phi = inputs.single_mode(shape, m)
    lam = mode_eigenvalue(shape, m)
    u = oracle.star7_run(phi, C_CFG, 8)
    rel = np.linalg.norm(u - lam ** 8 * phi) / np.linalg.norm(lam ** 8 * phi)
    assert rel < 1e-12


def test_closed_form_values_match_decimal_table():
    # independent arithmetic of the same closed form at N = 64 (decimal values)
    lam = mode_eigenvalue((64, 64, 64), (1, 1, 1))
    assert abs(lam - 0.999299336099) < 1e-11
    assert abs(lam ** 8 - 0.994408415587) < 1e-11
    lam4 = mode_eigenvalue((64, 64, 64), (4, 4, 4))
    assert abs(lam4 - 0.988822075684) < 1e-11


def test_non_cubic_mode_pins_axis_order():
    shape = (10, 14, 22)             # nz, ny, nx all different
    m = (3, 2, 1)                    # (mx, my, mz)
    phi = inputs.single_mode(shape, m)
    lam = mode_eigenvalue(shape, m)
    u = oracle.star7_run(phi, C_CFG, 5)
    assert np.abs(u - lam ** 5 * phi).max() < 1e-13


def test_constant_field_invariant_inside_light_cone_dyadic():
    # dyadic weights summing to 1: a constant is reproduced bit-exactly where
    # the zero ghosts have not been felt yet (distance > steps from every face)
    c = [0.25, 0.125, 0.125, 0.125, 0.125, 0.125, 0.125]
    steps = 5
    u = oracle.star7_run(np.full((16, 16, 16), 3.0), c, steps)
    core = u[steps:-steps, steps:-steps, steps:-steps]
    assert np.all(core == 3.0)
    # and the boundary cells have lost mass (zero Dirichlet)
    assert u[0, 0, 0] < 3.0


def test_constant_field_nearly_invariant_config_weights():
    steps = 4
    u = oracle.star7_run(np.full((14, 14, 14), 1.0), C_CFG, steps)
    core = u[steps:-steps, steps:-steps, steps:-steps]
    assert np.abs(core - 1.0).max() < 1e-7 * steps


def test_linearity():
    rng = np.random.default_rng(7)
    a = rng.standard_normal((9, 10, 11))
    b = rng.standard_normal((9, 10, 11))
    ua = oracle.star7_run(a, C_CFG, 3)
    ub = oracle.star7_run(b, C_CFG, 3)
    uab = oracle.star7_run(2.0 * a - 0.5 * b, C_CFG, 3)
    assert np.abs(uab - (2.0 * ua - 0.5 * ub)).max() < 1e-12


def test_norms_do_not_grow():
    rng = np.random.default_rng(8)
    u = rng.standard_normal((12, 12, 12))
    prev_inf, prev_2 = np.abs(u).max(), np.linalg.norm(u)
    for _ in range(6):
        u = oracle.star7_run(u, C_CFG, 1)
        assert np.abs(u).max() <= prev_inf + 1e-15
        assert np.linalg.norm(u) <= prev_2 + 1e-12
        prev_inf, prev_2 = np.abs(u).max(), np.linalg.norm(u)


@pytest.mark.parametrize("shape", [(8, 8, 8), (5, 7, 9)])
def test_dense_matrix_brute_force(shape):
    rng = np.random.default_rng(9)
    c = [0.3, 0.05, 0.15, 0.07, 0.13, 0.11, 0.09]   # every coefficient different
    c0f = rng.uniform(0.3, 0.5, size=shape)
    u0 = rng.standard_normal(shape)
    nz, ny, nx = shape
    A = brute.dense_star7(nx, ny, nz, c, c0f)
    want = np.linalg.matrix_power(A, 4) @ u0.reshape(-1)
    got = oracle.star7_run(u0, c, 4, c0f)
    assert np.abs(got.reshape(-1) - want).max() < 1e-13
    # transpose operator
    v = rng.standard_normal(shape)
    gotT = oracle.star7_step(v, c, c0f, transpose=True)
    assert np.abs(gotT.reshape(-1) - A.T @ v.reshape(-1)).max() < 1e-13


def test_zero_steps_is_identity():
    rng = np.random.default_rng(10)
    u = rng.standard_normal((4, 5, 6))
    assert np.array_equal(oracle.star7_run(u, C_CFG, 0), u)
