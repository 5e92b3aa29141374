"""Pins of the oracle's compressed path as a composition (CPU only).

`oracle.compressed_sweeps` strings together the load-time encode, one decode /
k steps / encode per residency (the last residency runs steps mod k steps), and
the store-time decode (Sec. 1 and Sec. 4.2: the host keeps only codes; every
chunk is decompressed after its copy-in and compressed before its copy-back).

The pins use a case where every piece has a closed form independent of the
oracle's code:

* a field that is constant on each 4x4x4 block codes exactly at every rate
  (the codec's constant-block pin), so the codec steps are the identity;
* a stencil with only the diagonal coefficient (c0 = 1/3, neighbours 0) keeps
  such a field block-constant, and one residency of s steps is s successive
  FP64 multiplications by c0, after which the field is handed to the encoder
  as FP32.

So the composition must equal, bit for bit, a chain of numpy products rounded
to FP32 once per residency.  A wrong number or length of residencies (the
short last one above all) or a skipped FP32 rounding between residencies
changes the bits.
"""
import numpy as np
import pytest

import oracle

DIAG = (1.0 / 3.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0)


def block_constant_field(nb, seed, lo=0.5, hi=4.0):
    """(4*nbz, 4*nby, 4*nbx) FP32 field, one random value per 4x4x4 block,
    magnitudes in [lo, hi) with random signs (no subnormals, no overflow)."""
    rng = np.random.default_rng(seed)
    nbz, nby, nbx = nb
    vals = rng.uniform(lo, hi, size=nb) * rng.choice([-1.0, 1.0], size=nb)
    f = np.repeat(np.repeat(np.repeat(vals, 4, axis=0), 4, axis=1), 4, axis=2)
    return f.astype(np.float32)


def diag_chain(u0, c0, steps, k):
    """The closed form: per residency of s = min(k, steps left) steps, s FP64
    products by c0 (per cell when c0 is an array), then one rounding to FP32."""
    v = np.asarray(u0, dtype=np.float32)
    c = np.asarray(c0, dtype=np.float64)
    done = 0
    while done < steps:
        s = min(k, steps - done)
        w = v.astype(np.float64)
        for _ in range(s):
            w = w * c
        v = w.astype(np.float32)
        done += s
    return v


@pytest.mark.parametrize("R", [1, 3, 8, 16, 32])
@pytest.mark.parametrize("steps,k", [(10, 4), (7, 3), (4, 4), (1, 4), (9, 2)])
def test_composition_equals_closed_form_on_block_constant_fields(R, steps, k):
    u0 = block_constant_field((3, 2, 5), seed=100 + steps + R)
    got = oracle.compressed_sweeps(u0, DIAG, steps, k, R)
    want = diag_chain(u0, 1.0 / 3.0, steps, k)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_closed_form_distinguishes_the_residency_split():
    """The pin is sensitive: the 10-step job in residencies of 4, 4, 2 differs
    from 4, 4, 4 (a last residency of k steps), from one unrounded run of 10
    FP64 products, and from residencies of 2."""
    u0 = block_constant_field((3, 2, 5), seed=7)
    good = diag_chain(u0, 1.0 / 3.0, 10, 4)
    assert not np.array_equal(good, diag_chain(u0, 1.0 / 3.0, 12, 4))
    assert not np.array_equal(good.view(np.uint32), diag_chain(u0, 1.0 / 3.0, 10, 10).view(np.uint32))
    assert not np.array_equal(good.view(np.uint32), diag_chain(u0, 1.0 / 3.0, 10, 2).view(np.uint32))
    got = oracle.compressed_sweeps(u0, DIAG, 10, 4, 8)
    assert np.array_equal(got.view(np.uint32), good.view(np.uint32))


def test_composition_with_a_c0_field():
    """Per-cell diagonal coefficients that are constant on each block keep the
    field block-constant: the composition equals the per-cell product chain."""
    u0 = block_constant_field((2, 3, 2), seed=11)
    c0 = np.abs(block_constant_field((2, 3, 2), seed=12, lo=0.3, hi=0.5))
    c = (0.4, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0)   # c0 is overridden by the field
    got = oracle.compressed_sweeps(u0, c, 6, 4, 12, c0f=c0)
    want = diag_chain(u0, c0.astype(np.float64), 6, 4)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


@pytest.mark.parametrize("R", [1, 8, 32])
def test_zero_steps_is_one_codec_round_trip(R):
    """No residency: load-encode and store-decode only, which is the identity
    on block-constant fields."""
    u0 = block_constant_field((2, 2, 2), seed=13)
    got = oracle.compressed_sweeps(u0, DIAG, 0, 4, R)
    assert np.array_equal(got.view(np.uint32), u0.view(np.uint32))


@pytest.mark.parametrize("R,L", [(3, 8), (5, 9), (1, 32)])
@pytest.mark.parametrize("steps,k", [(10, 4), (4, 4), (1, 4)])
def test_load_rate_keeps_the_residency_structure(R, L, steps, k):
    # a separate rate for the load-time encode changes no residency: the
    # block-constant closed form holds whatever the two rates are
    u0 = block_constant_field((3, 2, 5), seed=300 + steps + R)
    got = oracle.compressed_sweeps(u0, DIAG, steps, k, R, load_rate=L)
    want = diag_chain(u0, 1.0 / 3.0, steps, k)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_load_rate_decides_the_first_decode_and_a_store_without_steps():
    # with no residency the store decodes the load's codes: one round trip at
    # the load rate, whose error is the codec's at that rate (smaller than at R)
    from paper_2204_11315_amd import inputs
    u0 = inputs.grf_field((16, 16, 16), seed=4)
    a = oracle.compressed_sweeps(u0, (0.4,) + (0.1,) * 6, 0, 4, 3, load_rate=9)
    assert np.array_equal(a.view(np.uint32), oracle.decompress(oracle.compress(u0, 9), u0.shape, 9).view(np.uint32))
    # the load rate equal to R is the plain composition
    b = oracle.compressed_sweeps(u0, (0.4,) + (0.1,) * 6, 6, 4, 5, load_rate=5)
    assert np.array_equal(b.view(np.uint32), oracle.compressed_sweeps(u0, (0.4,) + (0.1,) * 6, 6, 4, 5).view(np.uint32))
    # a finer load rate lowers the job's error on a rough field
    ref = oracle.star7_run(u0, (0.4,) + (0.1,) * 6, 8)
    err = lambda v: np.linalg.norm(v.astype(np.float64) - ref) / np.linalg.norm(ref)
    assert err(oracle.compressed_sweeps(u0, (0.4,) + (0.1,) * 6, 8, 4, 3, load_rate=10)) < \
        err(oracle.compressed_sweeps(u0, (0.4,) + (0.1,) * 6, 8, 4, 3))
