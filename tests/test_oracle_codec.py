"""Pins of the scalar reference codec (CPU only).

Each step of the fixed-rate format is tied to something other than the C code:
the published decorrelating matrix on inputs whose shifts are exact, a
brute-forced bound on the inverse's error, the definition of base -2, the sort key of the coefficient order, an independent
closed form of the embedded coder's stream length per bit plane, the embedded
prefix property across rates, the reconstruction of digits a budget cut off
(against an independent model of the coder and the exact mean of the unread
digits), exact reconstruction of zero / constant blocks, the lossless bound,
and the block layout of a field.
"""
import math

import numpy as np
import pytest

import oracle

RNG = np.random.default_rng(1234)


def rand_blocks(n, rng=RNG):
    """A mix of block kinds: Gaussian, smooth, offset, mixed exponents."""
    out = []
    t = np.arange(64)
    i, j, k = t % 4, (t // 4) % 4, t // 16
    for b in range(n):
        kind = b % 5
        if kind == 0:
            v = rng.standard_normal(64)
        elif kind == 1:
            v = np.sin(0.3 * i + 0.2 * j + 0.1 * k + rng.uniform(0, 6)) * rng.uniform(0.1, 10)
        elif kind == 2:
            v = 100.0 + rng.standard_normal(64) * 1e-3
        elif kind == 3:
            v = rng.standard_normal(64) * np.exp2(rng.integers(-20, 20, size=64))
        else:
            v = rng.standard_normal(64) * 1e-40       # subnormal range
        out.append(v.astype(np.float32))
    return out


# ---- step 4: transform -----------------------------------------------------
# The published decorrelating matrix of the compressor the paper runs (Lindstrom
# 2014): one line of four integers maps to A x, applied along x, then y, then z.
A_ZFP = np.array([[4, 4, 4, 4],
                  [5, 1, -1, -5],
                  [-4, 4, 4, -4],
                  [-2, 6, -6, 2]], dtype=np.float64) / 16.0
# Largest |inv(fwd(q)) - q| over a block, in units of the 27-bit integers: the
# floor halvings of the forward steps drop low bits that the inverse cannot
# restore.  A line loses at most 2 (brute force below); an error e entering the
# inverse of an axis undone later leaves it as about 3.75 |e| (the largest
# absolute row sum of the inverse matrix) on top of that axis's own 2, so over
# the three axes about 2 + 3.75 (2 + 3.75 * 2) = 40 units, below 64.
XFORM_ROUND_TRIP_ULPS = 64


def _lines_3d(q, M):
    blk = q.astype(np.float64).reshape(4, 4, 4)               # [k][j][i]
    w = np.einsum("ai,kji->kja", M, blk)                      # along x
    w = np.einsum("bj,kja->kba", M, w)                        # along y
    return np.einsum("ck,kba->cba", M, w)                     # along z


def test_transform_equals_the_published_matrix_when_shifts_are_exact():
    # inputs that are multiples of 2^12 keep every floor halving exact on all
    # three axes (each axis divides by at most 16), so the integer transform
    # must equal the linear map, and its inverse must return the input exactly
    for _ in range(100):
        q = (RNG.integers(-2 ** 14, 2 ** 14, size=64) * 4096).astype(np.int32)
        got = oracle.fwd_xform(q).astype(np.float64).reshape(4, 4, 4)
        assert np.array_equal(got, _lines_3d(q, A_ZFP))
        assert np.array_equal(oracle.inv_xform(oracle.fwd_xform(q)), q)
    # and the linear inverse of the published matrix, applied in reverse axis
    # order, maps those coefficients back
    Ainv = np.linalg.inv(A_ZFP)
    q = (RNG.integers(-2 ** 14, 2 ** 14, size=64) * 4096).astype(np.int32)
    c = oracle.fwd_xform(q).astype(np.float64).reshape(4, 4, 4)
    assert np.allclose(_lines_3d(c.reshape(64), Ainv).reshape(64), q, rtol=0, atol=1e-6)


def test_one_line_transform_and_round_trip_brute_force():
    # Adding 16 m to a line adds 16 A m (integers: every halving stays exact) to
    # its coefficients, and the inverse then adds 16 m back, so a line's
    # round-trip error depends only on its residues mod 16: all 16^4 of them.
    base = (RNG.integers(-2 ** 20, 2 ** 20, size=4) * 16).astype(np.int64)
    shift = np.rint(A_ZFP @ base).astype(np.int64)
    worst = 0
    for a in range(16):
        for b in range(16):
            for c in range(16):
                for d in range(16):
                    r = np.array([a, b, c, d], dtype=np.int64)
                    f0 = oracle.fwd_lift_line(r)
                    f1 = oracle.fwd_lift_line(base + r)
                    assert np.array_equal(f1.astype(np.int64) - f0, shift)
                    e = oracle.inv_lift_line(f1).astype(np.int64) - (base + r)
                    worst = max(worst, int(np.abs(e).max()))
    # the halvings lose at most 2 units on a line
    assert 0 < worst <= 2


def test_transform_round_trip_error_bound():
    for _ in range(2000):
        q = RNG.integers(-2 ** 27 + 1, 2 ** 27, size=64).astype(np.int32)
        e = oracle.inv_xform(oracle.fwd_xform(q)).astype(np.int64) - q
        assert np.abs(e).max() <= XFORM_ROUND_TRIP_ULPS


def test_transform_range_growth_bound():
    # every row of A has absolute sum <= 1, so the exact map cannot grow a
    # magnitude; the floors add at most a few units
    worst = 0
    for _ in range(300):
        q = RNG.choice([-(2 ** 27 - 1), 2 ** 27 - 1], size=64).astype(np.int32)
        worst = max(worst, int(np.abs(oracle.fwd_xform(q).astype(np.int64)).max()))
    assert worst <= 2 ** 27 + 8


# ---- step 6: negabinary ---------------------------------------------------------
def test_negabinary_definition_and_round_trip():
    vals = list(RNG.integers(-2 ** 30, 2 ** 30, size=500)) + [0, 1, -1, 2 ** 30 - 1, -2 ** 30]
    for c in vals:
        u = oracle.to_negabinary(int(c))
        assert sum(((u >> b) & 1) * (-2) ** b for b in range(32)) == int(c)
        assert oracle.from_negabinary(u) == int(c)


# ---- step 5: order ----------------------------------------------------------------
def test_sequency_order_is_the_sorted_key():
    perm = list(oracle.sequency_order())
    key = lambda t: ((t % 4) + (t // 4 % 4) + t // 16,
                     (t % 4) ** 2 + (t // 4 % 4) ** 2 + (t // 16) ** 2, t)
    assert perm == sorted(range(64), key=key)
    assert perm[0] == 0 and sorted(perm) == list(range(64))


# ---- steps 2-3: quantisation --------------------------------------------------------
def test_quantisation_is_exact_block_floating_point():
    for v in rand_blocks(40):
        q, eb = oracle.quantize(v)
        for t in range(64):
            x = float(v[t])
            # independent decomposition of the float: x = m * 2^e, 0.5 <= |m| < 1
            m, e = math.frexp(x)
            if x == 0.0:
                assert q[t] == 0
                continue
            # x = q * 2^(eb-153) when nothing was shifted off; otherwise q is the
            # truncation toward zero of x / 2^(eb-153)
            scaled = math.ldexp(x, 153 - eb)
            assert int(q[t]) == int(scaled)          # int() truncates toward zero


def test_non_finite_rejected():
    for bad in (np.inf, -np.inf, np.nan):
        v = np.zeros(64, dtype=np.float32)
        v[17] = bad
        with pytest.raises(oracle.OracleError):
            oracle.block_encode(v, 16)
    f = np.zeros((4, 4, 8), dtype=np.float32)
    f[1, 2, 5] = np.nan
    with pytest.raises(oracle.OracleError):
        oracle.compress(f, 8)


# ---- step 7: the embedded coder -------------------------------------------------------
def plane_coefficients(v):
    """Negabinary coefficient words in coding order, built from the pinned sub-steps."""
    q, eb = oracle.quantize(v)
    c = oracle.fwd_xform(q)
    perm = oracle.sequency_order()
    return [oracle.to_negabinary(int(c[p])) for p in perm], eb


def closed_form_plane_lengths(u):
    """Bits of each plane (31 down to 0) without a budget.

    With n significant coefficients before plane p and plane word x:
    n verbatim bits; then, if x has bits at or above n, one group bit and one
    scanned bit per set bit plus the zeros scanned up to the highest set bit h,
    i.e. popcount(x >> n) + (h + 1 - n); then a closing group bit 0 unless
    n has reached 64.  n becomes max(n, h + 1).
    """
    n, out = 0, []
    for p in range(31, -1, -1):
        x = sum(((u[q] >> p) & 1) << q for q in range(64))
        L = n
        if n < 64:
            hi = x >> n
            if hi:
                h = x.bit_length() - 1
                L += bin(hi).count("1") + (h + 1 - n)
                n = max(n, h + 1)
            if n < 64:
                L += 1
        out.append((p, L, n))
    return out


def test_stream_length_matches_closed_form():
    for v in rand_blocks(60):
        u, _ = plane_coefficients(v)
        total = 8 + sum(L for _, L, _ in closed_form_plane_lengths(u))
        _, nbits = oracle.block_encode(v, 32)
        assert nbits == total


def _bits(slot):
    return np.unpackbits(np.asarray(slot, dtype=np.uint8), bitorder="little")


def test_embedded_prefix_property():
    for v in rand_blocks(40):
        s32, _ = oracle.block_encode(v, 32)
        b32 = _bits(s32)
        for R in (1, 2, 3, 5, 8, 12, 16, 24, 31):
            sR, _ = oracle.block_encode(v, R)
            assert np.array_equal(_bits(sR), b32[:64 * R])


def test_decoder_on_streams_cut_at_plane_boundaries():
    """Zeroing a stream after plane P's last bit must decode the coefficients
    with planes below P cleared (zeros read as verbatim 0 and group bit 0)."""
    perm = oracle.sequency_order()
    for v in rand_blocks(25):
        u, eb = plane_coefficients(v)
        s32, nbits = oracle.block_encode(v, 32)
        if nbits > 64 * 32:
            continue
        pos = 8
        for p, L, _ in closed_form_plane_lengths(u):
            pos += L
            if p % 5:
                continue
            bits = _bits(s32).copy()
            bits[pos:] = 0
            cut = np.packbits(bits, bitorder="little")
            got = oracle.block_decode(cut, 32)
            keep = ~((1 << p) - 1) & 0xFFFFFFFF
            c = np.zeros(64, dtype=np.int32)
            for o in range(64):
                c[perm[o]] = oracle.from_negabinary(u[o] & keep)
            qh = oracle.inv_xform(c)
            want = np.ldexp(qh.astype(np.float32), eb - 153).astype(np.float32)
            assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


# ---- step 7': reconstruction of digits the budget cut off ------------------------------
def test_unread_mean_is_the_floored_mean_of_the_unread_digits():
    from fractions import Fraction
    # exhaustive for small d: average of sum_j b_j (-2)^j over all 2^d digit patterns
    for d in range(0, 17):
        total = 0
        for pat in range(1 << d):
            total += sum(((pat >> j) & 1) * (-2) ** j for j in range(d))
        mean = Fraction(total, 1 << d)
        assert oracle.unread_mean(d) == math.floor(mean), d
    # larger d: each further digit adds its own mean (-2)^d / 2
    mean = Fraction(0)
    for d in range(0, 32):
        assert oracle.unread_mean(d) == math.floor(mean), d
        mean += Fraction((-2) ** d, 2)


def coded_bits(u, budget):
    """Independent model of step 7 (bit plane coding with group tests), cut at
    `budget` bits: returns, per coefficient, the digits known to the decoder
    (as a mask of planes) and the lowest known plane (32 = none)."""
    known = [0] * 64
    low = [32] * 64
    used = 0
    n = 0
    for p in range(31, -1, -1):
        x = sum(((u[q] >> p) & 1) << q for q in range(64))
        for q in range(n):                          # verbatim digits
            if used == budget:
                return known, low
            used += 1
            known[q] |= 1 << p
            low[q] = p
        while n < 64:
            if used == budget:                      # group bit
                return known, low
            used += 1
            if (x >> n) == 0:
                break
            while True:                             # run up to the next 1
                if used == budget:
                    return known, low
                used += 1
                bit = (x >> n) & 1
                known[n] |= 1 << p
                low[n] = p
                n += 1
                if bit:
                    break
        for q in range(n, 64):                      # closed: the rest is 0 in plane p
            known[q] |= 1 << p
            low[q] = p
    return known, low


def test_budget_cut_reconstruction_matches_an_independent_model():
    perm = oracle.sequency_order()
    for v in rand_blocks(40, rng=np.random.default_rng(77)):
        u, eb = plane_coefficients(v)
        for R in (1, 2, 3, 5, 8, 9, 12, 16):
            known, low = coded_bits(u, 64 * R - 8)
            c = np.zeros(64, dtype=np.int32)
            for o in range(64):
                w = u[o] & known[o]
                val = oracle.from_negabinary(w)
                if w and 0 < low[o] < 32:
                    val = (val + oracle.unread_mean(low[o]) + 2 ** 31) % 2 ** 32 - 2 ** 31
                c[perm[o]] = val
            want = np.ldexp(oracle.inv_xform(c).astype(np.float32), eb - 153).astype(np.float32)
            slot, _ = oracle.block_encode(v, R)
            got = oracle.block_decode(slot, R)
            assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), R


def test_unread_mean_lowers_the_error_of_cut_streams():
    """Smooth blocks at 8 bits per value: reconstructing the unread digits at
    their mean gives a smaller squared error than filling them with zeros."""
    perm = oracle.sequency_order()
    rng = np.random.default_rng(5)
    t = np.arange(64)
    i, j, k = t % 4, (t // 4) % 4, t // 16
    e_mean = e_zero = 0.0
    for _ in range(60):
        v = (np.sin(0.4 * i + 0.3 * j + 0.2 * k + rng.uniform(0, 6)) + 0.05 * rng.standard_normal(64))
        v = v.astype(np.float32)
        u, eb = plane_coefficients(v)
        known, _ = coded_bits(u, 64 * 8 - 8)
        c = np.zeros(64, dtype=np.int32)
        for o in range(64):
            c[perm[o]] = oracle.from_negabinary(u[o] & known[o])
        zero = np.ldexp(oracle.inv_xform(c).astype(np.float32), eb - 153)
        got = oracle.block_decode(oracle.block_encode(v, 8)[0], 8)
        e_mean += float(np.sum((got.astype(np.float64) - v) ** 2))
        e_zero += float(np.sum((zero.astype(np.float64) - v) ** 2))
    assert e_mean < 0.8 * e_zero


# ---- special cases and bounds ----------------------------------------------------------
@pytest.mark.parametrize("R", [1, 2, 4, 8, 16, 32])
def test_zero_and_constant_blocks_exact(R):
    for c in (0.0, 1.0, -3.75, 1e-40, -7e-45, 3.3e38, 123456.789, -1e-30):
        v = np.full(64, c, dtype=np.float32)
        s, _ = oracle.block_encode(v, R)
        assert np.array_equal(oracle.block_decode(s, R).view(np.uint32), v.view(np.uint32))


def test_lossless_bound_when_every_plane_fits():
    for v in rand_blocks(80):
        s, nbits = oracle.block_encode(v, 32)
        if nbits > 64 * 32:
            continue
        _, eb = oracle.quantize(v)
        d = oracle.block_decode(s, 32).astype(np.float64)
        # truncation to 27 bits (< 1 unit) plus the transform's round trip, in
        # units of 2^(eb-153), plus the FP32 rounding of the reconstruction
        tol = (XFORM_ROUND_TRIP_ULPS + 1) * math.ldexp(1.0, eb - 153)
        assert np.abs(d - v.astype(np.float64)).max() < tol + np.abs(v).max() * 2.0 ** -24


def test_aggregate_error_decreases_with_rate():
    from paper_2204_11315_amd import inputs
    f = inputs.grf_field((16, 16, 16), seed=3)
    errs = []
    for R in (8, 12, 16, 24, 32):
        g = oracle.decompress(oracle.compress(f, R), f.shape, R)
        errs.append(np.sqrt(np.mean((g.astype(np.float64) - f) ** 2)))
    assert all(a > b for a, b in zip(errs, errs[1:]))
    assert errs[2] < 1e-3 * np.sqrt(np.mean(f.astype(np.float64) ** 2))


def test_field_layout_slot_index():
    nz, ny, nx, R = 8, 12, 16, 4
    bx, by, bz = 2, 1, 1
    f = np.zeros((nz, ny, nx), dtype=np.float32)
    f[4 * bz:4 * bz + 4, 4 * by:4 * by + 4, 4 * bx:4 * bx + 4] = RNG.standard_normal((4, 4, 4))
    buf = oracle.compress(f, R)
    slot = (bz * (ny // 4) + by) * (nx // 4) + bx
    zero_slot, _ = oracle.block_encode(np.zeros(64, np.float32), R)
    for b in range((nx // 4) * (ny // 4) * (nz // 4)):
        piece = buf[b * 8 * R:(b + 1) * 8 * R]
        if b == slot:
            blk = f[4 * bz:4 * bz + 4, 4 * by:4 * by + 4, 4 * bx:4 * bx + 4].reshape(64)
            s, _ = oracle.block_encode(blk, R)
            assert np.array_equal(piece, s)
        else:
            assert np.array_equal(piece, zero_slot)
    g = oracle.decompress(buf, f.shape, R)
    assert g.shape == f.shape


def test_shape_must_be_block_aligned():
    with pytest.raises(oracle.OracleError):
        oracle.compress(np.zeros((4, 4, 6), np.float32), 8)


def test_thread_count_does_not_change_codes():
    # blocks are coded independently, so the host thread count the oracle's
    # loops run on must not change a byte of the stream or of the decode
    f = RNG.standard_normal((8, 12, 16)).astype(np.float32)
    ref = oracle.compress(f, 9)
    prev = oracle.set_threads(1)
    try:
        assert oracle.set_threads(0) == 1
        one = oracle.compress(f, 9)
        dec1 = oracle.decompress(one, f.shape, 9)
    finally:
        oracle.set_threads(prev)
    assert np.array_equal(one, ref)
    assert np.array_equal(dec1.view(np.uint32), oracle.decompress(ref, f.shape, 9).view(np.uint32))


def test_run_past_the_last_coefficient_ends_the_stream():
    """A group bit 1 whose run reaches past coefficient 63 without a closing 1
    is never written by the encoder; the format ends the stream there (as a
    budget cut would): whatever follows is ignored, and the digits read up to
    that point decode as usual."""
    R = 4
    perm = oracle.sequency_order()
    rng = np.random.default_rng(77)
    eb = 150
    head = [(eb >> b) & 1 for b in range(8)]
    # (a) plane 31: group bit 1, then 64 zeros: no coefficient is significant
    # (b) plane 31: group 1, digit 1 (coefficient 0), group 1, then 63 zeros
    for body, sig in (([1] + [0] * 64, False), ([1, 1, 1] + [0] * 63, True)):
        outs = []
        for _ in range(3):
            bits = np.array(head + body, dtype=np.uint8)
            tail = rng.integers(0, 2, size=64 * R - bits.size, dtype=np.uint8)
            slot = np.packbits(np.concatenate([bits, tail]), bitorder="little")
            outs.append(oracle.block_decode(slot, R))
        for o in outs[1:]:
            assert np.array_equal(o.view(np.uint32), outs[0].view(np.uint32))
        c = np.zeros(64, dtype=np.int32)
        if sig:
            c[perm[0]] = oracle.from_negabinary(1 << 31) + oracle.unread_mean(31)
        want = np.ldexp(oracle.inv_xform(c).astype(np.float32), eb - 153).astype(np.float32)
        assert np.array_equal(outs[0].view(np.uint32), want.view(np.uint32))


@pytest.mark.parametrize("R", [1, 3, 8, 17, 32])
def test_any_byte_string_decodes_deterministically(R):
    # streams no encoder writes (random bytes) still decode: the same bits on
    # every call, no NaN (values are integers times a power of two, so at
    # worst infinite), and equal to a block-by-block decode of the same slots
    rng = np.random.default_rng(900 + R)
    shape = (8, 8, 12)
    codes = rng.integers(0, 256, size=oracle.codec_bytes(12, 8, 8, R), dtype=np.uint8)
    a = oracle.decompress(codes, shape, R)
    b = oracle.decompress(codes.copy(), shape, R)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    assert not np.isnan(a).any()
    nbx, nby = 3, 2
    for blk in range(nbx * nby * 2):
        bx, by, bz = blk % nbx, (blk // nbx) % nby, blk // (nbx * nby)
        v = oracle.block_decode(codes[blk * 8 * R:(blk + 1) * 8 * R], R).reshape(4, 4, 4)
        got = a[4 * bz:4 * bz + 4, 4 * by:4 * by + 4, 4 * bx:4 * bx + 4]
        assert np.array_equal(got.view(np.uint32), v.view(np.uint32))
