"""GPU codec parity: HIP bitstreams equal the CPU oracle's byte for byte.

Compared through the C ABI (oc_codec_compress / oc_codec_decompress) on
seeded fields of several kinds, rates 1..32, and shapes spanning several
workgroups with a ragged tail.
"""
import numpy as np
import pytest

import oracle
from paper_2204_11315_amd import inputs, oc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _fields(shape, seed):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    out = {
        "normal": rng.standard_normal(shape).astype(np.float32),
        "grf": inputs.grf_field(shape, seed=seed) if min(shape) >= 4 else None,
        "modes": inputs.modes_field(shape, seed=seed),
        "denormal": (rng.standard_normal(shape) * 1e-39).astype(np.float32),
        "extreme": (np.clip(rng.standard_normal(shape), -1.9, 1.9)
                    * np.exp2(rng.integers(-126, 127, size=shape))
                    ).astype(np.float32),
        "offset": (1000.0 + 1e-3 * rng.standard_normal(shape)).astype(np.float32),
    }
    z = rng.standard_normal(shape).astype(np.float32)
    z[rng.random(shape) < 0.5] = 0.0
    z[rng.random(shape) < 0.1] = -0.0
    out["signed_zeros"] = z
    const = np.repeat(rng.standard_normal((nz // 4, ny // 4, nx // 4)).astype(np.float32), 4, 0)
    out["blockwise_const"] = np.repeat(np.repeat(const, 4, 1), 4, 2)
    if out["grf"] is not None:
        # smoothed by the stencil, as the out-of-core sweeps meet it: more bit
        # planes fit the budget, long verbatim prefixes, cuts at low planes
        out["diffused"] = oracle.star7_run(out["grf"], DIFFUSE, 24).astype(np.float32)
    return {k: v for k, v in out.items() if v is not None}


DIFFUSE = (0.4, 0.1, 0.1, 0.1, 0.1, 0.1, 0.1)


SHAPES = [(12, 20, 44), (8, 64, 1028)]


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("R", [1, 2, 3, 7, 8, 12, 16, 24, 31, 32])
def test_gpu_encode_matches_cpu_bytes(shape, R):
    for name, f in _fields(shape, 100 + R).items():
        want = oracle.compress(f, R)
        got = oc.compress(_dev(f), R).cpu().numpy()
        torch.cuda.synchronize()
        assert got.shape == want.shape
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, "%s R=%d: %d bytes differ, first at %d" % (name, R, bad.size, bad[0])


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("R", [1, 5, 8, 12, 16, 32])
def test_gpu_decode_matches_cpu_values(shape, R):
    for name, f in _fields(shape, 200 + R).items():
        codes = oracle.compress(f, R)
        want = oracle.decompress(codes, shape, R)
        got = oc.decompress(_dev(codes), shape, R).cpu().numpy()
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), (name, R)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("R", [1, 8, 13, 32])
def test_gpu_decode_of_arbitrary_bytes_matches_cpu(shape, R):
    # every byte string of the right length decodes: exponents up to 255 (so
    # infinities), group-test tokens and runs cut anywhere, streams no encoder
    # writes; the two decoders must still agree on every bit
    rng = np.random.default_rng(300 + R)
    codes = rng.integers(0, 256, size=oracle.codec_bytes(shape[2], shape[1], shape[0], R), dtype=np.uint8)
    want = oracle.decompress(codes, shape, R)
    got = oc.decompress(_dev(codes), shape, R).cpu().numpy()
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), R


def test_round_trip_error_budget_r16():
    f = inputs.grf_field((32, 32, 32), seed=7)
    g = oc.decompress(oc.compress(_dev(f), 16), f.shape, 16).cpu().numpy()
    rel = np.linalg.norm((g - f).astype(np.float64)) / np.linalg.norm(f.astype(np.float64))
    assert rel < 1e-3


def test_nonfinite_sets_status_and_clears():
    assert oc.codec_status() == oc.OC_OK
    f = np.zeros((4, 8, 8), dtype=np.float32)
    f[2, 3, 5] = np.inf
    oc.compress(_dev(f), 8)
    assert oc.codec_status() == oc.OC_ERR_NONFINITE
    assert oc.codec_status() == oc.OC_OK
    oc.compress(_dev(np.ones((4, 8, 8), np.float32)), 8)
    assert oc.codec_status() == oc.OC_OK


def test_bad_arguments_rejected_before_launch():
    d = torch.zeros((4, 8, 6), dtype=torch.float32, device="cuda")
    with pytest.raises(oc.OCError):
        oc.compress(d, 8)
    d = torch.zeros((4, 8, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(oc.OCError):
        oc.compress(d, 33)
    small = torch.zeros(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(oc.OCError):
        oc.compress(d, 8, out=small)


@pytest.mark.parametrize("R", [5, 8, 16])
def test_full_slab_shape_diffused_field(R):
    # a slab-sized piece of the field after 32 stencil steps (the decoder's
    # longest loops: many planes and significant coefficients per block)
    f = oracle.star7_run(inputs.grf_field((16, 512, 512), seed=5), DIFFUSE, 32).astype(np.float32)
    want = oracle.compress(f, R)
    got = oc.compress(_dev(f), R).cpu().numpy()
    assert np.array_equal(got, want)
    back = oc.decompress(_dev(want), f.shape, R).cpu().numpy()
    assert np.array_equal(back.view(np.uint32), oracle.decompress(want, f.shape, R).view(np.uint32))


@pytest.mark.parametrize("R", [5, 16])
def test_full_slab_shape_grf(R):
    # the shape of one C2/C3 slab interior (64 planes of 512 x 512), at the
    # bench job's headline rate and at 16 bits per value
    f = inputs.grf_field((64, 512, 512), seed=2)
    want = oracle.compress(f, R)
    got = oc.compress(_dev(f), R).cpu().numpy()
    assert np.array_equal(got, want)
    back = oc.decompress(_dev(want), f.shape, R).cpu().numpy()
    assert np.array_equal(back.view(np.uint32), oracle.decompress(want, f.shape, R).view(np.uint32))
