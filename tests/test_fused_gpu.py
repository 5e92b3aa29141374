"""The fused codec kernel (oc_config.fused_codec: one launch per coded slab
that decodes, runs the k 7-point steps and encodes, with no FP32 working
buffer in device memory) against the three-kernel path, through the C ABI.

Both paths must write the same codes: after every job both host levels of the
fused handle equal the three-kernel handle's byte for byte (the last sweep's
state and the one before it), and so does the decoded output.  Cases cover
ragged xy tiles (the kernel tiles the plane in 56 x 24 output cells, so grids
of 40, 60, 100 and 120 cells leave partial tiles), grids smaller than one
tile, ragged last slabs, k = 1..4 with steps mod k != 0 (a short last sweep),
rates 1..16, region sharing on and off, other ring sizes and one host level
updated in place.  The fused path is also checked against the oracle's
composition of residencies, at the tolerance the three-kernel path meets.
"""
import numpy as np
import pytest

import oracle
from paper_2204_11315_amd import inputs, oc

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

C = (0.4, 0.1, 0.1, 0.1, 0.1, 0.1, 0.1)


def run(u0, steps, fused, runs=None, **kw):
    o = oc.OutOfCore(u0.shape, C, fused_codec=fused, **kw)
    try:
        o.load(u0)
        for s in (runs or [steps]):
            o.run(s)
        torch.cuda.synchronize()
        levels = [lv.numpy().copy() for lv in o.levels]
        return o.store(), levels, o.stats()
    finally:
        o.close()


def same_codes_and_output(u0, steps, runs=None, **kw):
    a, la, sa = run(u0, steps, True, runs, **kw)
    b, lb, sb = run(u0, steps, False, runs, **kw)
    assert len(la) == len(lb)
    for x, y in zip(la, lb):
        assert np.array_equal(x, y)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    return a, sa, sb


SHAPES = [((44, 24, 40), 8), ((36, 64, 60), 12), ((24, 8, 8), 12), ((32, 100, 120), 16),
          ((16, 28, 56), 16)]


@pytest.mark.parametrize("shape,S", SHAPES)
@pytest.mark.parametrize("k,steps", [(4, 10), (3, 7), (2, 5), (1, 3)])
def test_fused_equals_three_kernels_bitwise(shape, S, k, steps):
    u0 = inputs.grf_field(shape, seed=31)
    _, sa, sb = same_codes_and_output(u0, steps, k=k, rate=8, slab_planes=S, budget=64 << 20)
    slabs = len(range(0, shape[0], S))
    assert sa["n_slabs"] == slabs and sa["slab_visits"] == sb["slab_visits"]
    assert sa["peak_dev_bytes"] < sb["peak_dev_bytes"]


@pytest.mark.parametrize("R", [1, 5, 12, 16])
@pytest.mark.parametrize("share", [True, False])
def test_fused_equals_three_kernels_at_every_rate(R, share):
    u0 = inputs.grf_field((44, 24, 40), seed=32)
    same_codes_and_output(u0, 10, k=4, rate=R, slab_planes=8, budget=64 << 20, share=share)


@pytest.mark.parametrize("slots,prefetch", [(2, 1), (4, 3)])
def test_fused_ring_sizes(slots, prefetch):
    u0 = inputs.grf_field((44, 24, 40), seed=33)
    same_codes_and_output(u0, 9, k=3, rate=8, slab_planes=8, budget=64 << 20, ring_slots=slots,
                          prefetch=prefetch)


def test_fused_in_place_and_split_runs():
    u0 = inputs.grf_field((44, 24, 40), seed=34)
    same_codes_and_output(u0, 11, runs=[4, 7], k=4, rate=8, slab_planes=8, budget=64 << 20,
                          in_place=True)


def test_fused_with_timing_counts_one_launch_per_slab_visit():
    u0 = inputs.grf_field((44, 24, 40), seed=35)
    a, sa, _ = same_codes_and_output(u0, 8, k=4, rate=8, slab_planes=8, budget=64 << 20, timing=True)
    assert sa["n_fused"] == sa["slab_visits"] == 2 * 6
    assert sa["n_decode"] == 0 and sa["n_stencil"] == 0 and sa["n_encode"] == 0
    assert sa["ms_fused"] > 0.0
    assert sa["blocks_decode"] > 0 and sa["blocks_encode"] == 2 * 11 * 6 * 10


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("R", [16, 8])
def test_fused_close_to_oracle_composition(R):
    shape = (44, 24, 40)
    u0 = inputs.grf_field(shape, seed=8)
    steps, k = 10, 4
    got, _, _ = run(u0, steps, True, k=k, rate=R, slab_planes=8, budget=64 << 20)
    want = oracle.compressed_sweeps(u0, C, steps, k, R)
    e_comp = rel_l2(want, oracle.star7_run(u0, C, steps))
    n_res = -(-steps // k)
    assert rel_l2(got, want) <= 10.0 * np.sqrt(n_res * 2.0 ** -24 * e_comp)


def test_fused_refuses_what_it_does_not_cover():
    u0 = np.zeros((16, 8, 8), np.float32)
    for kw in (dict(rate=0), dict(rate=17), dict(rate=8, k=5), dict(rate=8, c0_field=True)):
        with pytest.raises(oc.OCError) as e:
            oc.OutOfCore(u0.shape, C, fused_codec=True, budget=16 << 20, **kw)
        assert e.value.status == oc.OC_ERR_UNSUPPORTED, kw


def test_fused_with_an_error_budget_runs_the_picked_rate():
    shape = (128, 64, 64)
    u0 = inputs.grf_field(shape, seed=2)
    o = oc.OutOfCore(shape, C, k=4, rate=16, slab_planes=16, budget=64 << 20, fused_codec=True,
                     error_budget=1e-3, error_steps=16)
    try:
        o.load(u0)
        o.run(16)
        got = o.store()
        R = o.stats()["rate_bits"]
    finally:
        o.close()
    fixed, _, _ = run(u0, 16, False, k=4, rate=R, slab_planes=16, budget=64 << 20)
    assert np.array_equal(got.view(np.uint32), fixed.view(np.uint32))


@pytest.mark.parametrize("R,steps", [(8, 4), (16, 3), (5, 1)])
def test_fused_kernel_on_one_slab_equals_three_kernels(R, steps):
    # an interior slab of a ragged grid (120 x 100 cells: partial tiles in x
    # and y), 16 interior planes and a 4-plane halo on either side
    nz, ny, nx = 48, 100, 120
    gz0, planes = 12, 24
    f = inputs.grf_field((nz, ny, nx), seed=36)
    slab = torch.from_numpy(np.ascontiguousarray(f[gz0:gz0 + planes])).cuda()
    codes = oc.compress(slab, R)
    got = oc.codec_star7(codes, (planes, ny, nx), gz0, nz, R, steps)
    u = oc.decompress(codes, (planes, ny, nx), R)
    u = oc.star7_incore(u, C, steps)
    want = oc.compress(u[4:planes - 4].contiguous(), R)
    assert torch.equal(got.cpu(), want.cpu())
    assert oc.codec_status() == oc.OC_OK


def test_fused_kernel_entry_checks_its_arguments():
    t = torch.zeros(1 << 16, dtype=torch.uint8, device="cuda")
    for kw, st in ((dict(R=17), oc.OC_ERR_UNSUPPORTED), (dict(steps=5), oc.OC_ERR_UNSUPPORTED),
                   (dict(gz0=2), oc.OC_ERR_SHAPE), (dict(lay=(0, 7)), oc.OC_ERR_ARG),
                   (dict(gz0=-8), oc.OC_ERR_ARG)):
        with pytest.raises(oc.OCError) as e:
            oc.codec_star7(t, (24, 8, 8), kw.get("gz0", 0), 32, kw.get("R", 8), kw.get("steps", 4),
                           lay=kw.get("lay"), out=t)
        assert e.value.status == st, kw

