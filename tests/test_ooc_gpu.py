"""Out-of-core pipeline parity on the GPU (through the C ABI).

* uncompressed out-of-core == in-core on the same GPU, bitwise (the schedule
  changes where cells are computed, not how), and within 1e-5 of FP64;
* compressed out-of-core (single working buffer and per-stream buffers) ==
  the in-core composition Dec(Enc(S^k(...))) built from the same kernels,
  bitwise, and close to the oracle's composition;
* ragged last slab, steps not divisible by k, several oc_run calls, c0 field;
* an injected HIP failure surfaces as OC_ERR_HIP and the handle can still be
  destroyed.
"""
import numpy as np
import pytest

import oracle
from paper_2204_11315_amd import inputs, oc

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

C = (0.4, 0.1, 0.1, 0.1, 0.1, 0.1, 0.1)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def gpu_compressed_incore(u0, R, k, steps, c=C, load_rate=0, runs=None):
    """The compressed path as a composition of the GPU's own codec and in-core
    steps: the load at `load_rate` (else R), residencies of k steps within each
    of `runs` (the job split into oc_run calls; default one run of `steps`),
    every encode after a residency at R."""
    shape = u0.shape
    rate = load_rate or R
    codes = oc.compress(_dev(u0), rate)
    for n in (runs or [steps]):
        done = 0
        while done < n:
            s = min(k, n - done)
            u = oc.decompress(codes, shape, rate)
            u = oc.star7_incore(u, c, s)
            rate = R
            codes = oc.compress(u, rate)
            done += s
    out = oc.decompress(codes, shape, rate).cpu().numpy()
    assert oc.codec_status() == oc.OC_OK
    return out


def run_ooc(u0, steps, c0=None, runs=None, **kw):
    o = oc.OutOfCore(u0.shape, **kw)
    try:
        o.load(u0, c0)
        for s in (runs or [steps]):
            o.run(s)
        return o.store(), o.stats()
    finally:
        o.close()


SHAPE = (44, 24, 40)     # nz = 5 slabs of 8 + a ragged slab of 4


@pytest.mark.parametrize("k,S,steps", [(3, 8, 10), (4, 8, 8), (1, 12, 3), (2, 44, 6), (4, 20, 9)])
def test_uncompressed_ooc_equals_incore_bitwise(k, S, steps):
    u0 = inputs.modes_field(SHAPE, seed=5)
    need = oc.plan_bytes(SHAPE, oc.make_star7(), k, S, 0)
    got, st = run_ooc(u0, steps, k=k, rate=0, slab_planes=S, budget=need)
    want = oc.star7_incore(_dev(u0), C, steps).cpu().numpy()
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    assert rel_l2(got, oracle.star7_run(u0, C, steps)) <= 1e-5
    assert st["peak_dev_bytes"] == need


def test_uncompressed_ooc_split_runs():
    u0 = inputs.modes_field(SHAPE, seed=6)
    a, _ = run_ooc(u0, 10, k=3, rate=0, slab_planes=8, runs=[4, 6])
    b, _ = run_ooc(u0, 10, k=3, rate=0, slab_planes=8, runs=[10])
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


@pytest.mark.parametrize("R", [16, 8, 12, 5])
@pytest.mark.parametrize("swb", [True, False])
@pytest.mark.parametrize("k,S,steps", [(4, 8, 12), (3, 12, 7), (2, 44, 4)])
def test_compressed_ooc_equals_incore_composition_bitwise(R, swb, k, S, steps):
    u0 = inputs.grf_field(SHAPE, seed=7)
    got, st = run_ooc(u0, steps, k=k, rate=R, slab_planes=S, single_buffer=swb,
                      budget=64 << 20)
    want = gpu_compressed_incore(u0, R, k, steps)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


@pytest.mark.parametrize("R", [16, 12, 8, 5])
@pytest.mark.parametrize("shape,S,seed", [(SHAPE, 8, 8), (SHAPE, 8, 9), ((64, 64, 64), 16, 8)])
def test_compressed_ooc_close_to_oracle_composition(R, shape, S, seed):
    # 10 steps at k = 4: two residencies of 4 steps and a short one of 2
    steps, k = 10, 4
    u0 = inputs.grf_field(shape, seed=seed)
    got, _ = run_ooc(u0, steps, k=k, rate=R, slab_planes=S)
    want = oracle.compressed_sweeps(u0, C, steps, k, R)
    ref64 = oracle.star7_run(u0, C, steps)
    e_comp = rel_l2(want, ref64)
    # The GPU steps in FP32 and the oracle in FP64 rounded to FP32 once per
    # residency: inputs to each re-encode differ by a few ulp, which changes a
    # block's codes only where a digit at the budget's cut flips; such a flip
    # costs about the block's codec error.  The expected squared difference
    # is then ~ (flip probability ~ ulp / codec error) x (codec error)^2 per
    # residency: rel-L2 ~ sqrt(n_res * 2^-24 * e_comp), bounded with a factor
    # of 10 (measured at 0.08-0.2 of the bound at R = 5, 8, 12 and 16).
    n_res = -(-steps // k)
    assert rel_l2(got, want) <= 10.0 * np.sqrt(n_res * 2.0 ** -24 * e_comp)
    if R == 16:
        assert rel_l2(got, want) <= 1e-5
    # and the job's error against FP64 is the composition's, to that bound
    assert abs(rel_l2(got, ref64) - e_comp) <= 10.0 * np.sqrt(n_res * 2.0 ** -24 * e_comp)


def test_compressed_r16_meets_error_bar():
    u0 = inputs.grf_field((64, 64, 64), seed=2)
    got, _ = run_ooc(u0, 64, k=4, rate=16, slab_planes=16)
    assert rel_l2(got, oracle.star7_run(u0, C, 64)) <= 1e-3


def test_c0_field_ooc():
    u0 = inputs.modes_field(SHAPE, seed=9)
    c0 = inputs.c0_field(SHAPE)
    st = oc.make_star7(C, c0_field=True)
    for R, swb in ((0, True), (8, True), (8, False)):
        got, _ = run_ooc(u0, 8, c0=c0, k=4, rate=R, slab_planes=8, single_buffer=swb,
                         c0_field=True)
        if R == 0:
            want = oc.star7_incore(_dev(u0), C, 8, c0f=_dev(c0)).cpu().numpy()
            assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
            assert rel_l2(got, oracle.star7_run(u0, C, 8, c0)) <= 1e-5
        else:
            codes = oc.compress(_dev(u0), R)
            for _ in range(2):
                u = oc.star7_incore(oc.decompress(codes, SHAPE, R), C, 4, c0f=_dev(c0))
                codes = oc.compress(u, R)
            want = oc.decompress(codes, SHAPE, R).cpu().numpy()
            assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    assert st.c0_is_field == 1


@pytest.mark.parametrize("fuse", [2, 3, 4])
@pytest.mark.parametrize("R", [0, 8])
def test_fused_stencil_launches_equal_single_steps_bitwise(fuse, R):
    u0 = inputs.grf_field(SHAPE, seed=12)
    c0 = inputs.c0_field(SHAPE, seed=13)
    kw = dict(k=4, rate=R, slab_planes=8, c0_field=True, runs=[8, 3])
    want, _ = run_ooc(u0, 0, c0, fuse=1, **kw)
    got, st = run_ooc(u0, 0, c0, fuse=fuse, timing=True, **kw)   # counts need timing
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    assert st["n_stencil"] == 6 * -(-3 // fuse)      # the short sweep of 3 steps


@pytest.mark.parametrize("k,S,steps", [(4, 8, 10), (4, 4, 8), (3, 12, 7), (1, 12, 3), (2, 20, 6)])
def test_region_sharing_uncompressed_equals_incore_bitwise(k, S, steps):
    u0 = inputs.modes_field(SHAPE, seed=14)
    got, st = run_ooc(u0, steps, k=k, rate=0, slab_planes=S, share=True)
    want = oc.star7_incore(_dev(u0), C, steps).cpu().numpy()
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    unshared, st0 = run_ooc(u0, steps, k=k, rate=0, slab_planes=S, share=False)
    assert np.array_equal(got.view(np.uint32), unshared.view(np.uint32))
    assert st["bytes_h2d"] < st0["bytes_h2d"]


@pytest.mark.parametrize("R", [8, 16])
@pytest.mark.parametrize("swb", [True, False])
@pytest.mark.parametrize("k,S,steps", [(4, 8, 12), (3, 12, 7), (4, 4, 8)])
def test_region_sharing_compressed_equals_incore_composition_bitwise(R, swb, k, S, steps):
    u0 = inputs.grf_field(SHAPE, seed=15)
    got, st = run_ooc(u0, steps, k=k, rate=R, slab_planes=S, single_buffer=swb, budget=64 << 20,
                      share=True)
    want = gpu_compressed_incore(u0, R, k, steps)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_region_sharing_with_c0_field_and_split_runs():
    # the field and the c0 slab both share their planes around slab faces
    u0 = inputs.grf_field(SHAPE, seed=16)
    c0 = inputs.c0_field(SHAPE, seed=17)
    for R, swb in ((0, True), (8, True), (8, False)):
        kw = dict(k=4, rate=R, slab_planes=8, c0_field=True, runs=[5, 8], single_buffer=swb,
                  budget=64 << 20)
        a, sa = run_ooc(u0, 0, c0, share=True, **kw)
        b, sb = run_ooc(u0, 0, c0, share=False, **kw)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
        assert sa["bytes_h2d"] < sb["bytes_h2d"]


@pytest.mark.parametrize("R,k,S,runs", [(0, 4, 8, [10]), (0, 3, 12, [4, 7]), (8, 4, 8, [12]),
                                         (16, 3, 12, [5, 2]), (8, 4, 4, [8]), (8, 4, 44, [9])])
def test_in_place_host_level_equals_two_levels_bitwise(R, k, S, runs):
    # one host level updated in place (Algorithm 1, Ensure) computes exactly
    # what the two alternating levels compute
    u0 = inputs.grf_field(SHAPE, seed=18)
    kw = dict(k=k, rate=R, slab_planes=S, budget=64 << 20, runs=runs)
    a, st = run_ooc(u0, 0, in_place=True, **kw)
    b, st2 = run_ooc(u0, 0, in_place=False, **kw)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    assert st["bytes_h2d"] == st2["bytes_h2d"] and st["bytes_d2h"] == st2["bytes_d2h"]


def test_in_place_with_c0_field_and_single_buffer_off():
    u0 = inputs.grf_field(SHAPE, seed=19)
    c0 = inputs.c0_field(SHAPE, seed=20)
    for R, swb in ((0, True), (8, True), (8, False)):
        kw = dict(k=4, rate=R, slab_planes=8, c0_field=True, single_buffer=swb, runs=[6, 5],
                  budget=64 << 20)
        a, _ = run_ooc(u0, 0, c0, in_place=True, **kw)
        b, _ = run_ooc(u0, 0, c0, in_place=False, **kw)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_in_place_without_sharing_is_rejected():
    with pytest.raises(oc.OCError) as e:
        oc.OutOfCore(SHAPE, k=4, rate=8, slab_planes=8, share=False, in_place=True)
    assert e.value.status == oc.OC_ERR_ARG


def test_stats_bytes_and_visits():
    u0 = inputs.modes_field(SHAPE, seed=10)
    _, st = run_ooc(u0, 8, k=4, rate=8, slab_planes=8, timing=True, share=False)
    lb = oc.codec_bytes(SHAPE, 8)
    layer = lb // (SHAPE[0] // 4)
    assert st["slab_visits"] == 2 * 6
    assert st["bytes_d2h"] == 2 * lb
    # each slab also loads one 4-plane layer of halo per interior face
    assert st["bytes_h2d"] == 2 * (lb + 2 * 5 * layer)
    # one fused 4-step stencil launch per slab visit (the default)
    assert st["n_decode"] == 12 and st["n_encode"] == 12 and st["n_stencil"] == 12
    # every cell is updated 8 times; halo recomputation is credited on top
    assert st["cells_stencil"] >= 8 * int(np.prod(SHAPE))
    assert st["ms_decode"] > 0 and st["ms_stencil"] > 0 and st["ms_encode"] > 0


def test_injected_hip_failure_is_reported_and_handle_destroyable():
    u0 = inputs.modes_field(SHAPE, seed=11)
    o = oc.OutOfCore(SHAPE, k=4, rate=8, slab_planes=8)
    o.load(u0)
    o.fail_after(7)
    with pytest.raises(oc.OCError) as e:
        o.run(8)
    assert e.value.status == oc.OC_ERR_HIP
    with pytest.raises(oc.OCError) as e:
        o.run(4)
    assert e.value.status == oc.OC_ERR_STATE
    o.close()


def test_failed_run_leaves_the_last_complete_level_intact():
    # two host levels: a run that fails in its first sweep writes only the
    # level the state is not in
    u0 = inputs.grf_field(SHAPE, seed=21)
    for R in (8, 0):
        o = oc.OutOfCore(SHAPE, k=4, rate=R, slab_planes=8, share=False)
        try:
            o.load(u0)
            o.run(4)                                   # one sweep: the state is in level 1
            want = o.levels[1].numpy().copy()
            o.fail_after(9)
            with pytest.raises(oc.OCError) as e:
                o.run(8)
            assert e.value.status == oc.OC_ERR_HIP
            assert np.array_equal(o.levels[1].numpy(), want)
        finally:
            o.close()


def test_budget_too_small_is_rejected():
    with pytest.raises(oc.OCError) as e:
        oc.OutOfCore(SHAPE, k=4, rate=0, slab_planes=8, budget=1 << 16)
    assert e.value.status == oc.OC_ERR_BUDGET


@pytest.mark.parametrize("shape,kw", [
    ((1, 3, 5), dict(k=1, rate=0, slab_planes=1)),            # one plane, one slab
    ((7, 1, 9), dict(k=2, rate=0, slab_planes=2)),            # a line per plane, ragged last slab
    ((4, 4, 4), dict(k=4, rate=1, slab_planes=4)),            # one block, the lowest rate
    ((4, 4, 4), dict(k=4, rate=32, slab_planes=4)),           # one block, the highest rate
    ((12, 4, 8), dict(k=1, rate=8, slab_planes=4, in_place=True)),
    ((20, 8, 4), dict(k=3, rate=0, slab_planes=3, in_place=True)),
])
def test_degenerate_grids_equal_incore(shape, kw):
    u0 = inputs.grf_field(shape, seed=22) if min(shape) >= 4 else \
        np.random.default_rng(22).standard_normal(shape).astype(np.float32)
    steps = 5
    got, _ = run_ooc(u0, steps, budget=64 << 20, **kw)
    R = kw["rate"]
    if R == 0:
        want = oc.star7_incore(_dev(u0), C, steps).cpu().numpy()
    else:
        want = gpu_compressed_incore(u0, R, kw["k"], steps)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


@pytest.mark.parametrize("in_place", [False, True])
def test_load_store_stage_through_the_free_level(in_place):
    # nz = 132 (8 chunks of 16 planes + a ragged 4), S = 8, k = 1, R = 16: a
    # host level holds two chunks, so load and store stage the caller's
    # pageable field through the level that holds no state; with in_place
    # there is none and the copies go direct.  Both must be exact.
    shape = (132, 32, 32)
    u0 = inputs.grf_field(shape, seed=12)
    o = oc.OutOfCore(shape, C, k=1, rate=16, slab_planes=8, budget=64 << 20, in_place=in_place)
    try:
        o.load(u0)
        got0 = o.store()
        o.run(3)
        got3 = o.store()
        got3b = o.store()
    finally:
        o.close()
    want0 = oracle.decompress(oracle.compress(u0, 16), shape, 16)
    assert np.array_equal(got0.view(np.uint32), want0.view(np.uint32))
    want3 = gpu_compressed_incore(u0, 16, 1, 3)
    assert np.array_equal(got3.view(np.uint32), want3.view(np.uint32))
    assert np.array_equal(got3b.view(np.uint32), want3.view(np.uint32))


def test_overlapping_host_levels_are_rejected():
    # each sweep reads one level and writes the other (and load / store stage
    # through the stateless one): levels that overlap cannot work
    import ctypes
    o = oc.OutOfCore(SHAPE, k=2, rate=16, slab_planes=8, budget=64 << 20)
    try:
        cfg = o.cfg
        h = ctypes.c_void_p()
        for second in (cfg.host_level[0], cfg.host_level[0] + 64):
            bad = oc.Config.from_buffer_copy(cfg)
            bad.host_level[1] = second
            st = oc.lib().oc_create(oc._ref(o.grid), oc._ref(o.stencil), oc._ref(bad), ctypes.byref(h))
            assert st == oc.OC_ERR_ARG
    finally:
        o.close()


# ---- a separate rate for the loaded codes -------------------------------------------------
@pytest.mark.parametrize("R,L", [(3, 8), (5, 9)])
@pytest.mark.parametrize("swb", [True, False])
@pytest.mark.parametrize("k,S,runs", [(4, 8, [12]), (3, 12, [7]), (4, 8, [5, 6]), (2, 44, [0, 4])])
def test_load_rate_ooc_equals_incore_composition_bitwise(R, L, swb, k, S, runs):
    # the first residency after oc_load decodes at the load rate; a second
    # oc_run (or a run after an empty one) continues from codes at R
    u0 = inputs.grf_field(SHAPE, seed=11)
    got, st = run_ooc(u0, sum(runs), runs=runs, k=k, rate=R, slab_planes=S, single_buffer=swb,
                      budget=64 << 20, load_rate=L)
    want = gpu_compressed_incore(u0, R, k, sum(runs), load_rate=L, runs=[r for r in runs if r])
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    assert st["peak_dev_bytes"] == oc.plan_bytes(SHAPE, oc.make_star7(C), k, S, R, swb, 64 << 20,
                                                 share=True, load_rate=L)


def test_load_rate_store_without_steps_decodes_at_the_load_rate():
    u0 = inputs.grf_field(SHAPE, seed=12)
    got, _ = run_ooc(u0, 0, runs=[], k=4, rate=3, slab_planes=8, budget=64 << 20, load_rate=10)
    want = oc.decompress(oc.compress(_dev(u0), 10), SHAPE, 10).cpu().numpy()
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


@pytest.mark.parametrize("shape,S,seed", [(SHAPE, 8, 8), ((64, 64, 64), 16, 8)])
def test_load_rate_close_to_oracle_composition(shape, S, seed):
    steps, k, R, L = 10, 4, 3, 8
    u0 = inputs.grf_field(shape, seed=seed)
    got, _ = run_ooc(u0, steps, k=k, rate=R, slab_planes=S, load_rate=L)
    want = oracle.compressed_sweeps(u0, C, steps, k, R, load_rate=L)
    ref64 = oracle.star7_run(u0, C, steps)
    e_comp = rel_l2(want, ref64)
    n_res = -(-steps // k)
    assert rel_l2(got, want) <= 10.0 * np.sqrt(n_res * 2.0 ** -24 * e_comp)
    # and the load rate helps: the same job with every encode at R is worse
    plain = oracle.compressed_sweeps(u0, C, steps, k, R)
    assert e_comp < rel_l2(plain, ref64)


def test_load_rate_refused_where_unsupported():
    u0 = inputs.grf_field(SHAPE, seed=13)
    with pytest.raises(oc.OCError) as e:
        oc.OutOfCore(SHAPE, k=4, rate=3, slab_planes=8, budget=64 << 20, load_rate=8, fused_codec=True)
    assert e.value.status == oc.OC_ERR_UNSUPPORTED
    with pytest.raises(oc.OCError) as e:
        oc.OutOfCore(SHAPE, k=4, rate=5, slab_planes=8, budget=64 << 20, load_rate=4)
    assert e.value.status == oc.OC_ERR_ARG
    with pytest.raises(oc.OCError) as e:
        oc.OutOfCore(SHAPE, k=4, rate=3, slab_planes=8, budget=64 << 20, load_rate=8, in_place=True)
    assert e.value.status == oc.OC_ERR_UNSUPPORTED
