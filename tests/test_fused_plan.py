"""Planner and race checker for the fused codec kernel (one launch per coded
slab: decode, k 7-point steps, encode; oc_config.fused_codec), on the CPU.

* the operation list is race-free and every wait in it is needed (dropping
  any one is caught), with and without region sharing, with other ring sizes
  and with one host level updated in place;
* each slab visit is one FUSED launch and nothing else on the kernel stream
  (no decode, stencil or encode launches; only the overlap copies of region
  sharing), and its codes go back from the slot's output region;
* the arena holds only the ring of coded slots (input layers and interior
  layers), i.e. no FP32 working buffer: 102 MiB at R = 8 on the
  512 x 512 x 2048 job against 198 MiB for three kernels;
* combinations the kernel does not cover are refused (OC_ERR_UNSUPPORTED).
"""
import pytest

from paper_2204_11315_amd import oc

ST = oc.make_star7()
MiB = 1 << 20
CASES = [((40, 12, 16), 4, 8), ((44, 8, 8), 4, 12), ((16, 8, 8), 4, 4), ((36, 8, 12), 3, 8),
         ((44, 24, 40), 4, 8), ((48, 8, 8), 4, 4), ((24, 8, 8), 1, 12), ((64, 8, 8), 2, 16),
         ((28, 64, 60), 3, 12)]


def _lines(dump, kind):
    return [line for line in dump.splitlines() if f" {kind} " in line]


def _field(line, name):
    return int(line.split(name + "=")[1].split()[0])


@pytest.mark.parametrize("shape,k,S", CASES)
@pytest.mark.parametrize("share", [False, True])
@pytest.mark.parametrize("R", [1, 8, 16])
def test_fused_operation_list_race_free_and_minimal(shape, k, S, share, R):
    for slots, pre in ((0, 0), (2, 1), (4, 3)):
        kw = dict(ring_slots=slots, prefetch=pre, share=share, fused_codec=True)
        n, nw = oc.plan_ops(shape, ST, k, S, R, 3, **kw)
        assert n > 0 and nw > 0
        assert oc.check_plan(shape, ST, k, S, R, 3, **kw) == 0
        for i in range(nw):
            assert oc.check_plan(shape, ST, k, S, R, 3, mutate=1, i=i, **kw) > 0, (slots, pre, i)
        assert oc.check_plan(shape, ST, k, S, R, 3, mutate=2, **kw) > 0


@pytest.mark.parametrize("shape,k,S", CASES)
def test_fused_in_place_race_free(shape, k, S):
    kw = dict(share=True, in_place=True, fused_codec=True)
    n, nw = oc.plan_ops(shape, ST, k, S, 8, 3, **kw)
    assert oc.check_plan(shape, ST, k, S, 8, 3, **kw) == 0
    for i in range(nw):
        assert oc.check_plan(shape, ST, k, S, 8, 3, mutate=1, i=i, **kw) > 0, i
    assert oc.check_plan(shape, ST, k, S, 8, 3, mutate=4, **kw) > 0


@pytest.mark.parametrize("share", [False, True])
def test_one_fused_launch_per_slab_visit(share):
    shape, k, S, R, sweeps = (44, 24, 40), 4, 8, 8, 3
    d = oc.plan_dump(shape, ST, k, S, R, sweeps, share=share, fused_codec=True)
    slabs = len(range(0, shape[0], S))
    fused = _lines(d, "FUSED")
    assert len(fused) == sweeps * slabs
    assert not _lines(d, "STAR7") and not _lines(d, "ENC")
    # the only DEC ops left are the overlap copies of region sharing
    decs = _lines(d, "DEC")
    assert all("z=[0,-1)" in line for line in decs)
    assert len(decs) == (sweeps * (slabs - 1) if share else 0)
    # every launch writes past its slot's input layers, and the copy-back of
    # the slab reads exactly those bytes
    lb = oc.codec_bytes((4, shape[1], shape[2]), R)
    outs = {(_field(f, "sweep"), _field(f, "slab")): (_field(f, "dst"), _field(f, "bytes")) for f in fused}
    for f in fused:
        assert _field(f, "dst") - _field(f, "src") >= (S + 8) // 4 * lb
        assert _field(f, "lv") == k
    for line in _lines(d, "D2H"):
        dst, nbytes = outs[(_field(line, "sweep"), _field(line, "slab"))]
        assert (_field(line, "src"), _field(line, "bytes")) == (dst, nbytes)


def test_fused_last_sweep_runs_the_remaining_steps():
    d = oc.plan_dump((40, 12, 16), ST, 4, 8, 8, 2, fused_codec=True)
    # build_ops gives the last sweep k steps here; the executor passes
    # steps mod k for a short last sweep (GPU tests cover it)
    assert {_field(f, "lv") for f in _lines(d, "FUSED")} == {4}


def test_fused_arena_is_the_ring_of_coded_slots():
    C2 = (2048, 512, 512)
    three = oc.plan_bytes(C2, ST, 4, 64, 8, budget=512 * MiB)
    fused = oc.plan_bytes(C2, ST, 4, 64, 8, budget=512 * MiB, fused_codec=True)
    assert three == 198 * MiB
    # 3 slots x (18 input + 16 interior layers) x 1 MiB of codes at R = 8
    assert fused == 3 * (18 + 16) * MiB == 102 * MiB
    assert oc.plan_bytes(C2, ST, 4, 64, 16, budget=512 * MiB, fused_codec=True) == 3 * 34 * 2 * MiB
    # small grids: at least two FP32 chunks of 4 planes and their codes, which
    # oc_load / oc_store stage through the arena
    tiny = oc.plan_bytes((16, 8, 8), ST, 4, 4, 1, fused_codec=True)
    assert tiny >= 2 * 4 * 8 * 8 * 4


@pytest.mark.parametrize("kw", [dict(R=0), dict(R=17), dict(k=5), dict(k=8), dict(c0=True)])
def test_fused_refuses_what_the_kernel_does_not_cover(kw):
    R, k = kw.get("R", 8), kw.get("k", 4)
    st = oc.make_star7(c0_field=True) if kw.get("c0") else ST
    shape = (40, 12, 16)
    assert oc.plan_bytes(shape, st, k, 8, R, fused_codec=True) == 0
    assert oc.check_plan(shape, st, k, 8, R, 2, fused_codec=True) == oc.OC_ERR_UNSUPPORTED


def test_fused_refuses_the_wave_stencil():
    st = oc.make_wave25(10.0, 1e-3, (4, 4, 4), 15.0, 0.1)
    assert oc.check_plan((48, 16, 16), st, 2, 16, 12, 2, fused_codec=True) == oc.OC_ERR_UNSUPPORTED
