"""Pipelined runs equal runs with no overlap at all, bitwise (through the C ABI).

The executor can wait for every operation to finish before issuing the next
(oc_debug_serialize).  A missing or misplaced wait in the pipelined operation
list would let a kernel or a copy touch a buffer too early or too late; the
comparison catches that on the GPU itself, beside the CPU race checker.
"""
import numpy as np
import pytest

from paper_2204_11315_amd import inputs, oc

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

C = (0.4, 0.1, 0.1, 0.1, 0.1, 0.1, 0.1)
SHAPE = (44, 24, 40)


def _run(u0, runs, serialize, aux=None, vel=None, **kw):
    o = oc.OutOfCore(u0.shape, **kw)
    try:
        o.serialize(serialize)
        o.load(u0, aux, vel)
        for s in runs:
            o.run(s)
        out = o.store()
        return out if isinstance(out, tuple) else (out,)
    finally:
        o.close()


def _same(a, b):
    for x, y in zip(a, b):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32))


@pytest.mark.parametrize("kw", [
    dict(k=4, rate=8, slab_planes=8),
    dict(k=4, rate=8, slab_planes=8, share=False),
    dict(k=4, rate=8, slab_planes=8, in_place=True),
    dict(k=3, rate=16, slab_planes=12, single_buffer=False),
    dict(k=4, rate=0, slab_planes=8),
    dict(k=4, rate=0, slab_planes=8, in_place=True),
    dict(k=3, rate=0, slab_planes=8, fuse=2),
    dict(k=4, rate=9, slab_planes=4, ring_slots=2, prefetch=1),
])
def test_star7_pipelined_equals_serialized(kw):
    u0 = inputs.grf_field(SHAPE, seed=31)
    kw = dict(kw, budget=64 << 20)
    _same(_run(u0, [6, 7], False, **kw), _run(u0, [6, 7], True, **kw))


@pytest.mark.parametrize("rate", [0, 8])
def test_star7_c0_field_pipelined_equals_serialized(rate):
    u0 = inputs.grf_field(SHAPE, seed=32)
    c0 = inputs.c0_field(SHAPE, seed=33)
    kw = dict(k=4, rate=rate, slab_planes=8, c0_field=True, budget=64 << 20)
    _same(_run(u0, [9], False, c0, **kw), _run(u0, [9], True, c0, **kw))


@pytest.mark.parametrize("rate,in_place", [(0, False), (0, True), (12, False), (12, True)])
def test_wave_pipelined_equals_serialized(rate, in_place):
    shape = (40, 24, 32)
    vel = inputs.layered_velocity(shape, seed=4)
    dt = 0.4 * 10.0 / float(vel.max())
    st = oc.make_wave25(10.0, dt, (16, 12, 20), 15.0, 1.0 / 15)
    p0 = np.zeros(shape, np.float32)
    kw = dict(k=2, rate=rate, slab_planes=8, stencil=st, budget=64 << 20, in_place=in_place)
    _same(_run(p0, [6], False, p0, vel, **kw), _run(p0, [6], True, p0, vel, **kw))


def test_adjoint_pipelined_equals_serialized():
    u0 = inputs.grf_field((44, 12, 16), seed=41)
    c0 = inputs.c0_field((44, 12, 16), seed=5)
    out = []
    for ser in (False, True):
        adj = oc.Adjoint((44, 12, 16), C, steps=12, k=2, ckpt_every=4, ckpt_rate=16,
                         budget=200 << 10, slab_planes=8)
        try:
            adj.ooc.serialize(ser)
            uT = adj.forward(u0, c0)
            g = np.zeros_like(uT)
            g[-1] = uT[-1]
            out.append((uT,) + adj.backward(g))
        finally:
            adj.close()
    _same(out[0], out[1])
