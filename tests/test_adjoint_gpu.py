"""Adjoint of the out-of-core 7-point path on the GPU, through the C ABI.

Loss L = 1/2 sum over the top plane of u_T^2.  Checked against the FP64
oracle's gradients (raw checkpoints: 1e-5; 16-bit codes: 1e-3), against
central finite differences of the GPU forward on random directions (the loss
is exactly quadratic in u0; along c0 the differences are Richardson
extrapolated, since the loss is a polynomial of degree 2*steps in c0), and
through torch.autograd.
"""
import numpy as np
import pytest

import oracle
from paper_2204_11315_amd import inputs, oc

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

C = (0.4, 0.1, 0.1, 0.1, 0.1, 0.1, 0.1)
SHAPE = (44, 12, 16)
STEPS, EVERY = 12, 4
BUDGET = 200 << 10      # forces several slabs in the forward and the reverse sweeps


def fields():
    u0 = inputs.grf_field(SHAPE, seed=41)
    c0 = inputs.c0_field(SHAPE, seed=5)
    return u0, c0


def top_grad(uT):
    g = np.zeros_like(uT)
    g[-1] = uT[-1]
    return g


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("rate,tol", [(0, 1e-5), (16, 1e-3)])
def test_gradients_vs_oracle(rate, tol):
    u0, c0 = fields()
    adj = oc.Adjoint(SHAPE, C, steps=STEPS, k=2, ckpt_every=EVERY, ckpt_rate=rate, budget=BUDGET)
    try:
        uT = adj.forward(u0, c0)
        g_u0, g_c0 = adj.backward(top_grad(uT))
    finally:
        adj.close()
    L, uT_ref, gu_ref, gc_ref = oracle.star7_grad(u0, C, STEPS, c0)
    assert rel(uT, uT_ref) < 1e-5
    assert rel(g_u0, gu_ref) < tol
    assert rel(g_c0, gc_ref) < tol


def _run_adjoint(rate, every=EVERY, **kw):
    u0, c0 = fields()
    adj = oc.Adjoint(SHAPE, C, steps=STEPS, k=2, ckpt_every=every, ckpt_rate=rate, budget=BUDGET, **kw)
    try:
        uT = adj.forward(u0, c0)
        g_u0, g_c0 = adj.backward(top_grad(uT))
        return (uT, g_u0, g_c0), adj.ooc.stats()["bytes_h2d"]
    finally:
        adj.close()


@pytest.mark.parametrize("rate", [0, 16])
def test_region_sharing_in_reverse_sweeps_is_bitwise_neutral(rate):
    # the shared planes are the same values the slab would copy in (or
    # decode), so sharing changes only the traffic
    a, h2d_a = _run_adjoint(rate, share=True)
    b, h2d_b = _run_adjoint(rate, share=False)
    for x, y in zip(a, b):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32))
    assert h2d_a < h2d_b


@pytest.mark.parametrize("rate,every", [(0, 5), (16, 4)])
def test_fused_recomputation_is_bitwise_neutral(rate, every):
    # the reverse sweeps recompute u from the checkpoint up to four steps per
    # launch; one step per launch gives the same bits
    a, _ = _run_adjoint(rate, every=every)
    b, _ = _run_adjoint(rate, every=every, fuse=1)
    for x, y in zip(a, b):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32))


@pytest.mark.parametrize("rate,fuse", [(16, 0), (0, 0), (16, 1)])
def test_checkpoints_written_by_the_forward_pipeline(rate, fuse):
    # with block-aligned slabs the last sweep of each forward segment writes
    # the next checkpoint itself (codes made on the device from the slab
    # results); 6-plane slabs make them from the host level between segments.
    # Both give the same checkpoint bytes and the same gradients.
    u0, c0 = fields()
    nseg = -(-STEPS // EVERY)
    field = int(np.prod(SHAPE)) * 4
    ck_bytes = field + (nseg - 1) * (oc.codec_bytes(SHAPE, rate) if rate else field)
    out = {}
    for S in (8, 6):
        adj = oc.Adjoint(SHAPE, C, steps=STEPS, k=2, ckpt_every=EVERY, ckpt_rate=rate,
                         budget=1 << 20, slab_planes=S, fuse=fuse)   # fuse 1: two launches
        try:
            uT = adj.forward(u0, c0)
            ck = adj.work[:ck_bytes].numpy().copy()
            g = adj.backward(top_grad(uT))
            out[S] = (ck, uT) + g
        finally:
            adj.close()
    assert np.array_equal(out[8][0], out[6][0])
    for a, b in zip(out[8][1:], out[6][1:]):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_directional_derivatives_vs_central_differences():
    u0, c0 = fields()
    adj = oc.Adjoint(SHAPE, C, steps=STEPS, k=2, ckpt_every=EVERY, ckpt_rate=16, budget=BUDGET)
    try:
        uT = adj.forward(u0, c0)
        g_u0, g_c0 = adj.backward(top_grad(uT))
    finally:
        adj.close()
    fwd = oc.OutOfCore(SHAPE, C, k=2, rate=0, budget=BUDGET, c0_field=True)

    def loss(u, c):
        fwd.load(u.astype(np.float32), c.astype(np.float32))
        fwd.run(STEPS)
        return 0.5 * float(np.sum(fwd.store()[-1].astype(np.float64) ** 2))

    def central(f, eps):
        return (f(eps) - f(-eps)) / (2 * eps)

    rng = np.random.default_rng(43)
    want, got = [], []
    try:
        for _ in range(4):
            d = rng.standard_normal(SHAPE)
            e = inputs.smooth_direction(SHAPE, rng)
            eu = 1e-2 * np.sqrt(np.mean(u0.astype(np.float64) ** 2)) / np.sqrt(np.mean(d ** 2))
            ec = 2e-3 * np.sqrt(np.mean(c0.astype(np.float64) ** 2)) / np.sqrt(np.mean(e ** 2))
            # L is quadratic in u0: the central difference is exact up to rounding
            want.append(central(lambda t: loss(u0 + t * d, c0), eu))
            got.append(np.vdot(g_u0.astype(np.float64), d))
            # L has degree 2*STEPS in c0: Richardson-extrapolated central
            # differences (truncation O(eps^4))
            fc = lambda t: loss(u0, c0 + t * e)
            want.append((4 * central(fc, ec / 2) - central(fc, ec)) / 3)
            got.append(np.vdot(g_c0.astype(np.float64), e))
    finally:
        fwd.close()
    assert rel(got, want) < 1e-3


def test_torch_autograd_function_and_linearity():
    u0, c0 = fields()
    runner = oc.Adjoint(SHAPE, C, steps=STEPS, k=2, ckpt_every=EVERY, ckpt_rate=16, budget=BUDGET)
    try:
        Fn = oc.stencil_function()
        tu = torch.from_numpy(u0.copy()).requires_grad_(True)
        tc = torch.from_numpy(c0.copy()).requires_grad_(True)
        uT = Fn.apply(tu, tc, runner)
        loss = 0.5 * (uT[-1].double() ** 2).sum()
        loss.backward()
        g_u0, g_c0 = runner.backward(2.0 * top_grad(uT.detach().numpy()))
    finally:
        runner.close()
    assert np.allclose(2.0 * tu.grad.numpy(), g_u0, rtol=1e-6, atol=1e-12)
    assert np.allclose(2.0 * tc.grad.numpy(), g_c0, rtol=1e-6, atol=1e-12)


def test_adjoint_needs_checkpoints_and_raw_handle():
    u0, c0 = fields()
    o = oc.OutOfCore(SHAPE, C, k=2, rate=8, budget=BUDGET, c0_field=True)
    try:
        assert oc.lib().oc_adjoint_host_bytes(o.h, STEPS, EVERY, 16) == 0   # coded handle
    finally:
        o.close()
    adj = oc.Adjoint(SHAPE, C, steps=STEPS, k=2, ckpt_every=EVERY, ckpt_rate=16, budget=BUDGET)
    try:
        with pytest.raises(oc.OCError) as e:
            adj.backward(np.zeros(SHAPE, np.float32))
        assert e.value.status == oc.OC_ERR_STATE
    finally:
        adj.close()


def test_load_after_forward_invalidates_the_checkpoints():
    """oc_load replaces the state and the c0 field the checkpoints came from:
    oc_adjoint then refuses (OC_ERR_STATE) until a new forward has run."""
    u0, c0 = fields()
    adj = oc.Adjoint(SHAPE, C, steps=STEPS, k=2, ckpt_every=EVERY, ckpt_rate=16, budget=BUDGET)
    try:
        uT = adj.forward(u0, c0)
        adj.ooc.load(u0, 0.9 * c0)
        with pytest.raises(oc.OCError) as e:
            adj.backward(top_grad(uT))
        assert e.value.status == oc.OC_ERR_STATE
        uT = adj.forward(u0, c0)            # a new forward makes it valid again
        g_u0, _ = adj.backward(top_grad(uT))
    finally:
        adj.close()
    _, _, gu_ref, _ = oracle.star7_grad(u0, C, STEPS, c0)
    assert rel(g_u0, gu_ref) < 1e-3
