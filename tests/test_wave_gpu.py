"""25-point acoustic wave (Sec. 6 workload) on the GPU, through the C ABI.

* in-core FP32 kernel vs the FP64 oracle (layered velocity, Ricker source);
* out-of-core uncompressed == in-core, bitwise, across slabs and sweeps;
* out-of-core compressed (single working buffer) == the in-core composition
  built from the same kernels (codes of p^n, p^{n-1} and the velocity, decoded
  every sweep), bitwise; and close to the oracle.
"""
import numpy as np
import pytest

import oracle
from paper_2204_11315_amd import inputs, oc

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SHAPE = (40, 24, 32)            # 5 slabs of 8 planes
H, F = 10.0, 15.0
T0 = 1.0 / F
SRC = (16, 12, 20)


def setup():
    vel = inputs.layered_velocity(SHAPE, seed=4)
    dt = 0.4 * H / float(vel.max())
    st = oc.make_wave25(H, dt, SRC, F, T0)
    rng = np.random.default_rng(31)
    # a smooth nonzero start so that every slab carries signal
    p0 = (inputs.modes_field(SHAPE, seed=32, noise=0.0) * 1e-3).astype(np.float32)
    pm1 = (p0 * 0.999).astype(np.float32)
    return vel, dt, st, p0, pm1


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def gpu_incore(p0, pm1, vel, st, n0, steps):
    dp, dc = oc.wave25_incore(_dev(pm1), _dev(p0), _dev(vel), st, n0, steps)
    return dc.cpu().numpy(), dp.cpu().numpy()


def test_incore_vs_fp64_oracle():
    # the FP32 leapfrog against FP64: 1.3e-6 after 20 steps (growing from
    # 5e-8 after one step, about linearly in the step count), inside the
    # 1e-5 bar of the uncompressed path
    vel, dt, st, p0, pm1 = setup()
    cur, prev = gpu_incore(p0, pm1, vel, st, 0, 20)
    rp, rc = oracle.wave25_run(pm1, p0, vel, H, dt, SRC, F, T0, 0, 20)
    assert rel_l2(cur, rc) < 1e-5
    assert rel_l2(prev, rp) < 1e-5


def test_source_only_first_step_matches_oracle():
    vel, dt, st, _, _ = setup()
    z = np.zeros(SHAPE, np.float32)
    cur, prev = gpu_incore(z, z, vel, st, 0, 1)
    _, rc = oracle.wave25_run(z, z, vel, H, dt, SRC, F, T0, 0, 1)
    assert np.count_nonzero(cur) == 1
    assert abs(cur[SRC[2], SRC[1], SRC[0]] - rc[SRC[2], SRC[1], SRC[0]]) <= 1e-6 * abs(rc).max()


@pytest.mark.parametrize("k,S,steps", [(2, 8, 6), (2, 8, 5), (1, 12, 3), (3, 40, 6), (3, 4, 7)])
@pytest.mark.parametrize("share,in_place", [(True, False), (False, False), (True, True)])
def test_ooc_uncompressed_equals_incore_bitwise(k, S, steps, share, in_place):
    # with sharing, each slab sets the planes the next one shares aside
    # before the leapfrog overwrites them; in place needs that sharing
    vel, dt, st, p0, pm1 = setup()
    o = oc.OutOfCore(SHAPE, k=k, rate=0, slab_planes=S, budget=64 << 20, stencil=st, share=share,
                     in_place=in_place)
    try:
        o.load(p0, pm1, vel)
        o.run(steps)
        cur, prev = o.store()
    finally:
        o.close()
    wc, wp = gpu_incore(p0, pm1, vel, st, 0, steps)
    assert np.array_equal(cur.view(np.uint32), wc.view(np.uint32))
    assert np.array_equal(prev.view(np.uint32), wp.view(np.uint32))


def gpu_compressed_composition(p0, pm1, vel, st, R, k, steps):
    cp, cm = oc.compress(_dev(p0), R), oc.compress(_dev(pm1), R)
    v = oc.decompress(oc.compress(_dev(vel), R), SHAPE, R)
    done = 0
    while done < steps:
        s = min(k, steps - done)
        dc, dp = oc.decompress(cp, SHAPE, R), oc.decompress(cm, SHAPE, R)
        dp, dc = oc.wave25_incore(dp, dc, v, st, done, s)
        cp, cm = oc.compress(dc, R), oc.compress(dp, R)
        done += s
    return oc.decompress(cp, SHAPE, R).cpu().numpy(), oc.decompress(cm, SHAPE, R).cpu().numpy()


@pytest.mark.parametrize("R", [12, 16])
@pytest.mark.parametrize("swb", [True, False])
@pytest.mark.parametrize("share,in_place", [(True, False), (False, False), (True, True)])
def test_ooc_compressed_equals_incore_composition_bitwise(R, swb, share, in_place):
    vel, dt, st, p0, pm1 = setup()
    o = oc.OutOfCore(SHAPE, k=2, rate=R, slab_planes=8, budget=64 << 20, stencil=st,
                     single_buffer=swb, share=share, in_place=in_place)
    try:
        o.load(p0, pm1, vel)
        o.run(6)
        cur, prev = o.store()
    finally:
        o.close()
    wc, wp = gpu_compressed_composition(p0, pm1, vel, st, R, 2, 6)
    assert np.array_equal(cur.view(np.uint32), wc.view(np.uint32))
    assert np.array_equal(prev.view(np.uint32), wp.view(np.uint32))
    _, rc = oracle.wave25_run(pm1, p0, vel, H, dt, SRC, F, T0, 0, 6)
    assert rel_l2(cur, rc) < (2e-3 if R == 12 else 2e-4)


def test_ooc_split_runs_keep_source_time():
    vel, dt, st, p0, pm1 = setup()
    outs = []
    for runs in ([6], [2, 4]):
        o = oc.OutOfCore(SHAPE, k=2, rate=0, slab_planes=8, budget=64 << 20, stencil=st)
        try:
            o.load(p0, pm1, vel)
            for r in runs:
                o.run(r)
            outs.append(o.store()[0])
        finally:
            o.close()
    assert np.array_equal(outs[0].view(np.uint32), outs[1].view(np.uint32))


def _misaligned(a):
    # the same values one float past a 16-byte boundary: the launch then takes
    # the one-x-per-lane kernel even when nx % 4 == 0
    buf = torch.empty(a.size + 1, dtype=torch.float32, device="cuda")
    v = buf[1:].view(a.shape)
    v.copy_(torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)))
    return v


@pytest.mark.parametrize("shape,src", [(SHAPE, SRC), ((12, 6, 264), (260, 3, 6)), ((9, 5, 516), (257, 2, 4))])
def test_four_x_kernel_equals_one_x_kernel_bitwise(shape, src):
    vel = inputs.layered_velocity(shape, seed=4)
    dt = 0.4 * H / float(vel.max())
    st = oc.make_wave25(H, dt, src, F, T0)
    p0 = (inputs.modes_field(shape, seed=32, noise=0.0) * 1e-3).astype(np.float32)
    pm1 = (p0 * 0.999).astype(np.float32)
    for steps in (1, 6):
        wp, wc = oc.wave25_incore(_dev(pm1), _dev(p0), _dev(vel), st, 0, steps)
        mp, mc = oc.wave25_incore(_misaligned(pm1), _misaligned(p0), _misaligned(vel), st, 0, steps)
        assert np.array_equal(wc.cpu().numpy().view(np.uint32), mc.cpu().numpy().view(np.uint32))
        assert np.array_equal(wp.cpu().numpy().view(np.uint32), mp.cpu().numpy().view(np.uint32))
    rp, rc = oracle.wave25_run(pm1, p0, vel, H, dt, src, F, T0, 0, 6)
    assert rel_l2(wc.cpu().numpy(), rc) < 1e-5
