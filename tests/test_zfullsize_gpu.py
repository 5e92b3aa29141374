"""Full-size out-of-core runs (512 x 512 x 2048, 512 MiB device budget, S = 64,
k = 4, 64 steps) in the configuration the benchmark times, checked on sampled
outputs: for a sample cell the oracle advances only the box of its dependency
cone (half-width = steps), clipped to the grid, which reproduces the full-grid
value exactly.
"""
import numpy as np
import pytest

import oracle
from paper_2204_11315_amd import inputs, oc

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

C = (0.4, 0.1, 0.1, 0.1, 0.1, 0.1, 0.1)
SHAPE = (2048, 512, 512)
STEPS = 64


@pytest.fixture(scope="module")
def u0():
    return inputs.grf_field(SHAPE, seed=2)


def sampled_reference(u0, pts, steps):
    out = []
    for (z, y, x) in pts:
        lo = [max(0, v - steps) for v in (z, y, x)]
        hi = [min(n, v + steps + 1) for v, n in zip((z, y, x), SHAPE)]
        box = u0[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
        # box faces inside the grid are not true boundaries, but their
        # influence travels one cell per step and never reaches the centre
        r = oracle.star7_run(box, C, steps)
        out.append(r[z - lo[0], y - lo[1], x - lo[2]])
    return np.array(out)


def sample_points():
    rng = np.random.default_rng(21)
    pts = [(0, 0, 0), (2047, 511, 511), (64, 256, 256), (63, 10, 500), (1024, 0, 300)]
    for _ in range(7):
        pts.append(tuple(int(rng.integers(0, n)) for n in SHAPE))
    return pts


def run_full(u0, R, fused=False, load_rate=0):
    o = oc.OutOfCore(SHAPE, k=4, rate=R, budget=512 << 20, slab_planes=64, fused_codec=fused,
                     load_rate=load_rate)
    try:
        o.load(u0)
        o.run(STEPS)
        return o.store(), o.stats()
    finally:
        o.close()


# R = 5 is the smallest uniform rate within 1e-3 over the full grid (6.6e-4,
# measured by the benchmark; R = 8: 8.3e-5); R = 3 with the load encoded at 5
# bits (the fastest leg within the budget): 7.7e-4, at 6 bits: 5.2e-4.  On 12
# sampled cells the bar is looser.
@pytest.mark.parametrize("R,L,tol", [(0, 0, 1e-5), (16, 0, 1e-4), (8, 0, 1e-3), (5, 0, 3e-3),
                                     (3, 5, 3e-3), (3, 6, 3e-3)])
def test_fullsize_sampled_vs_oracle(u0, R, L, tol):
    got, st = run_full(u0, R, load_rate=L)
    pts = sample_points()
    want = sampled_reference(u0, pts, STEPS)
    have = np.array([got[p] for p in pts], dtype=np.float64)
    assert np.linalg.norm(have - want) <= tol * np.linalg.norm(want)
    assert st["n_slabs"] == 32 and st["slab_visits"] == 32 * 16
    MiB = 1 << 20
    assert st["peak_dev_bytes"] == {(0, 0): 432 * MiB, (16, 0): 252 * MiB, (8, 0): 198 * MiB,
                                    (5, 0): int(177.75 * MiB), (3, 5): int(177.75 * MiB),
                                    (3, 6): int(184.5 * MiB)}[R, L]
    if (R, L) in ((5, 0), (8, 0)):
        # the fused codec kernel at full size: the same output, in 63.75 / 102 MiB
        fused, sf = run_full(u0, R, fused=True)
        assert np.array_equal(fused.view(np.uint32), got.view(np.uint32))
        assert sf["peak_dev_bytes"] == {5: int(63.75 * MiB), 8: 102 * MiB}[R] and sf["n_slabs"] == 32
