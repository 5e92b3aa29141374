"""The torch.autograd.Function wrapper of the adjoint, on the CPU with a
stand-in runner (the wrapper only marshals arrays; the runner's forward and
backward are the library's oc_forward_ckpt / oc_adjoint on a GPU).

A runner keeps the checkpoints of its latest forward only, so a backward whose
forward was followed by another forward on the same runner must raise instead
of returning the later forward's gradient."""
import numpy as np
import pytest

from paper_2204_11315_amd import oc

torch = pytest.importorskip("torch")


class LinearRunner:
    """u_T = a * u0 (c0 ignored): dL/du0 = a * gT, dL/dc0 = 0.  `generation`
    counts forwards, as oc.Adjoint does."""

    def __init__(self, a):
        self.a = a
        self.generation = 0

    def forward(self, u0, c0):
        self.generation += 1
        return (self.a * u0).astype(np.float32)

    def backward(self, gT):
        return (self.a * gT).astype(np.float32), np.zeros_like(gT)


def test_backward_of_the_latest_forward():
    Fn = oc.stencil_function()
    r = LinearRunner(3.0)
    u = torch.ones(4, 4, 4, requires_grad=True)
    c = torch.full((4, 4, 4), 0.4, requires_grad=True)
    Fn.apply(u, c, r).sum().backward()
    assert torch.equal(u.grad, torch.full((4, 4, 4), 3.0))
    assert torch.equal(c.grad, torch.zeros(4, 4, 4))


def test_backward_after_a_newer_forward_on_the_same_runner_raises():
    Fn = oc.stencil_function()
    r = LinearRunner(2.0)
    u1 = torch.ones(4, 4, 4, requires_grad=True)
    u2 = torch.ones(4, 4, 4, requires_grad=True)
    c = torch.full((4, 4, 4), 0.4)
    y1 = Fn.apply(u1, c, r)
    y2 = Fn.apply(u2, c, r)
    with pytest.raises(RuntimeError, match="another forward"):
        y1.sum().backward()
    y2.sum().backward()            # the latest forward still differentiates
    assert torch.equal(u2.grad, torch.full((4, 4, 4), 2.0))
