"""The allocation-free codec round trip (oc_codec_error_noalloc) against the
entry point it varies (oc_codec_error, which takes a caller's workspace):
the same kernels over the same blocks in the same order, so the three FP64
results agree bit for bit; two calls in a row on one device, the second on a
smaller field (the static scratch keeps the first call's partial sums, which
the second must not read); an input beyond the fixed scratch is rejected on
the host before anything is enqueued."""
import numpy as np
import pytest

from paper_2204_11315_amd import inputs, oc

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _bits(t):
    return np.array(t, dtype=np.float64).view(np.uint64)


@pytest.mark.parametrize("R", [8, 16, 17])
def test_noalloc_equals_workspace_entry_point_on_two_calls(R):
    big = _dev(inputs.grf_field((64, 96, 128), seed=11))        # 12,288 blocks
    small = _dev(inputs.grf_field((8, 20, 36), seed=12) * 3.0)   # 90 blocks
    out = torch.empty(3, dtype=torch.float64, device="cuda")
    a1 = oc.codec_error_noalloc(big, R, out=out)
    a2 = oc.codec_error_noalloc(small, R, out=out)
    b1 = oc.codec_error(big, R)
    b2 = oc.codec_error(small, R)
    assert np.array_equal(_bits(a1), _bits(b1))
    assert np.array_equal(_bits(a2), _bits(b2))
    assert a1 != a2 and a2[1] > 0.0


def test_noalloc_rejects_inputs_beyond_the_scratch():
    # 87,382 workgroups of 256 blocks at R = 8: one more than the scratch holds;
    # the size check runs on the host, so the tensor need not hold that many
    # cells (nothing is launched)
    t = torch.zeros(16, dtype=torch.float32, device="cuda")
    nz, ny, nx = 4 * 87382, 4 * 16, 4 * 16
    st = oc.lib().oc_codec_error_noalloc(oc.ctypes.c_void_p(t.data_ptr()), nx, ny, nz, 8,
                                         oc.ctypes.c_void_p(t.data_ptr()), None)
    assert st == oc.OC_ERR_TOO_LARGE
    assert oc.status_str(st) != "unknown status"
