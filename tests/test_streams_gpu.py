"""The stream check: whether two streams run their kernels side by side (the
pipeline overlaps the copy-back kernel of one slab with the kernels of the
next, Sec. 4.2, Fig. 4)."""
import pytest

from paper_2204_11315_amd import oc

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_one_stream_is_serialized():
    s = torch.cuda.Stream()
    assert oc.stream_overlap(s, s) < 0.02


def test_overlap_of_two_streams_is_a_share():
    a, b = torch.cuda.Stream(), torch.cuda.Stream()
    # side by side or not depends on the hardware queues the runtime gave the
    # streams; the probe reports a share of the shorter run either way
    assert 0.0 <= oc.stream_overlap(a, b) <= 1.0


def test_pipeline_streams_were_probed():
    streams = oc.pipeline_streams()
    assert len(streams) == 3
    assert 0.0 <= oc.pipeline_stream_overlap() <= 1.0


def test_null_arguments_are_rejected():
    assert oc.lib().oc_stream_overlap(None, None, None) == oc.OC_ERR_ARG
