"""Dataflow of the 7-point coded schedule (CPU only): the operation list the
executor would issue is replayed in issue order on labelled bytes.  Every byte
of the loaded host level carries the label (0, position); an encode of sweep t
labels the codes it writes (t + 1, position in the coded level); copies (host
to device, device to host, device to device) move labels.  Each decode must
then read exactly the codes of its slab's loaded planes as the previous sweep
(or the load) left them, wherever the schedule keeps them (its own staging
slot, or, for layers shared with the previous slab, that slab's slot), and the
host level the last sweep writes must hold every code of the last sweep.

The happens-before checker proves the order of the list is a legal execution
order (every dependency is issued before its dependant), so the issue-order
replay is what every legal concurrent execution computes.
"""
import re

import numpy as np
import pytest

from paper_2204_11315_amd import oc

ST = oc.make_star7()
TAG = 1 << 32


def parse(dump):
    ops = []
    for line in dump.splitlines():
        if " ev=" in line or " SYNC" in line:
            continue
        f = dict(re.findall(r"(\w+)=(-?\d+)", line))
        z = re.search(r"z=\[(-?\d+),(-?\d+)\)", line)
        ops.append(dict(kind=line.split()[2], **{k: int(v) for k, v in f.items()},
                        z_lo=int(z.group(1)), z_hi=int(z.group(2))))
    return ops


def replay(shape, k, S, R, sweeps, load_rate=0, **kw):
    nz, ny, nx = shape
    h = 4 * -(-k // 4)                               # halo: k planes rounded up to a block layer
    lb = {r: oc.codec_bytes((4, ny, nx), r) for r in (R, load_rate or R)}
    pb = nx * ny * 4
    ops = parse(oc.plan_dump(shape, ST, k, S, R, sweeps, load_rate=load_rate, **kw))
    arena = max(max(o["src"], o["src2"], o["dst"]) for o in ops) + 2 * (nz + 16) * pb
    dev = np.full(arena, -1, np.int64)
    level = (nz // 4) * lb[load_rate or R]
    host = [np.full(level, -1, np.int64), np.full(level, -1, np.int64)]
    host[0][:] = np.arange(level)                    # the load: tag 0
    decodes = 0
    for o in ops:
        kind = o["kind"]
        if kind == "H2D":
            dev[o["dst"]:o["dst"] + o["bytes"]] = host[o["host"]][o["off"]:o["off"] + o["bytes"]]
        elif kind == "D2H":
            host[o["host"]][o["off"]:o["off"] + o["bytes"]] = dev[o["src"]:o["src"] + o["bytes"]]
        elif kind == "DEC" and o["z_hi"] < 0:        # device-to-device move
            dev[o["dst"]:o["dst"] + o["bytes"]] = dev[o["src"]:o["src"] + o["bytes"]].copy()
        elif kind == "DEC":
            t, j = o["sweep"], o["slab"]
            b = lb[o["rate"] or R]
            n = o["z_hi"] * b
            lo = o["bytes"] if o["src2"] >= 0 else 0
            got = np.concatenate([dev[o["src2"]:o["src2"] + lo], dev[o["src"] + lo:o["src"] + n]])
            l0 = max(0, j * S - h)
            want = t * TAG + (l0 // 4) * b + np.arange(n)
            assert np.array_equal(got, want), (t, j, int(np.argmax(got != want)))
            dev[o["dst"]:o["dst"] + o["z_hi"] * 4 * pb] = -2   # FP32 planes
            decodes += 1
        elif kind == "ENC":
            t, j = o["sweep"], o["slab"]
            n = o["z_hi"] * lb[R]
            dev[o["dst"]:o["dst"] + n] = (t + 1) * TAG + (j * S // 4) * lb[R] + np.arange(n)
        elif kind == "STAR7":
            dev[o["dst"] + o["z_lo"] * pb:o["dst"] + o["z_hi"] * pb] = -2
    return host, decodes, (nz // 4) * lb[R]


CASES = [((40, 12, 16), 4, 8), ((44, 8, 8), 4, 12), ((16, 8, 8), 4, 4), ((36, 8, 12), 3, 8),
         ((44, 24, 40), 4, 8), ((48, 8, 8), 4, 4), ((24, 8, 8), 1, 12), ((64, 8, 8), 4, 16)]


@pytest.mark.parametrize("shape,k,S", CASES)
@pytest.mark.parametrize("share", [False, True])
@pytest.mark.parametrize("slots", [0, 2, 4])
def test_every_decode_reads_its_slabs_codes(shape, k, S, share, slots):
    R, sweeps = 8, 3
    host, decodes, level = replay(shape, k, S, R, sweeps, share=share, ring_slots=slots,
                                  prefetch=slots - 1 if slots else 0)
    assert decodes == sweeps * len(range(0, shape[0], S))
    last = sweeps % 2                                # two host levels: sweep t writes (t + 1) mod 2
    assert np.array_equal(host[last][:level], sweeps * TAG + np.arange(level))


@pytest.mark.parametrize("shape,k,S", [((40, 12, 16), 4, 8), ((16, 8, 8), 4, 4), ((48, 8, 8), 4, 4)])
def test_load_rate_first_sweep_reads_the_loaded_codes(shape, k, S):
    host, decodes, level = replay(shape, k, S, 3, 3, load_rate=8, share=True)
    assert np.array_equal(host[1][:level], 3 * TAG + np.arange(level))


@pytest.mark.parametrize("shape,k,S", [((40, 12, 16), 4, 8), ((16, 8, 8), 4, 4)])
def test_in_place_level(shape, k, S):
    host, decodes, level = replay(shape, k, S, 8, 3, share=True, in_place=True)
    assert np.array_equal(host[0][:level], 3 * TAG + np.arange(level))


def test_a_misrouted_decode_is_caught():
    # the replay itself: a decode pointed one layer off reads another slab's codes
    shape, k, S, R = (40, 12, 16), 4, 8, 8
    ops = parse(oc.plan_dump(shape, ST, k, S, R, 2, share=True))
    dec = next(o for o in ops if o["kind"] == "DEC" and o["z_hi"] > 0 and o["slab"] == 2)
    lb = oc.codec_bytes((4, 12, 16), R)
    dump = oc.plan_dump(shape, ST, k, S, R, 2, share=True)
    bad = dump.replace("src=%d " % dec["src"], "src=%d " % (dec["src"] + lb), 1)
    assert bad != dump
    orig = oc.plan_dump
    try:
        oc.plan_dump = lambda *a, **kw: bad
        with pytest.raises(AssertionError):
            replay(shape, k, S, R, 2, share=True)
    finally:
        oc.plan_dump = orig
