"""Host-side logic of bench.py (CPU only): the one-GPU guard, the host-link
roofline and the per-kernel roofline arithmetic on synthetic figures."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _link(ah, ad, xh, xd):
    return {"h2d_alone": ah, "d2h_alone": ad, "h2d_with_d2h": xh, "d2h_with_h2d": xd}


def test_link_roofline_closed_forms(bench):
    B = 8e9
    leg = {"bytes_h2d": B, "bytes_d2h": B, "ms_per_job": 500.0}
    # both directions at full rate together: the bound is one direction's time
    r = bench.link_roofline(leg, _link(40, 40, 40, 40))
    assert r["bound_ms"] == pytest.approx(B / 40e9 * 1e3)
    # sharing halves each rate: running both at once or one after the other
    # takes the same time
    r = bench.link_roofline(leg, _link(40, 40, 20, 20))
    assert r["bound_ms"] == pytest.approx(2 * B / 40e9 * 1e3)
    assert r["frac"] == pytest.approx(r["bound_ms"] / 500.0)
    # one direction only: its alone rate
    r = bench.link_roofline({"bytes_h2d": B, "bytes_d2h": 0, "ms_per_job": 500.0}, _link(50, 40, 30, 30))
    assert r["bound_ms"] == pytest.approx(B / 50e9 * 1e3)


def test_link_roofline_is_a_lower_bound_of_every_split(bench):
    # no split of the job's time between "both busy" and "each alone" beats it
    leg = {"bytes_h2d": 6e9, "bytes_d2h": 4e9, "ms_per_job": 1000.0}
    link = _link(55, 43, 47, 41)
    bound = bench.link_roofline(leg, link)["bound_ms"] * 1e-3
    bh, bd = 6e9, 4e9
    for i in range(201):
        tc = i / 200 * max(bh / 47e9, bd / 41e9)
        t = tc + max(0.0, bh - tc * 47e9) / 55e9 + max(0.0, bd - tc * 41e9) / 43e9
        assert t >= bound * (1 - 1e-12)


def test_kernel_roofline_arithmetic(bench):
    rate = 5
    st = {"ms_decode": 2.0, "n_decode": 20, "ms_encode": 1.0, "n_encode": 20, "ms_stencil": 3.0,
          "n_stencil": 30, "ms_fused": 0.0, "n_fused": 0, "blocks_decode": 20 * 1000,
          "blocks_encode": 20 * 800, "bytes_stencil": 30 * 1e6}
    k = bench.kernel_roofline([st], rate)
    assert set(k) == {"decode", "encode", "stencil"}
    d = k["decode"]
    assert d["avg_ms"] == pytest.approx(0.1) and d["launches"] == 20
    assert d["bytes_per_launch"] == pytest.approx(1000 * (8 * rate + 256))
    assert d["gbs"] == pytest.approx(1000 * (8 * rate + 256) / 1e-4 / 1e9)
    assert k["stencil"]["bytes_per_launch"] == pytest.approx(1e6)
    roof = bench.roofline_of(k, rate)
    assert roof["kernel"] == "stencil"            # the largest total time
    assert roof["frac"] == pytest.approx(roof["achieved"] / roof["peak"])
    assert roof["unit"] == "GB/s" and roof["bound"] == "hbm"


def test_kernel_roofline_counts_the_load_rate_sweep(bench):
    # one sweep of the STEPS / K decodes L-bit codes, the others R-bit codes
    rate, lr = 3, 8
    sweeps = bench.STEPS // bench.K
    st = {"ms_decode": 1.6, "n_decode": 16, "ms_encode": 1.0, "n_encode": 16, "ms_stencil": 3.0,
          "n_stencil": 16, "ms_fused": 0.0, "n_fused": 0, "blocks_decode": sweeps * 1000,
          "blocks_encode": sweeps * 900, "bytes_stencil": 16 * 1e6}
    d = bench.kernel_roofline([st], rate, lr)["decode"]
    per_launch = ((sweeps - 1) * 1000 * (8 * rate + 256) + 1000 * (8 * lr + 256)) / 16
    assert d["bytes_per_launch"] == pytest.approx(per_launch)
    e = bench.kernel_roofline([st], rate, lr)["encode"]
    assert e["bytes_per_launch"] == pytest.approx(sweeps * 900 * (256 + 8 * rate) / 16)


def test_leg_names(bench):
    assert bench.leg_name(0) == "0" and bench.leg_name(5) == "5"
    assert bench.leg_name(3, 8) == "3:8"


def _legs(spec):
    # spec: name -> (GCell/s, rel-L2 or None)
    legs = {}
    for n, (g, e) in spec.items():
        r, lr = (int(v) for v in n.split(":")) if ":" in n else (int(n), 0)
        legs[n] = {"gcell_per_s": g, "error_vs_fp64": None if e is None else {"rel_l2": e},
                   "rate_bits": r, "load_rate_bits": lr or r}
    return legs


def test_headline_is_the_fastest_leg_within_the_budget(bench):
    legs = _legs({"0": (34, 1e-6), "4": (290, 1.3e-3), "5": (237, 6.6e-4), "8": (146, 8e-5),
                  "2:8": (364, 1.2e-3), "3:5": (342, 7.7e-4), "3:6": (335, 5.2e-4)})
    head, how, met, frate = bench.choose_legs(legs, 0, 1e-3, "full")
    assert (head, met) == ("3:5", True) and how.startswith("fastest leg")
    assert frate == 5                      # the smallest uniform rate within the budget
    # a uniform headline takes the fused kernel at its own rate
    legs["3:5"]["error_vs_fp64"]["rel_l2"] = 2e-3
    legs["3:6"]["error_vs_fp64"]["rel_l2"] = 2e-3
    assert bench.choose_legs(legs, 0, 1e-3, "full")[0::3] == ("5", 5)


def test_headline_when_no_leg_meets_the_budget_or_a_rate_is_given(bench):
    legs = _legs({"0": (34, 1e-6), "4": (290, 1.3e-3), "8": (146, 2e-3), "3:5": (342, 1.5e-3)})
    head, how, met, frate = bench.choose_legs(legs, 0, 1e-3, "full")
    assert (head, met, frate) == ("8", False, 8) and how.startswith("NO candidate")
    head, how, met, frate = bench.choose_legs(legs, 4, 1e-3, "full")
    assert (head, met, frate) == ("4", None, 4) and how == "rate set on the command line"
    # no error reference at all: nothing meets the budget
    legs = _legs({"0": (34, None), "5": (237, None), "3:5": (342, None)})
    head, _, met, frate = bench.choose_legs(legs, 0, 1e-3, "none")
    assert (head, met, frate) == ("5", False, 5)
