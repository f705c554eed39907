"""CPU checks of bench.py's contract: the roofline object's arithmetic on
synthetic per-pair records, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _pair(launch, dwords, executed, dev_ms, ms=None):
    return {"launch": launch, "dwords": dwords, "executed": executed, "dev_ms": dev_ms,
            "ms": dev_ms if ms is None else ms}


def test_roofline_groups_launches_and_prices_against_the_peak():
    # two runs; launch 0 holds two short pairs (their span is the longer
    # one), launch 1 one long pair; all D = 3
    run = {"pairs": [_pair(0, 3, 1000, 0.010), _pair(0, 3, 3000, 0.020), _pair(1, 3, 6_000_000_000, 1.0)]}
    nominal = 256 * 64 * 2.4e9 / 2
    D, roof = bench.roofline([run, run], [run], nominal, mfma=False)
    assert D == 3
    sec = 2 * (0.020 + 1.0) * 1e-3
    cw = 2 * (1000 + 3000 + 6_000_000_000)
    assert roof["launches"] == 4
    assert roof["achieved"] == pytest.approx(cw * 3 / sec / 1e12)
    assert roof["peak"] == pytest.approx(nominal / 1e12)
    assert roof["frac"] == pytest.approx(cw * 3 / sec / nominal)
    # a measured ceiling above the derived figure becomes the denominator;
    # the nominal share stays beside it
    _, roof2 = bench.roofline([run, run], [run], 1.1 * nominal, mfma=False)
    assert roof2["peak"] == pytest.approx(1.1 * nominal / 1e12)
    assert roof2["frac"] == pytest.approx(roof["frac"] / 1.1)
    assert roof2["frac_nominal"] == pytest.approx(roof["frac"])
    assert roof2["peak_nominal"] == pytest.approx(nominal / 1e12)
    assert roof["bound"] == "alu"
    assert roof["avg_launch_us"] == pytest.approx(sec / 4 * 1e6)
    for key in ("unit", "traffic", "kernel", "avg_launch_us_events"):
        assert key in roof


def test_matrix_core_roofline_prices_int8_products():
    # the default inner loop at D <= 4: a 32 x 32 x 32 int8 product per word,
    # 64 D ops per codeword against the int8 peak; XOR+popcount figures beside
    run = {"pairs": [_pair(0, 3, 6_000_000_000, 1.0)]}
    valu = 21.58e12
    D, roof = bench.roofline([run], [run], valu)
    sec, cw = 1.0e-3, 6_000_000_000
    assert D == 3 and roof["bound"] == "mfma"
    assert roof["achieved"] == pytest.approx(cw * 192 / sec / 1e12)
    assert roof["peak"] == pytest.approx(5000.0)
    assert roof["frac"] == pytest.approx(cw * 192 / sec / 5.0e15)
    assert roof["xorpop_equiv_over_valu_peak"] == pytest.approx(cw * 3 / sec / valu)
    assert roof["kernel"].endswith("true>")
    # 5 words and more stay on the vector ALUs
    run7 = {"pairs": [_pair(0, 7, 10**9, 1.0)]}
    D7, roof7 = bench.roofline([run7], [run7], valu)
    assert D7 == 7 and roof7["bound"] == "alu" and roof7["kernel"].endswith("false>")


def test_dominant_kernel_is_the_instance_with_the_most_time():
    run = {"pairs": [_pair(0, 2, 10**9, 0.5), _pair(1, 3, 10**9, 2.0), _pair(2, 2, 10**9, 0.5)]}
    D, roof = bench.roofline([run], [run], 256 * 64 * 2.4e9 / 2)
    assert D == 3 and roof["launches"] == 1


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
