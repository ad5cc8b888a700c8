"""Host logic of bench.py, without a GPU: the single-GPU guard, the issue-slot
roofline model, the time-to-1bp path count and the bounded oracle samples
that stand beside every bench line."""
import json
import math
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import synth  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_alu_peak_is_the_chip_issue_rate():
    # 256 CUs x 2.4 GHz x 128 FMA lanes per clock.
    assert bench.ALU_PEAK_SLOTS == pytest.approx(256 * 2.4e9 * 128)
    assert bench.HBM_PEAK == 8.0e12


def test_slot_costs_of_a_normal():
    # An FP32 normal (path-per-lane kernels): 4.25 products, 5 three-input
    # xors, half a log and one and a half other transcendentals, 2.5 FP32
    # operations and one integer operation.
    want = (4.25 * bench.COST_MUL64 + 5 * bench.COST_BITOP3 + 0.5 * bench.COST_LOG
            + 1.5 * bench.COST_TRANS + 2.5 * bench.COST_FP32 + 1.0 * bench.COST_INT)
    assert bench.slots(**bench.NORMAL) == pytest.approx(want)
    assert 30.0 < want < 33.0
    # The basket's lanes draw two block indices per step: all 20 products count.
    assert bench.slots(**bench.NORMAL_BASKET) > bench.slots(**bench.NORMAL)
    assert bench.SLOTS_ASIAN_BARRIER == pytest.approx(
        want + bench.COST_TRANS + bench.COST_INT + 4 * bench.COST_FP32)


def test_alu_roofline_fraction():
    r = bench._alu_roofline(40.0, 1e9, 1.0, "k")
    assert r["bound"] == "alu" and r["peak"] == pytest.approx(bench.ALU_PEAK_SLOTS / 1e12)
    assert r["frac"] == pytest.approx(40.0 * 1e9 / 1e-3 / bench.ALU_PEAK_SLOTS)
    assert r["achieved"] == pytest.approx(r["frac"] * r["peak"])


@pytest.mark.parametrize("se,sigma", [(1e-3, 14.7), (5e-4, 5.8), (1.0, 0.5)])
def test_paths_for_one_bp(se, sigma):
    n = bench._paths_for(se, sigma)
    assert n % 256 == 0 and n >= 256
    assert n >= (sigma / se) ** 2 and n - (sigma / se) ** 2 < 256 + 1


def test_oracle_sample_is_bounded_and_a_power_of_two():
    calls = []

    def fn(k):
        calls.append(k)
    n, dt = bench._oracle_sample(fn, 1 << 4, 1 << 10, budget_s=1e-3)
    assert calls[0] == 1 << 4 and calls[-1] == n
    assert 1 << 4 <= n <= 1 << 10 and n & (n - 1) == 0 and dt >= 0.0


def test_cpu_baselines_state_what_they_measured():
    e = bench._cpu_european({}, synth)
    q = bench._cpu_qmc_basket({"config": {"n_points": 1 << 10, "replicates": 2}}, synth)
    for line, unit in ((e, "path-steps/s"), (q, "paths/s")):
        assert line["kind"] == "oracle" and line["unit"] == unit
        assert line["value"] > 0 and line["cores"] >= 1 and line["sample"]
        assert math.isfinite(line["value"])


def test_black_scholes_check_of_the_european_line():
    # Black-Scholes call S0 = K = 100, r = 0.05, sigma = 0.2, T = 1.
    r = {"price": 10.45, "std_err": 0.03, "delta": 0.637, "delta_se": 0.001, "vega": 37.5,
         "vega_se": 0.1}
    b = bench._bs_check(synth.EURO, r)
    assert b["price"] == pytest.approx(10.450583572185565, rel=1e-13)
    assert b["delta"] == pytest.approx(0.6368306511756191, rel=1e-13)
    assert b["vega"] == pytest.approx(37.52403469169379, rel=1e-13)
    assert b["price_z"] == pytest.approx((10.45 - b["price"]) / 0.03)


def test_geometric_asian_closed_form_of_the_default_line():
    # bench.py's own closed form against the tests' (written separately).
    from closed_forms import geo_asian_call
    c = synth.ASIAN_BARRIER
    for n in (1, 12, 252):
        want = geo_asian_call(c["S0"], c["K"], c["r"], c["sigma"], c["T"], n)
        assert bench._geo_asian_closed_form(c, n) == pytest.approx(want, rel=1e-12)
    # n = 1 is the European call on S_T.
    e = dict(c)
    b = bench._bs_check(e, {"price": 0.0, "std_err": 1.0, "delta": 0.0, "delta_se": 1.0,
                            "vega": 0.0, "vega_se": 1.0})
    assert bench._geo_asian_closed_form(c, 1) == pytest.approx(b["price"], rel=1e-12)
