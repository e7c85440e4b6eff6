"""bench.py's contract on the host: one GPU only, and a cost model that
agrees with the counter figures committed beside it."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_flops_per_element_match_the_committed_counters():
    b = load_bench()
    t = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))["kernels"]
    e64 = t["k_ns_jvp_lin<double,double>"]["rt_l10"]
    e32 = t["k_ns_jvp_lin<float,float>"]["rt_l10"]
    assert round(e64["f64_flops_per_launch"] / e64["leaves"]) == b.NS_JVP_FLOPS_PER_ELEMENT["fp64"]
    assert round(e32["f32_flops_per_launch"] / e32["leaves"]) == b.NS_JVP_FLOPS_PER_ELEMENT["mixed"]
    lin = t["k_ns_lin<double,double>"]["bubble_l9"]
    mid = t["k_ns_mid<double,double>"]["bubble_l9"]
    per_elem = (lin["f64_flops_per_launch"] + mid["f64_flops_per_launch"]) / lin["leaves"]
    assert abs(per_elem - b.ELEMENT_KERNELS["ns_lin_f64"][0]) <= 1


def test_kernel_roofline_arithmetic():
    b = load_bench()
    n, E = 1000, 1200
    kern = {"ns_jvp_lin_f64_ms": 0.5, "ch_residual_ms": 0.25, "ignored_ms": 1.0}
    out = b.kernel_roofline(kern, n, E)
    assert set(out) == {"ns_jvp_lin_f64", "ch_residual"}
    flops, bpn, bpe, peak = b.ELEMENT_KERNELS["ns_jvp_lin_f64"]
    gbs = (n * bpn + E * bpe) / 0.5e-3 / 1e9
    assert abs(out["ns_jvp_lin_f64"]["GBps"] - round(gbs, 1)) < 1e-9
    assert abs(out["ns_jvp_lin_f64"]["hbm_frac"] - round(gbs / b.PEAK_HBM_GBS, 4)) < 1e-12
    tf = flops * E / 0.5e-3 / 1e12
    assert abs(out["ns_jvp_lin_f64"]["alu_frac"] - round(tf / b.PEAK_TFLOPS[peak], 4)) < 1e-12
    for key, (fl, bn, be, pk) in b.ELEMENT_KERNELS.items():
        assert fl > 0 and bn > 0 and be > 0 and pk in b.PEAK_TFLOPS, key
