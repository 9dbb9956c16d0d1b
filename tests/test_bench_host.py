"""Host-side logic of bench.py (no GPU): the one-GPU rule, the roofline
arithmetic, and the traffic figure's tie to the kernel source it was
measured on."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_roofline_entry_arithmetic():
    b = load_bench()
    nc = 256 * 256 * 128
    cand = dict(kernel="k_cg_iter<fp32>", bound="hbm", avg_ms=0.08, per_step_ms=1.0,
                bytes_alg=60.0 * nc, bytes_fused=44.0 * nc, per_cell=(60.0, 44.0))
    e = b.roofline_entry(cand)
    want = 60.0 * nc / 0.08e-3 / 1e9
    assert abs(e["achieved"] - round(want, 1)) < 0.11
    assert e["peak"] == 8000.0 and e["unit"] == "GB/s"
    assert abs(e["frac"] - want / 8000.0) < 1e-4
    conv = dict(kernel="L4", bound="mfma", avg_ms=0.25, per_step_ms=0.25, flop=3.0e11)
    e = b.roofline_entry(conv)
    assert e["unit"] == "TFLOP/s" and e["peak"] == 2500.0
    assert abs(e["achieved"] - 1200.0) < 0.1 and e["traffic"] is None


def test_traffic_is_reported_only_for_the_measured_source():
    b = load_bench()
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    lines = [l for l in open(path) if "=" in l and not l.startswith("#")]
    assert lines
    name, rest = lines[0].split("=", 1)
    val, src = rest.split("@")
    fname, sha = src.split()
    expect = float(val) if b.source_sha(fname) == sha else None
    assert b.read_traffic(name.strip()) == expect
    assert b.read_traffic("no_such_kernel") is None
