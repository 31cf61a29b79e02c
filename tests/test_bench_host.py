"""Host-side logic of bench.py (no GPU): the one-GPU guard, the roofline
arithmetic of a launch kind, and the traffic record lookup."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"] and line["n_gpus"] == 2


def test_kernel_roofline_bounds():
    rec = {"ms": 2.0, "bytes": 8e9, "flops": 157.3e9, "launches": 1}
    mf = bench.kernel_roofline("gemm_out", rec, "f32")
    assert mf["bound"] == "mfma" and abs(mf["achieved"] - 78.65) < 1e-9 and abs(mf["frac"] - 0.5) < 1e-12
    # the line-search products are float64 whatever the context precision
    f64 = bench.kernel_roofline("ls_gemm_out", rec, "f32")
    assert f64["peak"] == 78.6
    # BF16 contexts keep the adjoint product in float32
    assert bench.kernel_roofline("gemm_adjoint", rec, "bf16")["peak"] == 157.3
    # BF16 decoder products: six BF16 MFMAs per float32-accurate product
    assert abs(bench.kernel_roofline("gemm_out", rec, "bf16")["peak"] - 2500.0 / 6) < 1e-9
    hb = bench.kernel_roofline("elem", rec, "f32")
    assert hb["bound"] == "hbm" and abs(hb["achieved"] - 4000.0) < 1e-9 and abs(hb["frac"] - 0.5) < 1e-12
    assert bench.kernel_roofline("newton_dir", rec, "f32")["bound"] == "alu"
    assert bench.kernel_roofline("param_grad", rec, "f32")["bound"] == "alu"


def test_traffic_record_needs_the_current_kernel_source(monkeypatch):
    # a record for another workload or another source hash is not used
    assert bench.recorded_traffic("gemm_out", "no_such_workload") is None
    monkeypatch.setattr(bench, "KERNEL_SOURCE", os.path.join(ROOT, "bench.py"))
    assert bench.recorded_traffic("gemm_out", "c2_b1024") is None
