"""Host logic of the benchmark's measurement contract (no GPU): the roofline
figures from a phase profile, the algorithmic FLOP count of the fused loop,
the digest gate on stored counter traffic, and the one-GPU rule."""

import json
import os
import subprocess
import sys

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

PHASES = ("scan", "gram", "coef", "resid", "refine", "norm", "init", "pass", "fused")


def profile(**kw):
    p = {"ms": {k: 0.0 for k in PHASES}, "launches": {k: 0 for k in PHASES},
         "scan_bytes": 0.0, "pass_bytes": 0.0, "fused_bytes": 0.0}
    for k, v in kw.items():
        if k in ("scan_bytes", "pass_bytes", "fused_bytes"):
            p[k] = v
        else:
            phase, what = k.rsplit("_", 1)
            p["ms" if what == "ms" else "launches"][phase] = v
    return p


def test_hbm_roofline_from_pass_phase():
    # 10 pass launches of 1 ms each moving 4 GB apiece: 4000 GB/s, half of 8 TB/s
    r = bench.roofline(profile(pass_ms=10.0, pass_n=10, scan_ms=2.0, scan_n=10,
                               pass_bytes=10 * 4e9))
    assert r["bound"] == "hbm" and r["kernel"].startswith("coef_pass_kernel")
    assert r["achieved"] == pytest.approx(4000.0) and r["frac"] == pytest.approx(0.5)
    assert r["avg_launch_us"] == pytest.approx(1000.0) and r["bytes_per_launch"] == 4e9


def test_hbm_roofline_falls_back_to_scan():
    r = bench.roofline(profile(scan_ms=6.0, scan_n=3, scan_bytes=3 * 2e9), method="iht")
    assert r["kernel"].startswith("iht_grad_kernel")
    assert r["achieved"] == pytest.approx(1000.0)


def brute_fused_flops(n, m, k, method, T=32):
    tot = 0.0
    for t in range(min(k, m, n)):
        t1 = t + 1
        tot += 2 * m * n            # scan
        tot += 2 * m * (t + 2)      # Gram column and b
        tot += 2 * m * t1           # residual
        tot += T * (2 * t1 * t1 + 10 * t1) if method == "clomp" else 6 * t * t
    return tot


@pytest.mark.parametrize("method", ["clomp", "omp"])
def test_fused_flops_count(method):
    items = [dict(At=torch.zeros((256, 64)), m=64, k=8), dict(At=torch.zeros((100, 20)), m=20, k=30)]
    want = brute_fused_flops(256, 64, 8, method) + brute_fused_flops(100, 20, 30, method)
    assert bench.fused_flops(items, method) == pytest.approx(want)


def test_fused_roofline_is_alu_bound():
    items = [dict(At=torch.zeros((256, 64)), m=64, k=8)] * 4
    p = profile(fused_ms=2.0, fused_n=1, refine_ms=0.1, refine_n=1, fused_bytes=1e6)
    r = bench.roofline(p, items, "clomp")
    fl = bench.fused_flops(items, "clomp")
    assert r["bound"] == "alu" and r["peak"] == bench.VALU_PEAK_TFLOPS
    assert r["achieved"] == pytest.approx(fl / 2e-3 / 1e12)
    assert r["flops_per_launch"] == fl


@pytest.mark.parametrize("bf16", [False, True])
def test_shared_dictionary_roofline_is_mfma(bf16):
    A = torch.zeros((2160, 648), dtype=torch.bfloat16 if bf16 else torch.float32)
    items = [dict(At=A, m=648, k=108)] * 3840
    p = profile(scan_ms=10.0, scan_n=100, coef_ms=5.0, coef_n=100)
    r = bench.roofline(p, items, "clomp")
    fl = 2.0 * 2160 * 648 * 3840
    assert r["bound"] == "mfma" and r["flops_per_launch"] == fl
    peak = bench.MFMA_BF16_PEAK_TFLOPS if bf16 else bench.MFMA_FP32_PEAK_TFLOPS
    assert r["peak"] == peak
    assert r["achieved"] == pytest.approx(fl / 0.1e-3 / 1e12)


def test_stored_traffic_only_for_the_measured_code(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "hbm_traffic_demo.json").write_text(
        json.dumps({"traffic_bytes_per_launch": 123.0, "kernel_digest": "abc"}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_digest", lambda: "abc")
    assert bench.measured_traffic("demo", "coef_pass_kernel (x)") == 123.0
    assert bench.measured_traffic("demo", "cscan/ypass kernels") is None
    assert bench.measured_traffic("other", "coef_pass_kernel (x)") is None
    monkeypatch.setattr(bench, "kernel_digest", lambda: "changed")
    assert bench.measured_traffic("demo", "coef_pass_kernel (x)") is None


def test_kernel_digest_covers_the_pass_code():
    d = bench.kernel_digest()
    assert len(d) == 16 and d == bench.kernel_digest()


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
