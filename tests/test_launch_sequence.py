"""The library's host code (plan builder, schedules, launch sequence) run on
the CPU against launch checks instead of kernels (tests/launch_harness): every
launch's instance and tile ranges, LDS needs, team sizes and workspace
buffers, and the per-signal order of scan, coefficient update and pass, for
the batch shapes of the workloads and the schedule switches.  Needs hipcc
(cross-compiles the host code; no GPU)."""

import os
import re
import shutil
import subprocess

import pytest

from paper_2501_11592_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2501_11592_amd", "csrc")
HARNESS = os.path.join(ROOT, "tests", "launch_harness")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

CLOMP, OMP, IHT, PAPER = 0, 1, 2, 3
F_GRAPH, F_NO_FUSED, F_RESID, F_CORR, F_NO_SHARED, F_NO_REFINE, F_IMAGE = 1, 2, 16, 32, 64, 128, 256


@pytest.fixture(scope="session")
def driver(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("launch_harness")
    flags = ["-O1", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
             "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
             "-x", "hip"]
    objs = []
    for src in (os.path.join(CSRC, "runtime.cpp"), os.path.join(HARNESS, "mock_launchers.cpp"),
                os.path.join(HARNESS, "mock_hip.cpp"), os.path.join(HARNESS, "driver.cpp")):
        obj = str(out / (os.path.basename(src) + ".o"))
        r = subprocess.run([HIPCC, *flags, "-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        objs.append(obj)
    exe = str(out / "driver")
    r = subprocess.run([HIPCC, "-o", exe, *objs], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe, out


def run(driver, specs, method, flags=0, bf16=1, shared=0, tmr=0, prior_tv=0.0, prior_lv=0.0):
    exe, out = driver
    f = out / f"specs_{abs(hash(tuple(specs)))}.txt"
    if not f.exists():
        f.write_text("".join(f"{n} {m} {k}\n" for n, m, k in specs))
    r = subprocess.run([exe, str(f), str(method), str(flags), str(bf16), str(shared), str(tmr),
                        str(prior_tv), str(prior_lv)], capture_output=True, text=True, timeout=600)
    counts = {m.group(1): int(m.group(2))
              for m in re.finditer(r"^\s+(\w+)\s+(\d+)$", r.stdout, re.M)}
    return r.returncode, r.stdout, counts


def uneven(count=4096):
    return [(s.n, s.m, s.k) for s in W.uneven_specs(count)]


def ok(rc, text):
    assert rc == 0 and "violations 0" in text, text[-4000:]


@pytest.mark.parametrize("method", [CLOMP, OMP])
def test_uneven_batch(driver, method):
    """The default workload: 4096 signals, BF16 bulk with an FP32 master, the
    correlation-update schedule with lane-width classes, splits, teams and the
    fused small-signal loop."""
    specs = uneven()
    rc, text, n = run(driver, specs, method)
    ok(rc, text)
    # one pass launch per class and iteration, one H scan per class and
    # iteration except each class's last; one first pass (A^T y) per class
    assert n["coef_pass"] > 0 and n["init"] == 1
    assert n["coef_pass"] - n["cscan"] == n["ypass"], n


@pytest.mark.parametrize("method", [CLOMP, OMP])
@pytest.mark.parametrize("tmr", [16, 64])
def test_uneven_batch_with_teams(driver, method, tmr):
    """Coefficient teams from 16 or 64 atoms on: their sizes, LDS and the
    rule that all members of a launch fit on the device at once."""
    rc, text, n = run(driver, uneven(1024), method, tmr=tmr)
    ok(rc, text)


@pytest.mark.parametrize("method", [CLOMP, OMP])
@pytest.mark.parametrize("flags", [F_RESID, F_CORR | F_NO_FUSED, F_GRAPH, F_NO_REFINE])
def test_schedule_switches(driver, method, flags):
    rc, text, n = run(driver, uneven(512), method, flags=flags)
    ok(rc, text)


@pytest.mark.parametrize("method", [CLOMP, OMP])
def test_fp32_bulk(driver, method):
    rc, text, n = run(driver, uneven(512), method, bf16=0)
    ok(rc, text)


@pytest.mark.parametrize("method", [CLOMP, OMP, IHT, PAPER])
@pytest.mark.parametrize("flags", [0, F_NO_FUSED, F_NO_SHARED | F_NO_FUSED])
def test_shared_dictionary_image(driver, method, flags):
    """256 columns of a 256 x 256 image sharing A (m = 77, k = 32): the fused
    loop, the shared-dictionary schedule and per-signal scans."""
    rc, text, n = run(driver, [(256, 77, 32)] * 256, method, flags=flags, bf16=0, shared=1)
    ok(rc, text)


@pytest.mark.parametrize("method", [CLOMP, OMP])
def test_image4k_columns(driver, method):
    """A 4K-scale shared-dictionary batch (n = 2160, m = 648, k = 108) with a
    BF16 bulk copy: the matrix-core scan and support-sized coefficient
    workgroups."""
    rc, text, n = run(driver, [(2160, 648, 108)] * 384, method, shared=1)
    ok(rc, text)
    assert n.get("shared_rscan", 0) > 0


@pytest.mark.parametrize("method", [IHT, PAPER])
def test_iterative_methods_uneven(driver, method):
    rc, text, n = run(driver, uneven(256), method)
    ok(rc, text)


@pytest.mark.parametrize("method", [CLOMP, OMP])
def test_flat_signal(driver, method):
    """The flattened image as one signal (n = 65536, m = 19661, k = 2048):
    supports beyond the register tile and the split rows."""
    rc, text, n = run(driver, [(65536, 19661, 2048)], method)
    ok(rc, text)


@pytest.mark.parametrize("lv", [0.0, 0.5])
def test_image_mode(driver, lv):
    """CLOMP_FLAG_IMAGE: one Adam launch per step (two with the local
    variation) over all columns, k * T steps."""
    rc, text, n = run(driver, [(256, 77, 32)] * 256, CLOMP, flags=F_IMAGE, bf16=0, shared=1,
                      prior_tv=0.01, prior_lv=lv)
    ok(rc, text)
    assert n["image_step"] == 32 * 32
    assert n.get("image_synth", 0) == (32 * 32 if lv else 0)


def test_image_mode_refuses_distinct_dictionaries(driver):
    rc, text, n = run(driver, [(256, 77, 32)] * 8, CLOMP, flags=F_IMAGE, bf16=0, shared=0,
                      prior_tv=0.01)
    assert rc == 4 and "CLOMP_NOT_SUPPORTED" in text, text
