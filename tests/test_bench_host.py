"""Host logic of bench.py (CPU): the per-class roofline arithmetic, the traffic summary it reads
and its source-digest guard, and the one-GPU contract."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _cls(ms, timed_flops, launches=10, timed=10, flops=None):
    return {"ms": ms, "timed_flops": timed_flops, "timed_launches": timed, "launches": launches,
            "flops": timed_flops if flops is None else flops}


def test_class_rooflines_shares_rates_and_peaks():
    cls = {"sweep": _cls(60.0, 3.0e12), "lu_update": _cls(30.0, 0.6e12), "panel": _cls(10.0, 0.0),
           "fused": _cls(0.0, 0.0, launches=0, timed=0)}
    out = bench.class_rooflines(cls, "fp64")
    assert set(out) == {"sweep", "lu_update", "panel"}  # a class with no launches is left out
    assert abs(sum(c["share_of_kernel_time"] for c in out.values()) - 1.0) < 1e-12
    assert abs(out["sweep"]["achieved_tflops"] - 3.0e12 / 0.060 / 1e12) < 1e-9
    assert abs(out["sweep"]["frac"] - out["sweep"]["achieved_tflops"] / 78.6) < 1e-12
    assert out["panel"]["achieved_tflops"] is None and out["panel"]["frac"] is None
    assert out["lu_update"]["avg_launch_ms"] == 3.0


def test_class_rooflines_mixed_uses_the_fp32_peak_for_fp32_parts():
    cls = {"sweep": _cls(10.0, 1e12), "solve": _cls(10.0, 1e12), "lead": _cls(10.0, 1e12)}
    out = bench.class_rooflines(cls, "mixed", mixed_parts=1)  # only the sweep products in FP32
    assert out["sweep"]["peak_tflops"] == 157.3
    assert out["solve"]["peak_tflops"] == 78.6 and out["lead"]["peak_tflops"] == 78.6
    out = bench.class_rooflines(cls, "mixed", mixed_parts=7)
    assert out["solve"]["peak_tflops"] == 157.3 and out["lead"]["peak_tflops"] == 78.6


def test_decimation_class_reports_executed_flops_but_no_rate():
    """A decimation launch counts every energy of its batch while converged energies skip it, so
    the class keeps its (corrected) flop total for the whole-step count but reports no rate."""
    cls = {"sweep": _cls(10.0, 1e12), "lead": _cls(10.0, 2e12, flops=5e12)}
    out = bench.class_rooflines(cls, "fp64")
    assert out["lead"]["achieved_tflops"] is None and out["lead"]["frac"] is None
    assert out["lead"]["flops"] == 5e12 and "flops_note" in out["lead"]
    assert out["sweep"]["frac"] is not None


def test_measured_traffic_reads_the_summary_and_checks_the_digest(monkeypatch):
    kv = {}
    with open(bench.TRAFFIC_SUMMARY) as f:
        for line in f:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                kv[k.strip()] = v.strip().strip("`")
    expect = ((float(kv["sweep product FETCH_SIZE KiB/launch"]) * float(kv["FETCH_SIZE scale"])
               + float(kv["sweep product WRITE_SIZE KiB/launch"]) * float(kv["WRITE_SIZE scale"]))
              * 1024 / float(kv["energies per launch"]))
    monkeypatch.setattr(bench, "source_digest", lambda: kv["gemm.hip + engine.hip sha256 prefix"])
    assert abs(bench.measured_traffic() - expect) < 1e-6 * expect
    monkeypatch.setattr(bench, "source_digest", lambda: "0000000000000000")
    assert bench.measured_traffic() is None  # counters taken on another source are not reported


def test_source_digest_is_a_16_hex_prefix():
    d = bench.source_digest()
    assert len(d) == 16 and int(d, 16) >= 0 and d == bench.source_digest()


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
