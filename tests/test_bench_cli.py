"""bench.py's command line on the CPU: more than one GPU is refused with a
message, unknown sections are refused, and a traffic summary is reduced from
counter runs (synthetic CSV files of the rocprofv3 layout)."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          cwd=ROOT, timeout=300)


def test_more_than_one_gpu_is_refused():
    r = _bench("--gpus", "2")
    assert r.returncode != 0 and "one GPU only" in r.stderr


def test_unknown_section_is_refused():
    r = _bench("--only", "nonesuch")
    assert r.returncode != 0 and "unknown sections" in (r.stderr + r.stdout)


def _write_counters(d, kernel, counters, dispatches=2):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for disp in range(dispatches):
            for name, value in counters.items():
                # one row per counter and dispatch, summed over instances
                w.writerow([disp, kernel, name, value])


def test_write_traffic_reduces_counter_runs(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    kern = bench.TRAFFIC["small"]["kernel"]
    pmc = str(tmp_path)
    # a 1 GiB copy read back as 2^23 64-byte requests (half its size) and written as 2^24
    _write_counters(os.path.join(pmc, "copy_fetch"), "__amd_rocclr_copyBuffer",
                    {"TCC_EA0_RDREQ_sum": 1 << 23, "TCC_EA0_RDREQ_32B_sum": 0, "TCC_BUBBLE_sum": 0}, 1)
    _write_counters(os.path.join(pmc, "copy_write"), "__amd_rocclr_copyBuffer",
                    {"TCC_EA0_WRREQ_sum": 1 << 24, "TCC_EA0_WRREQ_64B_sum": 1 << 24}, 1)
    _write_counters(os.path.join(pmc, "small_fetch"), f"void lap::{kern}(lap::WilsonParams)",
                    {"TCC_EA0_RDREQ_sum": 1000, "TCC_EA0_RDREQ_32B_sum": 100, "TCC_BUBBLE_sum": 10})
    _write_counters(os.path.join(pmc, "small_write"), f"void lap::{kern}(lap::WilsonParams)",
                    {"TCC_EA0_WRREQ_sum": 300, "TCC_EA0_WRREQ_64B_sum": 200})
    _write_counters(os.path.join(pmc, "small_valu"), f"void lap::{kern}(lap::WilsonParams)",
                    {"SQ_INSTS_VALU": 5000, "SQ_INSTS_VALU_INT64": 1000})
    with open(os.path.join(pmc, "small_fetch", "bench.json"), "w") as f:
        f.write(json.dumps({"small": {"wilson_steps_per_step": 500}}) + "\n")
    out = tmp_path / "summary.json"
    monkeypatch.setitem(bench.TRAFFIC["small"], "file", str(out))
    bench.write_traffic(pmc, "small")
    t = json.loads(out.read_text())
    # fetched: bubbles 128 B, 32-byte requests 32 B, the rest 64 B; calibration 1 GiB / 512 MiB = 2
    fetched = 10 * 128 + (1000 - 10 - 100) * 64 + 100 * 32
    assert t["fetch"]["calibration"] == pytest.approx(2.0)
    assert t["fetch"]["bytes"] == pytest.approx(2.0 * fetched)
    # written: 64-byte requests 64 B, the rest 32 B; calibration 1
    assert t["write"]["calibration"] == pytest.approx(1.0)
    assert t["write"]["bytes"] == pytest.approx(100 * 32 + 200 * 64)
    assert t["read_requests_per_draw"] == pytest.approx(1000 / 500)
    assert t["valu"]["instructions_per_draw"] == pytest.approx(10.0)
    assert t["valu"]["int64_share"] == pytest.approx(0.2)
    assert t["kernel_hash"] == bench.kernel_hash()
