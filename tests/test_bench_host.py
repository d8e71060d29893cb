"""Host-side logic of bench.py (no GPU): the traffic summary of two counter
runs, the code hash the calibration is keyed to, and the refusal of more
than one GPU."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _counter_dir(tmp_path, name, counter, rows):
    d = tmp_path / name
    d.mkdir()
    with open(d / "run_counter_collection.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for i, (kernel, kib) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": kernel, "Counter_Name": counter, "Counter_Value": kib})
    return str(d)


COPY = "k_copy(float __vector(4)*, float __vector(4) const*, long long)"
EVEN = "void k_step<false, mclbm::StorF32<false, false>, unsigned int, 3>(mclbm::StepParams)"
ODD = "void k_step<true, mclbm::StorF32<false, false>, unsigned int, 3>(mclbm::StepParams)"
PAIR = "void k_step2<mclbm::StorF32<false, false> >(mclbm::StepParams)"


def test_traffic_summary_scales_by_the_copy_kernel(tmp_path):
    """FETCH_SIZE counts half the bytes of the 1 GiB copy and WRITE_SIZE all
    of them: the summary scales each counter so that the copy reads 1 GiB
    each way, and averages the two parities."""
    gib_kib = 1 << 20
    fetch = _counter_dir(tmp_path, "f", "FETCH_SIZE",
                         [(COPY, gib_kib / 2), (COPY, gib_kib / 2), (EVEN, 1000.0), (ODD, 1100.0), (EVEN, 1000.0)])
    write = _counter_dir(tmp_path, "w", "WRITE_SIZE", [(COPY, gib_kib), (EVEN, 2000.0), (ODD, 2100.0)])
    out = tmp_path / "t.json"
    bench.pmc_summary(fetch, write, "cavity512_ra1e5", str(out))
    t = json.load(open(out))
    assert t["steps_per_launch"] == 1 and t["storage"] == "fp32"
    assert t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    assert t["fetch_bytes"]["step_even"] == pytest.approx(2000.0 * 1024)
    assert t["fetch_bytes"]["step_odd"] == pytest.approx(2200.0 * 1024)
    assert t["write_bytes"]["step_odd"] == pytest.approx(2100.0 * 1024)
    assert t["bytes_per_launch"] == pytest.approx(0.5 * (2000 + 2000 + 2200 + 2100) * 1024)
    assert t["kernel_hash"] == bench.kernel_hash()


def test_traffic_summary_of_two_steps_per_launch(tmp_path):
    fetch = _counter_dir(tmp_path, "f", "FETCH_SIZE", [(COPY, 512.0), (PAIR, 300.0), (PAIR, 310.0)])
    write = _counter_dir(tmp_path, "w", "WRITE_SIZE", [(COPY, 1024.0), (PAIR, 200.0)])
    out = tmp_path / "t.json"
    bench.pmc_summary(fetch, write, "cavity4096_ra1e6", str(out))
    t = json.load(open(out))
    assert t["steps_per_launch"] == 2 and list(t["fetch_bytes"]) == ["step_pair"]
    scale_f, scale_w = (1 << 20) / 512.0, (1 << 20) / 1024.0
    assert t["bytes_per_launch"] == pytest.approx((305.0 * scale_f + 200.0 * scale_w) * 1024)


def test_code_hash_ignores_comments_and_blank_lines():
    a = "int f(int x) {\n  // the square\n  return x * x;  // fast\n}\n"
    b = "int f(int x) {\n\n  return x * x;\n}\n// end\n"
    c = "int f(int x) {\n  return x * x + 1;\n}\n"
    assert bench.code_text(a) == bench.code_text(b)
    assert bench.code_text(a) != bench.code_text(c)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr


def test_stored_headline_traffic_belongs_to_the_current_kernels():
    """The bench reports the HBM bytes of its headline launch from the
    stored counter summary only while the step kernels' source is the one
    the counters were taken with; a kernel change needs new counter runs."""
    import json
    t = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert t["workload"] == "cavity512_ra1e5" and t["storage"] == "fp32"
    assert t["kernel_hash"] == bench.kernel_hash()
