"""Host logic of bench.py: the HBM-traffic summary built from rocprofv3
counter files and its lookup by kernel-source hash and launch configuration."""
import csv
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture()
def bench(tmp_path, monkeypatch):
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    monkeypatch.setattr(mod, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    return mod


FIELDS = ["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"]


def write_run(d, counter, march_kib, copy_kib, small_copy_kib=1.5):
    os.makedirs(d)
    rows = [dict(Dispatch_Id=1, Grid_Size=512, Kernel_Name="__amd_rocclr_copyBuffer",
                 Counter_Name=counter, Counter_Value=small_copy_kib)]
    rows += [dict(Dispatch_Id=2 + i, Grid_Size=8192, Kernel_Name="void lbm::lbm_march_kernel<float>()",
                  Counter_Name=counter, Counter_Value=v) for i, v in enumerate(march_kib)]
    rows += [dict(Dispatch_Id=20 + i, Grid_Size=131072, Kernel_Name="__amd_rocclr_copyBuffer",
                  Counter_Name=counter, Counter_Value=copy_kib) for i in range(3)]
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        w.writerows(rows)


def test_traffic_summary_scales_by_the_calibration_copy(bench, tmp_path):
    pmc = tmp_path / "pmc"
    # a 1024 MiB copy reads 1,048,576 KiB: FETCH_SIZE reading half of it gets a scale of 2
    write_run(str(pmc / "pmc_vaporisation512_fp32_5x2_FETCH_SIZE"), "FETCH_SIZE", [100.0, 300.0],
              524288.0)
    write_run(str(pmc / "pmc_vaporisation512_fp32_5x2_WRITE_SIZE"), "WRITE_SIZE", [50.0, 50.0],
              1048576.0)
    out = bench.write_traffic(str(pmc), 1024)
    d = out["detail"]["vaporisation512_fp32"]["5x2"]
    assert d["fetch_scale"] == 2.0 and d["write_scale"] == 1.0 and d["dispatches"] == 2
    assert d["read_bytes"] == 2 * 200 * 1024 and d["write_bytes"] == 50 * 1024
    assert d["algorithmic_bytes"] == 80 * 512 * 512
    assert out["per_launch_bytes"]["vaporisation512_fp32"]["5x2"] == 450 * 1024
    # lookup: right configuration only, and only while the kernel sources hash to the stored value
    assert bench.measured_traffic("vaporisation512_fp32", 5, 2) == 450 * 1024
    assert bench.measured_traffic("vaporisation512_fp32", 5, 1) is None
    assert bench.measured_traffic("pool4096_fp32", 128, 1) is None


def test_traffic_lookup_rejects_a_changed_kernel_source(bench, tmp_path):
    pmc = tmp_path / "pmc"
    write_run(str(pmc / "pmc_pool4096_fp64_64x1_FETCH_SIZE"), "FETCH_SIZE", [10.0], 524288.0)
    write_run(str(pmc / "pmc_pool4096_fp64_64x1_WRITE_SIZE"), "WRITE_SIZE", [10.0], 1048576.0)
    bench.write_traffic(str(pmc), 1024)
    assert bench.measured_traffic("pool4096_fp64", 64, 1) == 30 * 1024
    import json

    t = json.load(open(bench.TRAFFIC_FILE))
    t["kernel_sha256"] = "0" * 64
    json.dump(t, open(bench.TRAFFIC_FILE, "w"))
    assert bench.measured_traffic("pool4096_fp64", 64, 1) is None

