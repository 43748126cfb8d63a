"""Host logic of bench.py's profiler ingestion (CPU): kernel-name
normalisation of the forms rocprofv3 prints, and the HBM traffic record
built from FETCH_SIZE / WRITE_SIZE counter files (calibration from the run's
first device copies, records keyed as the bench looks kernels up)."""

import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture()
def bench(monkeypatch, tmp_path):
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import bench as b
    monkeypatch.setattr(b, "traffic_path", lambda wl: str(tmp_path / f"traffic_{wl}.json"))
    return b


def test_profiler_names_of_bf16_templates(bench):
    n = bench.profiler_kernel_name
    # left mangled by the profiler
    assert n("_ZN2kp9mp_kernelILi2EDF16bDF16bLi8ELi2ELi1ELb1EEEvPKDv4_jiiPKT0_PT1_iilPKNS_8Rhs") == \
        "kp::mp_kernel<2, __bf16, __bf16, 8, 2, 1, true>"
    assert n("_ZN2kp9mp_kernelILi2EdDF16bLi16ELi1ELi1ELb1EEEvPKDv4_jiiPKT0_PT1_iilPKNS_8RhsSta") == \
        "kp::mp_kernel<2, double, __bf16, 16, 1, 1, true>"
    assert n("_ZN2kp6mp_resILi2EDF16bDF16bLi8ELi1EEEvPKDv4_jiPKT0_PT1_iilPKNS_8RhsStateEii") == \
        "kp::mp_res<2, __bf16, __bf16, 8, 1>"
    # the (__bf16, double) pair demangled as 'bool _Accum'
    assert n("void kp::mp_kernel<2, bool _Accum, 8, 4, 2, true>") == \
        "kp::mp_kernel<2, __bf16, double, 8, 4, 2, true>"
    # everything else passes through
    assert n("void kp::mp_ozh<4, 1, 7>") == "kp::mp_ozh<4, 1, 7>"
    assert n("kp::k_zm<1>") == "kp::k_zm<1>"


def _counter_file(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (name, grid, v) in enumerate(rows, start=1):
            w.writerow([i, grid, name, counter, v])


def test_traffic_record_calibration_and_keys(bench, tmp_path):
    cal = bench.COPY_CAL_BYTES // 1024                # KiB
    big = 4 * cal                                     # a later, larger copy of the workload's data
    prod = "void kp::mp_ozh<4, 1, 7>(unsigned int __vector(4) const*, int const*)"
    vec = "void kp::k_zm<1>(kp::Geom, kp::ZGrid)"
    copy = "__amd_rocclr_copyBuffer"
    fetch = [(copy, 131072, cal / 2)] * bench.COPY_CAL_RUNS + [(copy, 131072, big / 2),
                                                               (prod, 2097152, 1000.0),
                                                               (prod, 2097152, 1200.0),
                                                               (vec, 524288, 300.0)]
    write = [(copy, 131072, cal)] * bench.COPY_CAL_RUNS + [(copy, 131072, big),
                                                           (prod, 2097152, 500.0),
                                                           (prod, 2097152, 500.0),
                                                           (vec, 524288, 200.0)]
    _counter_file(str(tmp_path / "f"), "FETCH_SIZE", fetch)
    _counter_file(str(tmp_path / "w"), "WRITE_SIZE", write)
    rec = bench.ingest_traffic("large512", str(tmp_path / "f"), str(tmp_path / "w"), "cmd")
    # the calibration is the first copies', not the larger later one's
    assert rec["copy_fetch_kib"] == cal / 2 and rec["copy_write_kib"] == cal
    assert json.load(open(bench.traffic_path("large512")))["command"] == "cmd"
    # read factor 2, write factor 1, bytes per launch averaged over dispatches
    got = bench.measured_traffic("large512", "kp::mp_ozh<4, 1, 7>|2097152")
    assert got == pytest.approx(1100.0 * 1024 * 2 + 500.0 * 1024)
    assert bench.measured_traffic("large512", "kp::k_zm<1>") == pytest.approx(
        300.0 * 1024 * 2 + 200.0 * 1024)
    assert bench.measured_traffic("large512", "kp::mp_ozh<4, 1, 7>|1048576") is None
