"""The benchmark's profile post-processing (CPU): the kernel-trace summary
split by launch grid, and the HBM traffic record built from two counter
passes scaled by a plain copy's reading."""
import csv
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402

STEP = ("void cdbm::(anonymous namespace)::k_step_fused<float, true>"
        "(float const*, float*, cdbm::KParams const*, int, int)")
TORCH = ("void at::native::elementwise_kernel_manual_unroll<128, 4, at::native::gpu_kernel_impl"
         "<at::native::CUDAFunctor_add<double> >(at::TensorIteratorBase&)::{lambda(int, bool)#1}>"
         "(int, at::native::gpu_kernel_impl<at::native::CUDAFunctor_add<double> >)")


def _write_csv(path, fields, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_short_kernel_name():
    assert bench.short_kernel_name(STEP) == "k_step_fused<float, true>"
    assert bench.short_kernel_name(TORCH) == "at::native::elementwise_kernel_manual_unroll"
    assert bench.short_kernel_name("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_trace_summary_splits_by_launch_grid(tmp_path, capsys):
    fields = ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Workgroup_Size_X",
              "Workgroup_Size_Y", "Workgroup_Size_Z", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"]
    rows = []
    t = 0
    # three launches on 256 blocks of 768 threads (600, 590, 610 us), one on 100 blocks
    for dur_us, blocks in ((600, 256), (590, 256), (610, 256), (80, 100)):
        rows.append({"Kernel_Name": STEP, "Start_Timestamp": t, "End_Timestamp": t + dur_us * 1000,
                     "Workgroup_Size_X": 768, "Workgroup_Size_Y": 1, "Workgroup_Size_Z": 1,
                     "Grid_Size_X": blocks * 768, "Grid_Size_Y": 1, "Grid_Size_Z": 1})
        t += 10 ** 6
    path = tmp_path / "trace.csv"
    _write_csv(path, fields, rows)
    bench.trace_summary(str(path))
    out = capsys.readouterr().out.splitlines()
    body = [line for line in out if line.startswith("| `")]
    assert len(body) == 2
    first = [c.strip() for c in body[0].strip("|").split("|")]
    assert first[0] == "`k_step_fused<float, true>`"
    assert first[1] == "256 x 768"
    assert first[2] == "3"
    assert abs(float(first[3]) - 600.0) < 1e-9            # average
    assert float(first[4]) == 590.0 and float(first[5]) == 610.0
    second = [c.strip() for c in body[1].strip("|").split("|")]
    assert second[1] == "100 x 768" and second[2] == "1"
    share = float(first[6].rstrip("% "))
    assert abs(share - 100 * 1800 / 1880) < 0.01


def test_traffic_record_scales_by_the_copy(tmp_path, monkeypatch):
    """FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the step, each scaled
    so that the 1 GiB copy reads or writes exactly 1 GiB."""
    fields = ["Kernel_Name", "Counter_Name", "Counter_Value", "Grid_Size"]
    copy = "__amd_rocclr_copyBuffer"
    gib_kib = (1 << 30) / 1024
    fetch = [{"Kernel_Name": copy, "Counter_Name": "FETCH_SIZE", "Counter_Value": gib_kib / 2,
              "Grid_Size": 1 << 20}]
    fetch += [{"Kernel_Name": STEP, "Counter_Name": "FETCH_SIZE", "Counter_Value": v,
               "Grid_Size": 256 * 768} for v in (500000.0, 520000.0)]
    write = [{"Kernel_Name": copy, "Counter_Name": "WRITE_SIZE", "Counter_Value": gib_kib,
              "Grid_Size": 1 << 20}]
    write += [{"Kernel_Name": STEP, "Counter_Name": "WRITE_SIZE", "Counter_Value": 1050000.0,
               "Grid_Size": 256 * 768}]
    fpath, wpath = tmp_path / "fetch.csv", tmp_path / "write.csv"
    _write_csv(fpath, fields, fetch)
    _write_csv(wpath, fields, write)
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    bench.record_traffic(str(fpath), str(wpath), "test_workload")
    rec = json.loads(out.read_text())
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    assert rec["read_bytes"] == 510000.0 * 1024 * 2
    assert rec["write_bytes"] == 1050000.0 * 1024
    assert rec["bytes_per_launch"] == rec["read_bytes"] + rec["write_bytes"]
    assert rec["kernel_digest"] == bench.kernel_digest()
    assert rec["dispatches"] == [2, 1]
