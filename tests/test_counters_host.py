"""The counter reduction behind bench.py's traffic figure, on a synthetic
rocprofv3 counter file: per-dispatch sums over counter instances, the median
over the kernel's dispatches, and the copy-calibrated scaling."""
import csv

from paper_1701_08547_amd import counters

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(FIELDS, r)))


def test_traffic_reduction(tmp_path):
    k = "void sa::(anonymous namespace)::sa_plan_kernel<(sa::Mode)0, true, true, 1, 4>(...)"
    # two instances per dispatch, three dispatches of the kernel, one of another kernel
    _write(tmp_path / "f.csv", [(1, k, "FETCH_SIZE", 50.0), (1, k, "FETCH_SIZE", 50.0), (2, k, "FETCH_SIZE", 60.0),
                                (2, k, "FETCH_SIZE", 60.0), (3, k, "FETCH_SIZE", 55.0), (3, k, "FETCH_SIZE", 55.0),
                                (4, "other", "FETCH_SIZE", 9e9)])
    _write(tmp_path / "w.csv", [(1, k, "WRITE_SIZE", 100.0), (2, k, "WRITE_SIZE", 100.0)])
    _write(tmp_path / "cf.csv", [(1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 128000.0)])
    _write(tmp_path / "cw.csv", [(1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 256000.0)])
    d = counters.per_dispatch(str(tmp_path / "f.csv"), "sa_plan_kernel")
    assert d == {"FETCH_SIZE": [100.0, 120.0, 110.0]}

    class A:
        fetch, write = str(tmp_path / "f.csv"), str(tmp_path / "w.csv")
        copy_fetch, copy_write = str(tmp_path / "cf.csv"), str(tmp_path / "cw.csv")
        copy_kernel, algorithmic, shape, workload = "copyBuffer", 330 * 1024, "8192,1,4", "test"

    rec = counters.traffic(A)
    # median fetch 110 KiB x 2 (the copy reads half its size) + 100 KiB written x 1
    assert rec["bytes_per_launch"] == (110 * 2 + 100) * 1024
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0 and rec["shape"] == [8192, 1, 4]
    assert rec["launches_counted"] == 3
