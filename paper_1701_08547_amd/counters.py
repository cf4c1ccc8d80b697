"""Reduce rocprofv3 counter collections into the per-launch figures bench.py
reports beside the scoring kernel's roofline.

Input: the ``*_counter_collection.csv`` files of ``rocprofv3 --pmc ... -f csv``
runs (one counter set per run).  Counts of one kernel are taken per dispatch
(summed over the counter's instances), and the median over that kernel's
dispatches is kept.

  traffic  FETCH_SIZE and WRITE_SIZE (KiB) of the scoring kernel, each scaled
           by what the same counter reads for a device copy of known size
           (bench.py --copy-calibration: 256,000 KiB read and written per
           launch), in bytes per launch
  valu     SQ_INSTS_VALU and its neighbours per launch

CLI:
  python -m paper_1701_08547_amd.counters traffic --fetch F.csv --write W.csv \\
      --copy-fetch CF.csv --copy-write CW.csv --shape 8192,2,4 --out profiles/traffic_c1.json
  python -m paper_1701_08547_amd.counters valu --csv V.csv --shape 8192,2,4 --out profiles/valu_c1.json
"""
from __future__ import annotations

import argparse
import csv
import json
import statistics

COPY_KIB = 256000
KERNEL = "sa_plan_kernel"


def per_dispatch(path: str, kernel_substr: str) -> dict:
    """{counter: [value per dispatch]} for the dispatches of kernels whose
    name contains `kernel_substr`."""
    acc: dict = {}
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            name = row.get("Kernel_Name", "")
            if kernel_substr not in name:
                continue
            key = (row.get("Dispatch_Id") or row.get("Correlation_Id"), row["Counter_Name"])
            acc[key] = acc.get(key, 0.0) + float(row["Counter_Value"])
    out: dict = {}
    for (_, counter), v in sorted(acc.items()):
        out.setdefault(counter, []).append(v)
    return out


def median_of(path: str, counter: str, kernel_substr: str) -> tuple[float, int]:
    vals = per_dispatch(path, kernel_substr).get(counter, [])
    if not vals:
        raise SystemExit("no %s dispatches of %s in %s" % (counter, kernel_substr, path))
    return statistics.median(vals), len(vals)


def traffic(a) -> dict:
    fetch, n = median_of(a.fetch, "FETCH_SIZE", KERNEL)
    write, _ = median_of(a.write, "WRITE_SIZE", KERNEL)
    cfetch, _ = median_of(a.copy_fetch, "FETCH_SIZE", a.copy_kernel)
    cwrite, _ = median_of(a.copy_write, "WRITE_SIZE", a.copy_kernel)
    fs, ws = COPY_KIB / cfetch, COPY_KIB / cwrite
    nbytes = int(round((fetch * fs + write * ws) * 1024))
    return {"kernel": KERNEL, "workload": a.workload, "shape": [int(x) for x in a.shape.split(",")],
            "bytes_per_launch": nbytes, "fetch_kib_raw_median": fetch, "write_kib_raw_median": write,
            "fetch_scale": round(fs, 5), "write_scale": round(ws, 5), "algorithmic_bytes": a.algorithmic,
            "ratio_to_algorithmic": round(nbytes / a.algorithmic, 5), "launches_counted": n,
            "source_digest": digest()}


def valu(a) -> dict:
    d = per_dispatch(a.csv, KERNEL)
    if "SQ_INSTS_VALU" not in d:
        raise SystemExit("no SQ_INSTS_VALU dispatches of %s in %s" % (KERNEL, a.csv))
    names = {"SQ_INSTS_VALU": "valu_wave_insts_per_launch", "SQ_INSTS_SALU": "salu_insts_per_launch",
             "SQ_INSTS_LDS": "lds_insts_per_launch", "SQ_INSTS_VMEM_RD": "vmem_rd_insts_per_launch",
             "SQ_INSTS_VMEM_WR": "vmem_wr_insts_per_launch", "SQ_WAVES": "waves_per_launch"}
    out = {"kernel": KERNEL, "workload": a.workload, "shape": [int(x) for x in a.shape.split(",")]}
    for c, key in names.items():
        if c in d:
            out[key] = int(round(statistics.median(d[c])))
    out["launches_counted"] = len(d["SQ_INSTS_VALU"])
    out["source_digest"] = digest()
    return out


def digest() -> str:
    from . import build

    return build.plain_kernel_digest()


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("traffic")
    for f in ("fetch", "write", "copy_fetch", "copy_write"):
        t.add_argument("--" + f.replace("_", "-"), dest=f, required=True)
    t.add_argument("--copy-kernel", default="copyBuffer")
    t.add_argument("--algorithmic", type=int, default=24 * 16384000)
    v = sub.add_parser("valu")
    v.add_argument("--csv", required=True)
    for p in (t, v):
        p.add_argument("--shape", required=True)
        p.add_argument("--workload", default="1000 variants x 16384 configurations, top-8")
        p.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    rec = traffic(a) if a.what == "traffic" else valu(a)
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
