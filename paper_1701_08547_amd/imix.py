"""Static against dynamic instruction mix of the measured kernel families.

The paper checks its statically derived instruction mix against the dynamic
mix that hardware counters report for the same runs (Sec. IV-B, the
error rates of the instruction-mix metrics).  Here the static side is this
library's own gfx950 assembly (asm_features: per-loop counts by the
hardware's issue classes, times the host-computed trip counts, times the
number of waves launched); the dynamic side is the per-dispatch SQ counters
(SQ_INSTS_VALU, _SALU, _SMEM, _VMEM_RD, _VMEM_WR, _LDS and SQ_WAVES) that
rocprofv3 collects while `run` launches each case exactly once.

  GPU, under rocprofv3 --pmc:  python -m paper_1701_08547_amd.imix run
  any host:                    python -m paper_1701_08547_amd.imix compare --counters X.csv
  any host:                    python -m paper_1701_08547_amd.imix table --counters X.csv --out T.txt
                               (the per-dispatch counts as a small text table,
                               which `compare --table T.txt` reads instead)

Static per-wave counts assume every lane takes the same path and every wave
runs the same trip counts; the differences the comparison reports are the
model's error: branches whose exec mask is empty for whole waves, and waves
that run fewer iterations than the counted trip count.
"""
from __future__ import annotations

import argparse
import csv
import ctypes
import json
import re
import sys

import numpy as np

from . import api, asm_features, runtime_dataset as rd

COUNTERS = {"SQ_INSTS_VALU": "valu", "SQ_INSTS_SALU": "salu", "SQ_INSTS_SMEM": "smem", "SQ_INSTS_VMEM_RD": "vmem_rd",
            "SQ_INSTS_VMEM_WR": "vmem_wr", "SQ_INSTS_LDS": "lds"}
SIZES = {"matvec": (1680, 8400, 32760), "stencil": (512, 2048, 8192), "reduce": (1 << 20, 1 << 24, 1 << 28)}
BLOCKS = (64, 256, 1024)
UNROLLS = (1, 4, 8)


def cases():
    """(family, n, T, U) in launch order."""
    return [(f, n, T, U) for f in rd.FAMILIES for n in SIZES[f] for T in BLOCKS for U in UNROLLS]


def predicted(cs, n_cu: int, kernels=None) -> list:
    """Static totals per case: waves launched and per-class instruction
    counts summed over them."""
    kernels = kernels or asm_features.runtime_kernels()
    out = []
    for fam, n, T, U in cs:
        km = kernels[(fam, U)]
        G = rd.grid(fam, n, T, U, n_cu)
        tr = rd.trips(fam, n, T, U, G, len(km.loops))
        waves = G * ((T + 63) // 64)
        per_wave = km.hw_counts(tr)
        out.append({"family": fam, "n": n, "T": T, "U": U, "grid": G, "waves": waves,
                    "static": {k: v * waves for k, v in per_wave.items()}})
    return out


def run(cs, device="cuda"):
    """One launch of every case, in order, on the library's timing harness
    (no warm-up, one timed launch)."""
    import torch

    L = api.lib()
    n_cu = torch.cuda.get_device_properties(device).multi_processor_count
    gen = torch.Generator(device=device)
    gen.manual_seed(170108547)
    bufs = {}
    for fam in rd.FAMILIES:
        nmax = max(n for f, n, _, _ in cs if f == fam)
        fid = rd.FAMILY_ID[fam]
        bufs[fam] = [torch.randn(m, generator=gen, device=device) if m else None
                     for m in (int(L.sa_rt_buffer_floats(fid, nmax, w)) for w in range(3))]
    torch.cuda.synchronize()
    ms = np.zeros(1, np.float32)
    stream = torch.cuda.current_stream(device).cuda_stream
    p = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
    for fam, n, T, U in cs:
        a, b, c = bufs[fam]
        Ta, Ua = np.array([T], np.int32), np.array([U], np.int32)
        st = L.sa_rt_measure(rd.FAMILY_ID[fam], n, p(a), p(b), p(c), Ta.ctypes.data_as(ctypes.c_void_p),
                             Ua.ctypes.data_as(ctypes.c_void_p), 1, n_cu, 0, 1, 1,
                             ms.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(stream))
        if st != 0:
            raise RuntimeError("sa_rt_measure: %s" % L.sa_rt_last_error().decode())
    torch.cuda.synchronize()
    return n_cu


def read_counters(path: str) -> list:
    """Per dispatch of a measured-family kernel, in dispatch order: counter
    name -> value (rocprofv3 counter-collection CSV)."""
    disp = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            if "rt_" not in r["Kernel_Name"]:
                continue
            d = disp.setdefault(int(r["Dispatch_Id"]), {"kernel": r["Kernel_Name"]})
            d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return [disp[k] for k in sorted(disp)]


TABLE_FIELDS = ("kernel", "SQ_WAVES") + tuple(COUNTERS)


def write_table(dyn: list, path: str):
    """The measured-family dispatches' counter sums as a text table (one
    line per dispatch, launch order)."""
    with open(path, "w") as f:
        f.write("# " + " ".join(TABLE_FIELDS) + "\n")
        for d in dyn:
            m = re.search(r"rt_\w+(<[^>]*>)?", d["kernel"])
            f.write(" ".join([m.group(0).replace(" ", "") if m else "unknown"] +
                             ["%d" % int(round(d.get(c, -1))) for c in TABLE_FIELDS[1:]]) + "\n")


def read_table(path: str) -> list:
    out = []
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            d = {"kernel": parts[0]}
            for c, v in zip(TABLE_FIELDS[1:], parts[1:]):
                if int(v) >= 0:
                    d[c] = float(v)
            out.append(d)
    return out


def compare(pred: list, dyn: list) -> dict:
    """Error rates (static - dynamic) / dynamic per case and class; mean
    absolute error per family and class."""
    if len(pred) != len(dyn):
        raise ValueError("%d cases, %d counted dispatches" % (len(pred), len(dyn)))
    rows = []
    for p, d in zip(pred, dyn):
        fam = p["family"]
        if ("rt_" + fam) not in d["kernel"]:
            raise ValueError("dispatch order: expected %s, got %s" % (fam, d["kernel"]))
        row = {k: p[k] for k in ("family", "n", "T", "U", "waves")}
        row["waves_counted"] = d.get("SQ_WAVES")
        for cn, cls in COUNTERS.items():
            if cn in d:
                dv, sv = d[cn], p["static"][cls]
                row[cls] = {"static": sv, "dynamic": dv, "error": (sv - dv) / dv if dv else (0.0 if sv == 0 else None)}
        rows.append(row)
    summary = {}
    for fam in rd.FAMILIES:
        fr = [r for r in rows if r["family"] == fam]
        s = {}
        for cls in COUNTERS.values():
            errs = [abs(r[cls]["error"]) for r in fr if cls in r and r[cls]["error"] is not None]
            if errs:
                s[cls] = {"mean_abs_error": float(np.mean(errs)), "max_abs_error": float(np.max(errs))}
        s["waves_exact"] = all(r["waves_counted"] is None or r["waves_counted"] == r["waves"] for r in fr)
        summary[fam] = s
    return {"summary": summary, "cases": rows}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=("run", "compare", "table"))
    ap.add_argument("--counters", help="rocprofv3 counter-collection CSV of a `run`")
    ap.add_argument("--table", help="per-dispatch text table written by `table` (instead of --counters)")
    ap.add_argument("--n-cu", type=int, default=256)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    cs = cases()
    if a.what == "run":
        n_cu = run(cs)
        print(json.dumps({"cases": len(cs), "n_cu": n_cu}), flush=True)
        return 0
    if a.what == "table":
        write_table(read_counters(a.counters), a.out)
        return 0
    dyn = read_table(a.table) if a.table else read_counters(a.counters)
    rep = compare(predicted(cs, a.n_cu), dyn)
    txt = json.dumps(rep, indent=1)
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt + "\n")
    print(json.dumps(rep["summary"], indent=1))
    return 0


if __name__ == "__main__":
    sys.exit(main())
