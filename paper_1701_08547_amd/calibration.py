"""Instruction costs of Eq. 6 measured on this device, and the plain model's
ranking with them.

The paper weights each instruction category by the inverse of its
instructions per cycle per multiprocessor (Table II, NVIDIA only).  The CDNA4
descriptor's defaults follow Table II's convention from unit counts
(c_fp = c_int = 2^-6, c_mem = c_ctrl = c_sync = 2^-4, c_reg = 2^-5).  Here
each category's cost is measured by a microbenchmark (sa_rt_cpi:
CU-cycles per thread-instruction) and put into the descriptor:

  c_fp, c_int, c_mem, c_reg   the measured cost per instruction;
  c_ctrl                      the measured cost of one loop iteration's
                              branch with its scalar counter;
  c_sync                      the measured cost per thread of one barrier of
                              a four-wave workgroup, divided by four (the
                              score charges c_sync x n_bar x W_B).

The plain model's top-1 regret and Spearman correlation against measured
runtimes (runtime_dataset) are then reported with the default and with the
measured constants.

CLI (GPU): python -m paper_1701_08547_amd.calibration [--parts P ... | --data D]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import sys

import numpy as np

from . import api, correction, runtime_dataset

CATEGORIES = ("fp", "int", "mem", "ctrl", "sync", "reg")
SYNC_WAVES = 4  # waves per workgroup of the barrier microbenchmark


def measure_cpi(reps: int = 9, device="cuda") -> dict:
    """Category -> (CU-cycles per thread-instruction, median ms)."""
    import torch

    L = api.lib()
    buf = torch.zeros(4096 + 256, dtype=torch.float32, device=device)
    out = {}
    for i, c in enumerate(CATEGORIES):
        cpi, ms = ctypes.c_float(), ctypes.c_float()
        st = L.sa_rt_cpi(i, reps, ctypes.c_void_p(buf.data_ptr()), ctypes.byref(cpi), ctypes.byref(ms),
                         ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream))
        if st != 0:
            raise RuntimeError("sa_rt_cpi(%s): %s" % (c, L.sa_rt_last_error().decode()))
        out[c] = (float(cpi.value), float(ms.value))
    return out


def calibrated_arch(arch: dict, measured: dict) -> dict:
    a = dict(arch)
    for c in ("fp", "int", "mem", "ctrl", "reg"):
        a["cpi_" + c] = measured[c][0]
    a["cpi_sync"] = measured["sync"][0] / SYNC_WAVES
    return a


def plain_ranking(data: dict, arch: dict, ids=None, device="cuda") -> dict:
    """Mean top-1 regret and Spearman of the plain key ln(score) over the
    dataset's instances (all, or `ids`)."""
    n_inst = int(data["instance"].max()) + 1
    var, cfg = correction.device_rows(data, device)
    ln_s = api.features(arch, var, cfg)[:, 22].cpu().numpy().astype(np.float64).reshape(n_inst, -1)
    ms = data["ms"].astype(np.float64).reshape(n_inst, -1)
    ids = np.arange(n_inst) if ids is None else np.asarray(ids)
    rg = np.array([correction.regret(ln_s[i], ms[i]) for i in ids])
    sp = np.array([correction.spearman(ln_s[i], ms[i]) for i in ids])
    fam = data["family"].reshape(n_inst, -1)[ids, 0]
    out = {"instances": int(ids.size), "regret": float(rg.mean()), "regret_ci": correction.bootstrap_ci(rg),
           "spearman": float(sp.mean())}
    for f, name in enumerate(runtime_dataset.FAMILIES):
        m = fam == f
        if m.any():
            out[name] = {"regret": float(rg[m].mean()), "spearman": float(sp[m].mean())}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    src = ap.add_mutually_exclusive_group()
    src.add_argument("--data")
    src.add_argument("--parts", nargs="+")
    ap.add_argument("--reps", type=int, default=9)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    arch = api.arch_default(0)
    meas = measure_cpi(a.reps)
    cal = calibrated_arch(arch, meas)
    rep = {"cpi": {c: {"measured": meas[c][0], "ms": meas[c][1], "descriptor": arch["cpi_" + c],
                       "calibrated": cal["cpi_" + c]} for c in CATEGORIES}}
    if a.data or a.parts:
        data = runtime_dataset.load(a.data) if a.data else runtime_dataset.assemble(a.parts)
        rep["plain_default"] = plain_ranking(data, arch)
        rep["plain_calibrated"] = plain_ranking(data, cal)
    txt = json.dumps(rep, indent=1)
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt + "\n")
    print(txt, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
