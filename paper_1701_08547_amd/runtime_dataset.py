"""Measured-runtime dataset for the learned correction.

Instances are (family, problem size) pairs of the three parametric kernel
families built into the library (matvec, 5-point stencil, reduction; see
``include/sa_runtime.h``).  Each instance is timed at the 128 configurations
T in {64, 128, ..., 1024} x U in {1, ..., 8} by the native harness with the
paper's protocol (one warm-up launch, ten timed launches, the fifth smallest
kept; Sec. IV-A).  Each (instance, configuration) row also gets the static
model's inputs, read from the family's own gfx950 code (asm_features):
per-thread instruction counts (loop bodies times trip counts), registers,
LDS bytes, a divergence share, block size, unroll factor and grid.

Sizes are log-uniform per family: matvec n in [1024, 32768] (rounded to a
multiple of 840 in [1680, 32760]), stencil n in [512, 8192], reduction n in [2^20, 2^28];
inputs N(0, 1).

CLI (GPU): python -m paper_1701_08547_amd.runtime_dataset --per-family 500 \\
              --out runtime.npz
A large dataset is measured in parts (--family, --part/--parts, --times-only:
only the timings and the instance list are written) and assembled on any
host with --assemble, which recomputes the static rows.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import sys
import time

import numpy as np

from . import api, asm_features, workloads

FAMILIES = ("matvec", "stencil", "reduce")
FAMILY_ID = {f: i for i, f in enumerate(FAMILIES)}
SIZE_RANGE = {"matvec": (1024, 32768), "stencil": (512, 8192), "reduce": (1 << 20, 1 << 28)}
T_VALUES = np.arange(64, 1025, 64, dtype=np.int32)
U_VALUES = np.arange(1, 9, dtype=np.int32)
N_CFG = T_VALUES.size * U_VALUES.size
DATASET_ID = 3  # seed stream of the measured-runtime workload
COUNT_FIELDS = ("n_fp", "n_int", "n_ld", "n_st", "n_br", "n_bar", "n_reg")


def config_grid():
    """The 128 (T, U) configurations, T slowest."""
    T, U = np.meshgrid(T_VALUES, U_VALUES, indexing="ij")
    return np.ascontiguousarray(T.reshape(-1)), np.ascontiguousarray(U.reshape(-1))


def sample_instances(per_family: int, seed: int = 0):
    """[(family, n)] with log-uniform sizes, `per_family` of each family."""
    g = workloads.rng(DATASET_ID, 100 + int(seed))
    out = []
    for fam in FAMILIES:
        lo, hi = SIZE_RANGE[fam]
        n = np.floor(np.exp(g.uniform(np.log(lo), np.log(hi + 1), per_family))).astype(np.int64)
        n = np.clip(n, lo, hi)
        if fam == "matvec":
            n = np.clip(np.round(n / 840.0).astype(np.int64) * 840, 1680, 32760)
        out += [(fam, int(x)) for x in n]
    return out


def _lib():
    return api.lib()


def grid(fam: str, n: int, T: int, U: int, n_cu: int) -> int:
    g = int(_lib().sa_rt_grid(FAMILY_ID[fam], n, T, U, n_cu))
    if g < 1:
        raise ValueError("(%s, n=%d, T=%d, U=%d) outside the family's domain" % (fam, n, T, U))
    return g


def trips(fam: str, n: int, T: int, U: int, G: int, n_loops: int):
    out = []
    for loop in range(n_loops):
        t = int(_lib().sa_rt_trips(FAMILY_ID[fam], n, T, U, G, loop))
        if t < 0:
            raise ValueError("%s has no loop %d" % (fam, loop))
        out.append(t)
    return out


def static_rows(instances, n_cu: int, kernels=None) -> dict:
    """Static model inputs of every (instance, configuration) row."""
    kernels = kernels or asm_features.runtime_kernels()
    T, U = config_grid()
    n_rows = len(instances) * N_CFG
    cols = {f: np.zeros(n_rows, np.int64) for f in COUNT_FIELDS}
    cols.update(family=np.zeros(n_rows, np.int32), n=np.zeros(n_rows, np.int64), block=np.zeros(n_rows, np.int32),
                unroll=np.zeros(n_rows, np.int32), grid=np.zeros(n_rows, np.int32), regs=np.zeros(n_rows, np.int32),
                lds=np.zeros(n_rows, np.int32), div=np.zeros(n_rows, np.float32))
    r = 0
    for fam, n in instances:
        for t, u in zip(T, U):
            km = kernels[(fam, int(u))]
            G = grid(fam, n, int(t), int(u), n_cu)
            tr = trips(fam, n, int(t), int(u), G, len(km.loops))
            c = km.counts(tr)
            for f in COUNT_FIELDS:
                cols[f][r] = c[f]
            cols["family"][r] = FAMILY_ID[fam]
            cols["n"][r] = n
            cols["block"][r] = t
            cols["unroll"][r] = u
            cols["grid"][r] = G
            cols["regs"][r] = km.regs
            cols["lds"][r] = km.lds
            cols["div"][r] = km.divergence(tr)
            r += 1
    return cols


def measure(instances, n_cu: int, device="cuda", warmup: int = 1, reps: int = 10, keep: int = 5, seed: int = 0,
            log=None):
    """Milliseconds [n_instances, 128]: the keep-th smallest of `reps` timed
    launches after `warmup` untimed ones, per configuration."""
    import torch

    T, U = config_grid()
    out = np.zeros((len(instances), N_CFG), np.float32)
    gen = torch.Generator(device=device)
    gen.manual_seed(170108547 + int(seed))
    L = _lib()
    bufs = {}
    # one set of buffers per family, sized for its largest instance
    for fam in FAMILIES:
        sizes = [n for f, n in instances if f == fam]
        if not sizes:
            continue
        nmax = max(sizes)
        fid = FAMILY_ID[fam]
        b = []
        for which in range(3):
            m = int(L.sa_rt_buffer_floats(fid, nmax, which))
            t = torch.randn(m, generator=gen, device=device) if m else None
            b.append(t)
        bufs[fam] = b
    ms = np.zeros(N_CFG, np.float32)
    t0 = time.time()
    stream = torch.cuda.current_stream(device).cuda_stream
    for i, (fam, n) in enumerate(instances):
        a, bb, c = bufs[fam]
        p = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
        st = L.sa_rt_measure(FAMILY_ID[fam], n, p(a), p(bb), p(c), T.ctypes.data_as(ctypes.c_void_p),
                             U.ctypes.data_as(ctypes.c_void_p), N_CFG, n_cu, warmup, reps, keep,
                             ms.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(stream))
        if st != 0:
            raise RuntimeError("sa_rt_measure: %s" % L.sa_rt_last_error().decode())
        out[i] = ms
        if log and (i + 1) % 50 == 0:
            log("measured %d / %d instances, %.1f s" % (i + 1, len(instances), time.time() - t0))
    return out


class Timer:
    """The timing harness on device buffers sized for a set of instances:
    time(fam, n, T, U) runs the paper's protocol (one warm-up launch, ten
    timed launches, the fifth smallest kept; Sec. IV-A) on the given
    configurations only and returns their milliseconds and the wall-clock
    seconds the whole measurement took (launches, events and the host's
    waits included): the cost an empirical search pays for them."""

    def __init__(self, instances, n_cu: int, device="cuda", seed: int = 0):
        import torch

        self.n_cu, self.device = n_cu, device
        gen = torch.Generator(device=device)
        gen.manual_seed(170108547 + int(seed))
        L = _lib()
        self.bufs = {}
        for fam in FAMILIES:
            sizes = [n for f, n in instances if f == fam]
            if sizes:
                self.bufs[fam] = [torch.randn(m, generator=gen, device=device) if m else None
                                  for m in (int(L.sa_rt_buffer_floats(FAMILY_ID[fam], max(sizes), w))
                                            for w in range(3))]
        torch.cuda.synchronize(device)

    def time(self, fam: str, n: int, T, U, warmup: int = 1, reps: int = 10, keep: int = 5):
        import torch

        T = np.ascontiguousarray(T, dtype=np.int32)
        U = np.ascontiguousarray(U, dtype=np.int32)
        ms = np.zeros(T.size, np.float32)
        a, b, c = self.bufs[fam]
        p = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
        stream = torch.cuda.current_stream(self.device).cuda_stream
        t0 = time.perf_counter()
        st = _lib().sa_rt_measure(FAMILY_ID[fam], n, p(a), p(b), p(c), T.ctypes.data_as(ctypes.c_void_p),
                                  U.ctypes.data_as(ctypes.c_void_p), int(T.size), self.n_cu, warmup, reps, keep,
                                  ms.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(stream))
        wall = time.perf_counter() - t0
        if st != 0:
            raise RuntimeError("sa_rt_measure: %s" % _lib().sa_rt_last_error().decode())
        return ms, wall


def build(per_family: int, seed: int = 0, device="cuda", log=None) -> dict:
    import torch

    n_cu = torch.cuda.get_device_properties(device).multi_processor_count
    inst = sample_instances(per_family, seed)
    rows = static_rows(inst, n_cu)
    ms = measure(inst, n_cu, device, seed=seed, log=log)
    rows["ms"] = ms.reshape(-1)
    rows["instance"] = np.repeat(np.arange(len(inst), dtype=np.int32), N_CFG)
    rows["n_cu"] = np.array([n_cu])
    return rows


def select(instances, family=None, part: int = 0, parts: int = 1):
    """Indices of one contiguous share of the instances (optionally of one
    family): part `part` of `parts` equal slices."""
    idx = [i for i, (f, _) in enumerate(instances) if family is None or f == family]
    lo, hi = len(idx) * part // parts, len(idx) * (part + 1) // parts
    return idx[lo:hi]


def measure_part(per_family: int, seed: int = 0, family=None, part: int = 0, parts: int = 1, device="cuda",
                 log=None) -> dict:
    """Timings of one share of the sampled instances, with their indices."""
    import torch

    n_cu = torch.cuda.get_device_properties(device).multi_processor_count
    inst = sample_instances(per_family, seed)
    idx = select(inst, family, part, parts)
    ms = measure([inst[i] for i in idx], n_cu, device, seed=seed, log=log)
    return {"index": np.asarray(idx, np.int64), "ms": ms, "n_cu": np.array([n_cu]),
            "per_family": np.array([per_family]), "seed": np.array([seed])}


def assemble(parts) -> dict:
    """Rows of the instances covered by the given parts (dicts or paths of
    `measure_part` outputs taken from one sampling): timings in instance
    order, static model inputs recomputed here."""
    parts = [load(p) if isinstance(p, str) else p for p in parts]
    meta = {(int(p["per_family"][0]), int(p["seed"][0]), int(p["n_cu"][0])) for p in parts}
    if len(meta) != 1:
        raise ValueError("parts come from different samplings or devices: %s" % sorted(meta))
    per_family, seed, n_cu = meta.pop()
    idx = np.concatenate([p["index"] for p in parts])
    ms = np.concatenate([p["ms"] for p in parts])
    if np.unique(idx).size != idx.size:
        raise ValueError("parts overlap")
    order = np.argsort(idx, kind="stable")
    idx, ms = idx[order], ms[order]
    inst = sample_instances(per_family, seed)
    rows = static_rows([inst[i] for i in idx], n_cu)
    rows["ms"] = ms.reshape(-1)
    rows["instance"] = np.repeat(np.arange(idx.size, dtype=np.int32), N_CFG)
    rows["n_cu"] = np.array([n_cu])
    return rows


def save(path: str, data: dict):
    np.savez_compressed(path, **data)


def load(path: str) -> dict:
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--per-family", type=int, default=500)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--family", choices=FAMILIES)
    ap.add_argument("--part", type=int, default=0)
    ap.add_argument("--parts", type=int, default=1)
    ap.add_argument("--times-only", action="store_true")
    ap.add_argument("--assemble", nargs="+", metavar="PART")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)
    t0 = time.time()
    if a.times_only:
        d = measure_part(a.per_family, a.seed, a.family, a.part, a.parts, log=log)
        save(a.out, d)
        print(json.dumps({"instances": int(d["index"].size), "seconds": time.time() - t0}), flush=True)
        return 0
    d = assemble(a.assemble) if a.assemble else build(a.per_family, a.seed, log=log)
    save(a.out, d)
    print(json.dumps({"rows": int(d["ms"].size), "instances": int(d["instance"].max() + 1),
                      "seconds": time.time() - t0}), flush=True)


if __name__ == "__main__":
    sys.exit(main())
