"""Throughput of the plain scoring pass on the other batch shapes, one JSON
object per workload:

  c0  one variant x 4,096 configurations (block x unroll x registers), top-8:
      launch-bound, so the figure is the time per launch, eager (host call
      included) and inside a graph of back-to-back launches, for the
      autotuned plan shape;
  c2  10,000 variants with search spaces log-uniform in [64, 262,144]
      (about 3.2e8 evaluations), grid column present, top-16 fused, no
      per-evaluation outputs: the plan shape is autotuned (tiles
      {1024, 2048, 4096, 8192} x {1, 2, 4} items per lane x {4, 8, 16} waves
      per workgroup), then K launches are replayed as one graph.

Algorithmic bytes per evaluation: 16 (four int32 configuration columns
read); per variant 44 (nine per-variant fields and the segment offset) plus
the top-k rows written (8 B per slot).

CLI (GPU): python -m paper_1701_08547_amd.report c0 c2 [--steps K]
"""
from __future__ import annotations

import argparse
import json

from . import api, workloads

HBM_PEAK_GBS = 8000.0


def _graph_time(fn, steps: int, warmup: int):
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(steps):
            fn()
    g.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _eager_time(fn, reps: int):
    import time

    import torch

    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def _bytes(b, k: int) -> int:
    return 16 * b.n_evals + (44 + 8 * k) * b.n_var


def c0(arch: dict, steps: int, warmup: int) -> dict:
    import torch

    b = workloads.c0()
    var, cfg = api.device_batch(b)
    dev = cfg["seg"].device
    out = {"idx": torch.empty((1, 8), dtype=torch.int32, device=dev),
           "val": torch.empty((1, 8), dtype=torch.float32, device=dev)}
    shape, _ = api.autotune(arch, var, cfg, k=8, reps=20, outputs=out, want_score=False, want_occ=False)
    plan = api.Plan(b.seg, k=8, shape=shape)
    ws = api.Workspace(plan.workspace_bytes, dev)
    fn = lambda: plan.score(arch, var, cfg, want_score=False, want_occ=False, outputs=out, workspace=ws)
    ms_graph = _graph_time(fn, steps, warmup)
    ms_eager = _eager_time(fn, steps)
    return {"workload": "1 variant x 4,096 configurations (T x U x R), top-8", "n_evals": b.n_evals,
            "plan_shape": list(plan.shape), "us_per_launch_graph": ms_graph * 1e3,
            "us_per_call_eager": ms_eager * 1e3, "configs_per_s_graph": b.n_evals / (ms_graph * 1e-3)}


def c2(arch: dict, steps: int, warmup: int, n_cu: int) -> dict:
    import torch

    b = workloads.c2(n_cu=n_cu)
    var, cfg = api.device_batch(b)
    k = 16
    dev = cfg["seg"].device
    out = {"idx": torch.empty((b.n_var, k), dtype=torch.int32, device=dev),
           "val": torch.empty((b.n_var, k), dtype=torch.float32, device=dev)}
    shape, ms_tune = api.autotune(arch, var, cfg, k=k, reps=5, outputs=out, want_score=False, want_occ=False)
    plan = api.Plan(b.seg, k=k, shape=shape)
    ws = api.Workspace(plan.workspace_bytes, dev)
    fn = lambda: plan.score(arch, var, cfg, want_score=False, want_occ=False, outputs=out, workspace=ws)
    ms = _graph_time(fn, steps, warmup)
    nbytes = _bytes(b, k)
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"workload": "10,000 variants, search spaces log-uniform in [64, 262144], top-16",
            "n_evals": b.n_evals, "plan_shape": list(shape), "autotune_ms": ms_tune, "ms_per_launch": ms,
            "configs_per_s": b.n_evals / (ms * 1e-3), "algorithmic_bytes": nbytes, "GBps": gbs,
            "hbm_frac": gbs / HBM_PEAK_GBS, "steps": steps}


def main(argv=None):
    import torch

    ap = argparse.ArgumentParser()
    ap.add_argument("workloads", nargs="+", choices=("c0", "c2"))
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    a = ap.parse_args(argv)
    arch = api.arch_default(0)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    for w in a.workloads:
        r = c0(arch, a.steps, a.warmup) if w == "c0" else c2(arch, a.steps, a.warmup, n_cu)
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
