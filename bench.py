#!/usr/bin/env python3
"""Benchmark: batched evaluation of the static autotuning model on one MI355X.

One step = one pass of the whole hot path (occupancy, score and per-variant
top-8 selection, with occupancy and score written out) over the batch of
1,000 kernel variants x 16,384 launch configurations (block x unroll x
registers x grid, 16,384,000 evaluations), inputs resident in HBM.  The step
is one persistent-kernel launch over a plan whose launch shape the library's
autotuner picks at start-up (outside the timed region); the K timed steps
are one replay of a HIP graph holding K such launches back to back.

Prints ONE JSON line (rank 0):
  value        configurations scored per second (whole job)
  roofline     the evaluation kernel against MI355X HBM peak (8 TB/s):
               algorithmic bytes = 24 B per evaluation (16 B of configuration
               columns read, 4 B occupancy + 4 B score written); valu_side
               sets its counted vector instructions against the FP32 vector
               peak, to show which bound is active
  cpu_baseline the CPU oracle (binary32 mode + top-8) on the host cores, over
               repetitions of the same workload for ~10 s
  regret       top-1 regret of the plain and the corrected ranking against
               measured runtimes of the library's own kernel families (a small
               dataset measured here, 10 % of its instances held out)
  corrected    the fused corrected pass (learned correction in the scoring
               kernel) on the same 16,384,000 evaluations
  product      the same evaluations as a product space scored without rows
               (the 16,384 configurations are the full product of the four
               value sets)
  stream_ceiling  a pure stream of the same 24 B per evaluation with no model
               arithmetic (fastest of a sweep of launch shapes): the practical
               memory ceiling of the plain pass on this device
  cold         the same pass rotating over three copies of the workload
               (columns and outputs, 1.18 GB), so that no launch finds its
               inputs in the 256 MB last-level cache
  c2           10,000 variants with search spaces log-uniform in
               [64, 262,144] (3.2e8 evaluations), top-16: one planned launch at
               the autotuner's shape, K launches as one graph
  c4           100,000 variants with spaces log-uniform in [256, 2^20]
               (1.26e10 evaluations), rows generated on the device per chunk:
               the plain and the corrected pass side by side, one pass each

The timed plan shape of the headline is the one the committed counters were
taken at (--shape); the autotuner's pick on the same batch is reported
beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "configs scored/sec, plain vs MLP-corrected; top-1 regret vs measured runtime"
HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK_TFLOPS = 2500.0
# 157.3 TFLOP/s FP32 vector peak, a fused multiply-add counting two: lane operations per second
VALU_PEAK_LANE_OPS = 157.3e12 / 2
# algorithmic dense work per evaluation: 24->128->128->1 (the K padding to 32 is not counted)
MLP_FLOP_PER_EVAL = 2 * (24 * 128 + 128 * 128 + 128)
# one training row: that forward, dL/dh1 = W2^T dL/da2, dW2, dW1 and dw3
TRAIN_FLOP_PER_ROW = MLP_FLOP_PER_EVAL + 2 * (128 * 128 + 128 * 128 + 24 * 128 + 128)
BYTES_PER_EVAL = 24
K = 8
def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--cpu-seconds", type=float, default=10.0, help="budget of the CPU-baseline leg")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic_c1.json"),
                   help="JSON with measured HBM bytes per launch of the evaluation kernel")
    p.add_argument("--valu", default=os.path.join(ROOT, "profiles", "valu_c1.json"),
                   help="JSON with counted vector instructions per launch of the evaluation kernel")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain device copy of 256,000 KiB (counter calibration under rocprofv3)")
    p.add_argument("--corrected-steps", type=int, default=10,
                   help="timed launches of the fused corrected pass on the same workload (0: skip)")
    p.add_argument("--regret-per-family", type=int, default=45,
                   help="instances per kernel family measured for the regret leg (0: skip)")
    p.add_argument("--product-steps", type=int, default=20,
                   help="timed launches of the same workload as a product space without rows (0: skip)")
    p.add_argument("--only-plain", action="store_true", help="the plain leg alone (profiling runs)")
    p.add_argument("--no-stream-ceiling", action="store_true", help="skip the stream-ceiling sweep (profiling runs)")
    p.add_argument("--cpu-baseline-batches", action="store_true",
                   help="host only: the cpu_baseline leg (the CPU oracle) on every batch shape, one thread and all "
                        "threads (no GPU work)")
    p.add_argument("--shape", default=None,
                   help="tile,items,waves of the timed plan ('auto': the autotuner's pick); default: the shape the "
                        "committed traffic counters were taken at")
    p.add_argument("--no-autotune", action="store_true", help="skip the autotuner run beside the headline")
    p.add_argument("--cold-steps", type=int, default=30, help="timed launches of the cold-cache leg (0: skip)")
    p.add_argument("--c2-steps", type=int, default=20, help="timed launches of the 10,000-variant leg (0: skip)")
    p.add_argument("--c4", type=int, default=1, help="run the 100,000-variant streamed leg (0: skip)")
    p.add_argument("--train-epochs", type=int, default=2,
                   help="timed epochs (256 steps of 4,096 rows each) of the training leg (0: skip)")
    return p.parse_args()


def source_digest() -> str:
    """Digest of the kernel sources: a traffic figure measured for other
    sources is not reported."""
    from paper_1701_08547_amd import build

    return build.plain_kernel_digest()


def copy_calibration():
    import torch

    n = 256000 * 1024 // 4  # 256,000 KiB of float32
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": 4 * n, "launches": 5}), flush=True)


def cpu_baseline(batch, seconds: float) -> dict:
    import oracle

    arch = oracle.arch_cdna4()
    nt = oracle.max_threads()
    reps, t0 = 0, time.perf_counter()
    while True:
        oracle.run(arch, batch.variants, batch.configs(), k=K, want_occ=True, want_f32=True, want_f64=False,
                   nthreads=nt)
        reps += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": reps * batch.n_evals / dt, "unit": "configs/s", "cores": nt, "kind": "oracle",
            "sample": "%d pass(es) over the full workload (%d evaluations each), binary32 scores + occupancy + "
                      "top-%d, %.1f s" % (reps, batch.n_evals, K, dt)}


def cpu_baseline_batches():
    """The cpu_baseline leg on every batch shape: the CPU oracle (binary32
    scores + occupancy + top-k) with one thread and with all, the best of a
    few repetitions, each a full pass; the streamed batch on a sample,
    extrapolated."""
    import platform

    import numpy as np

    import oracle
    from paper_1701_08547_amd import workloads

    arch = oracle.arch_cdna4()
    nt = oracle.max_threads()
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    out = {"host": {"cpu": model or platform.processor(), "threads": nt, "cpus": os.cpu_count()}, "batches": []}
    for name, batch, k in (("1 x 4,096 (T x U x R), top-8", workloads.c0(), 8),
                           ("1,000 x 16,384, top-8", workloads.c1(), 8),
                           ("10,000 variants, spaces log-uniform in [64, 262,144], top-16", workloads.c2(), 16)):
        cfgs = batch.configs()
        row = {"workload": name, "evaluations": batch.n_evals}
        for threads in (1, nt):
            best, reps, t_all = None, 0, time.perf_counter()
            while reps < 3 and (reps == 0 or time.perf_counter() - t_all < 20.0):
                t0 = time.perf_counter()
                oracle.run(arch, batch.variants, cfgs, k=k, want_occ=True, want_f32=True, want_f64=False,
                           nthreads=threads)
                dt = time.perf_counter() - t0
                best = dt if best is None else min(best, dt)
                reps += 1
            row["threads_%d" % threads] = {"seconds": best, "configs_per_s": batch.n_evals / best, "passes": reps}
        out["batches"].append(row)
        print(json.dumps(row), flush=True)
    # the 100,000-variant streamed batch: a seeded sample of 200 variants, rows rebuilt on the host (not
    # timed), extrapolated to the whole batch by evaluation count
    c4 = workloads.c4()
    vids = np.sort(np.random.default_rng(170108547).choice(c4.n_var, 200, replace=False))
    sub = c4.subset(vids)
    row = {"workload": "100,000 variants, spaces log-uniform in [256, 1,048,576], top-16: sample of 200 variants, "
                       "extrapolated", "evaluations": c4.n_evals, "sample_evaluations": sub.n_evals}
    cfgs = sub.configs()
    for threads in (1, nt):
        t0 = time.perf_counter()
        oracle.run(arch, sub.variants, cfgs, k=16, want_occ=True, want_f32=True, want_f64=False, nthreads=threads)
        dt = time.perf_counter() - t0
        row["threads_%d" % threads] = {"sample_seconds": dt, "configs_per_s": sub.n_evals / dt,
                                       "extrapolated_seconds": dt * c4.n_evals / sub.n_evals}
    out["batches"].append(row)
    print(json.dumps(row), flush=True)
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.cpu_baseline_batches:
        cpu_baseline_batches()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: a batch shards by variant, each GPU scoring its own segments "
              "with no exchange but a gather of the top-k rows; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1701_08547_amd import api, workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    arch = api.arch_default(0)
    batch = workloads.c1(n_cu=arch["n_cu"])
    var, cfg = api.device_batch(batch, dev)
    n_var, n_evals = batch.n_var, batch.n_evals
    outs = {
        "occ": torch.empty(n_evals, dtype=torch.int32, device=dev),
        "score": torch.empty(n_evals, dtype=torch.float32, device=dev),
        "idx": torch.empty((n_var, K), dtype=torch.int32, device=dev),
        "val": torch.empty((n_var, K), dtype=torch.float32, device=dev),
    }
    counted = counted_shape(args.traffic)
    tune = None
    if args.shape == "auto" or not (args.no_autotune or args.only_plain):
        # bring the clocks up before the autotuner measures anything
        plan0 = api.Plan(batch.seg, k=K)
        ws0 = api.Workspace(plan0.workspace_bytes, dev)
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < 0.5:
            plan0.score(arch, var, cfg, outputs=outs, workspace=ws0)
        torch.cuda.synchronize()
        pick, tune_ms = api.autotune(arch, var, cfg, k=K, reps=10, outputs=outs)
        tune = {"pick": {"tile": pick[0], "items_per_lane": pick[1], "waves_per_block": pick[2]},
                "median_ms": tune_ms}
    if args.shape == "auto":
        shape = pick
    elif args.shape:
        shape = tuple(int(x) for x in args.shape.split(","))
    else:
        shape = counted or (8192, 2, 4)
    plan = api.Plan(batch.seg, k=K, shape=shape)
    ws = api.Workspace(plan.workspace_bytes, dev)

    def step():
        plan.score(arch, var, cfg, outputs=outs, workspace=ws)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(max(1, args.warmup)):
            step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(args.steps):
            step()
    torch.cuda.synchronize()
    graph.replay()  # first replay uploads the graph
    torch.cuda.synchronize()

    # the graph's kernels run on the stream that replays it: the events go there
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    graph.replay()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    mean_ms = ev0.elapsed_time(ev1) / args.steps
    ms_per_step = wall * 1e3 / args.steps

    value = n_evals * args.steps / wall
    achieved = BYTES_PER_EVAL * n_evals / (mean_ms * 1e-3) / 1e9
    traffic = None
    t = counter_record(args.traffic, shape)
    if t is not None:
        traffic = t.get("bytes_per_launch")
    valu_side = None
    vc = counter_record(args.valu, shape)
    if vc is not None:
        lane_ops = vc["valu_wave_insts_per_launch"] * 64 / (mean_ms * 1e-3)
        valu_side = {"lane_ops_per_s": lane_ops, "peak": VALU_PEAK_LANE_OPS, "frac": lane_ops / VALU_PEAK_LANE_OPS,
                     "wave_insts_per_eval": vc["valu_wave_insts_per_launch"] / n_evals,
                     "note": "SQ_INSTS_VALU counted at the timed plan shape x 64 lanes / event time per launch"}

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "configs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "plain static model, 1000 variants x 16384 configs (block x unroll x regs x grid), "
                        "occupancy + score written, top-8 per variant",
            "n_variants": n_var,
            "n_evals": n_evals,
            "k": K,
            "mode": "plain",
            "plan_shape": {"tile": shape[0], "items_per_lane": shape[1], "waves_per_block": shape[2]},
            "autotune": tune,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_note": "FETCH_SIZE + WRITE_SIZE per launch at the timed plan shape, scaled by a plain copy; "
                            "null once the kernel sources differ from the counted ones",
            "kernel": "sa_plan_kernel, one launch per step (HIP events around the K-launch graph replay)",
            "event_ms_mean": mean_ms,
            "valu_side": valu_side,
        },
    }
    if not args.only_plain:
        sur = None
        if args.regret_per_family > 0:
            sur, line["regret"] = regret_leg(args.regret_per_family)
        if args.corrected_steps > 0:
            line["corrected"] = corrected_leg(arch, var, cfg, n_var, n_evals, sur, args.corrected_steps)
        if args.product_steps > 0:
            line["product"] = product_leg(arch, var, n_var, n_evals, outs, args.product_steps)
        if not args.no_stream_ceiling:
            line["stream_ceiling"] = stream_ceiling(cfg, n_evals, achieved)
        if args.cold_steps > 0:
            line["cold"] = cold_leg(arch, var, cfg, plan, n_var, n_evals, args.cold_steps)
        if args.c2_steps > 0:
            line["c2"] = c2_leg(arch, args.c2_steps)
        if args.c4:
            line["c4"] = c4_leg(arch, sur)
        if args.train_epochs > 0:
            line["training"] = training_leg(args.train_epochs)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(batch, args.cpu_seconds)
    print(json.dumps(line), flush=True)


def counted_shape(path: str):
    """The plan shape the committed counters were taken at, when they match
    the current kernel sources."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_digest") != source_digest() or "shape" not in t:
        return None
    return tuple(int(x) for x in t["shape"])


def counter_record(path: str, shape):
    """A committed counter record, if it was taken on the current kernel
    sources at this plan shape."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_digest") != source_digest() or tuple(t.get("shape", ())) != tuple(shape):
        return None
    return t


def _graph_ms(fn, steps: int) -> float:
    """Mean milliseconds per call of `fn` over `steps` calls captured in one
    HIP graph (after three eager warm-up calls and one untimed replay)."""
    import torch

    for _ in range(3):
        fn(0)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for i in range(steps):
            fn(i)
    graph.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    graph.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def cold_leg(arch, var, cfg, plan, n_var: int, n_evals: int, steps: int, copies: int = 3) -> dict:
    """The headline pass rotating over `copies` copies of the configuration
    columns and of the outputs: each launch reads and writes 393 MB that the
    previous launches did not touch, so the 256 MB last-level cache cannot
    hold them."""
    import torch

    from paper_1701_08547_amd import api

    dev = cfg["seg"].device
    cfgs, outs = [], []
    for _ in range(copies):
        c = {"seg": cfg["seg"]}
        for f in ("block", "unroll", "regs", "grid"):
            c[f] = cfg[f].clone()
        cfgs.append(c)
        outs.append({"occ": torch.empty(n_evals, dtype=torch.int32, device=dev),
                     "score": torch.empty(n_evals, dtype=torch.float32, device=dev),
                     "idx": torch.empty((n_var, K), dtype=torch.int32, device=dev),
                     "val": torch.empty((n_var, K), dtype=torch.float32, device=dev)})
    ws = api.Workspace(plan.workspace_bytes, dev)
    ms = _graph_ms(lambda i: plan.score(arch, var, cfgs[i % copies], outputs=outs[i % copies], workspace=ws), steps)
    gbs = BYTES_PER_EVAL * n_evals / (ms * 1e-3) / 1e9
    # the same rotation for a pure stream of the same bytes (sa_rt_stream, one
    # launch per copy in turn, each timed alone): the cold memory ceiling
    stream_ms = []
    for i in range(3 * copies + 1):
        c = cfgs[i % copies]
        t = api.rt_stream([c["block"], c["unroll"], c["regs"], c["grid"]],
                          [outs[i % copies]["occ"], outs[i % copies]["score"].view(torch.int32)],
                          items=1, blocks_per_cu=0, nontemporal=True, reps=1)
        if i > 0:
            stream_ms.append(t)
    sms = sum(stream_ms) / len(stream_ms)
    sgbs = BYTES_PER_EVAL * n_evals / (sms * 1e-3) / 1e9
    return {"value": n_evals / (ms * 1e-3), "unit": "configs/s", "ms_per_step": ms, "steps": steps,
            "copies": copies, "working_set_bytes": copies * BYTES_PER_EVAL * n_evals, "GBps": gbs,
            "frac_of_hbm_peak": gbs / HBM_PEAK_GBS,
            "stream": {"ms": sms, "GBps": sgbs, "frac_of_hbm_peak": sgbs / HBM_PEAK_GBS, "plain_vs_stream": gbs / sgbs,
                       "kernel": "sa_rt_stream over the same rotation, one launch per copy, each timed alone"}}


def c2_leg(arch, steps: int) -> dict:
    """10,000 variants, search spaces log-uniform in [64, 262,144], top-16
    fused, no per-evaluation outputs: the autotuner picks the plan shape, then
    `steps` launches replay as one graph.  Algorithmic bytes: 16 per
    evaluation read, 44 + 8 k per variant."""
    import torch

    from paper_1701_08547_amd import api, workloads

    t0 = time.perf_counter()
    b = workloads.c2(n_cu=arch["n_cu"])
    var, cfg = api.device_batch(b)
    k = 16
    dev = cfg["seg"].device
    out = {"idx": torch.empty((b.n_var, k), dtype=torch.int32, device=dev),
           "val": torch.empty((b.n_var, k), dtype=torch.float32, device=dev)}
    shape, tune_ms = api.autotune(arch, var, cfg, k=k, reps=5, outputs=out, want_score=False, want_occ=False)
    plan = api.Plan(b.seg, k=k, shape=shape)
    ws = api.Workspace(plan.workspace_bytes, dev)
    ms = _graph_ms(lambda i: plan.score(arch, var, cfg, want_score=False, want_occ=False, outputs=out, workspace=ws),
                   steps)
    nbytes = 16 * b.n_evals + (44 + 8 * k) * b.n_var
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"workload": "10,000 variants, search spaces log-uniform in [64, 262144], top-16, no per-evaluation "
                        "outputs", "n_evals": b.n_evals, "value": b.n_evals / (ms * 1e-3), "unit": "configs/s",
            "ms_per_step": ms, "steps": steps, "plan_shape": list(shape), "autotune_ms": tune_ms,
            "algorithmic_bytes": nbytes, "GBps": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS,
            "seconds": time.perf_counter() - t0}


def c4_leg(arch, sur) -> dict:
    """100,000 variants, spaces log-uniform in [256, 2^20] (1.26e10
    evaluations), rows generated on the device in chunks of whole segments:
    one pass of generation alone, one of generation + plain top-16 and one of
    generation + corrected top-16; the plain and corrected figures subtract
    the generation time."""
    import numpy as np
    import torch

    from paper_1701_08547_amd import api, streamed, workloads

    t0 = time.perf_counter()
    if sur is None:
        from paper_1701_08547_amd import correction

        sur = api.Surrogate(correction.init_params(0), np.zeros(24, np.float32), np.ones(24, np.float32))
    batch = workloads.c4(n_cu=arch["n_cu"])
    st = streamed.Streamed(batch, arch, k=16, chunk_evals=1 << 28, surrogate=sur, device="cuda:0")
    stream = torch.cuda.current_stream()

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    st.run(plain=True, corrected=False)  # warm-up: first launches of every chunk's plan
    t_gen = timed(lambda: [st.generate(i) for i in range(len(st.chunks))])
    t_plain = timed(lambda: st.run(plain=True, corrected=False)) - t_gen
    t_corr = timed(lambda: st.run(plain=False, corrected=True)) - t_gen
    n = batch.n_evals
    return {"workload": "100,000 variants, spaces log-uniform in [256, 1048576], rows generated on the device",
            "n_evals": n, "chunks": len(st.chunks), "k": 16, "generate_ms": t_gen,
            "plain": {"ms": t_plain, "value": n / (t_plain * 1e-3), "unit": "configs/s",
                      "read_GBps": 16 * n / (t_plain * 1e-3) / 1e9,
                      "frac_of_hbm_peak": 16 * n / (t_plain * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "corrected": {"ms": t_corr, "value": n / (t_corr * 1e-3), "unit": "configs/s",
                          "TFLOPs": MLP_FLOP_PER_EVAL * n / (t_corr * 1e-3) / 1e12,
                          "frac_of_bf16_peak": MLP_FLOP_PER_EVAL * n / (t_corr * 1e-3) / 1e12 / MFMA_BF16_PEAK_TFLOPS},
            "seconds": time.perf_counter() - t0}


def training_leg(epochs: int, n: int = 2_000_000, batch: int = 4096) -> dict:
    """Training steps of the learned correction as the training loop runs
    them on a training set of the measured dataset's size: 2,000,000
    synthetic rows (24 N(0, 1) features, N(0, 0.01) targets), batches of
    4,096, each epoch's 488 steps (one fused forward/backward kernel and one
    Adam kernel each) captured in one HIP graph; the timed region is `epochs`
    replays between HIP events on the replay stream."""
    import numpy as np
    import torch

    from paper_1701_08547_amd import api, correction

    g = torch.Generator(device="cuda")
    g.manual_seed(170108547)
    feat = torch.randn((n, 24), generator=g, device="cuda")
    target = torch.randn(n, generator=g, device="cuda") * 0.1
    sur = api.Surrogate(correction.init_params(0), np.zeros(24, np.float32), np.ones(24, np.float32))
    sur.reserve(batch)
    starts = list(range(0, n - batch + 1, batch))
    sur.steps_dev.fill_(0)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        for b0 in starts:
            sur.train_step(feat[b0:b0 + batch], target[b0:b0 + batch], lr=1e-3, device_counter=True)
    torch.cuda.current_stream().wait_stream(side)
    graph.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(epochs):
        graph.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    steps = epochs * len(starts)
    ms = e0.elapsed_time(e1) / steps
    tflops = TRAIN_FLOP_PER_ROW * batch / (ms * 1e-3) / 1e12
    loss = float(sur.grad[api.MLP_PARAMS].item())
    return {"us_per_step": ms * 1e3, "rows_per_step": batch, "steps": steps, "rows": n,
            "epoch_ms": ms * len(starts), "rows_per_s": batch / (ms * 1e-3),
            "kernels": "sa_train_kernel + sa_train_adam_kernel per step, one graph per epoch",
            "flop_per_row": TRAIN_FLOP_PER_ROW, "TFLOPs": tflops, "frac_of_bf16_peak": tflops / MFMA_BF16_PEAK_TFLOPS,
            "last_loss": loss, "device_steps": int(sur.steps_dev.item())}


def stream_ceiling(cfg, n_evals: int, achieved: float) -> dict:
    """A pure stream of the plain pass's traffic (the four configuration
    columns read, two 4-byte columns written, no model arithmetic) over a
    sweep of launch shapes: the fastest is the practical memory ceiling the
    plain pass is set against."""
    import torch

    from paper_1701_08547_amd import api

    cols = [cfg[c] for c in ("block", "unroll", "regs", "grid")]
    outs = [torch.empty(n_evals, dtype=torch.int32, device=cols[0].device) for _ in range(2)]
    best = None
    for nt in (False, True):
        for items in (1, 2, 4):
            for bpc in (0, 4, 8, 16, 32):
                ms = api.rt_stream(cols, outs, items=items, blocks_per_cu=bpc, nontemporal=nt, reps=20)
                if best is None or ms < best[0]:
                    best = (ms, items, bpc, nt)
    torch.cuda.synchronize()
    gbs = BYTES_PER_EVAL * n_evals / (best[0] * 1e-3) / 1e9
    return {"GBps": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS, "ms": best[0],
            "shape": {"items_per_lane": best[1], "blocks_per_cu": best[2], "nontemporal_stores": best[3]},
            "plain_vs_stream": achieved / gbs,
            "kernel": "sa_rt_stream: 16 B read + 8 B written per element, %d elements, mean of 20 back-to-back launches" % n_evals}


def product_leg(arch, var, n_var, n_evals, outs, steps: int) -> dict:
    """The same workload as a product space (every variant scores the same
    16 x 8 x 32 x 4 product, which is how the rows above are laid out): no
    configuration rows are read, occupancy + score written and top-8 as in
    the timed pass."""
    import numpy as np
    import torch

    from paper_1701_08547_amd import api, workloads

    space = {"block": workloads.BLOCK_VALUES, "unroll": workloads.UNROLL_VALUES, "regs": workloads.REG_VALUES,
             "grid": (workloads.GRID_MULTIPLIERS * arch["n_cu"]).astype(np.int32)}
    S = api.product_size(space)
    assert n_var * S == n_evals
    ws = api.Workspace(int(api.lib().sa_product_workspace_bytes(n_var, S, K)), outs["occ"].device)

    def step():
        api.score_product(arch, var, space, k=K, outputs=outs, workspace=ws)

    for _ in range(3):
        step()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(steps):
            step()
    graph.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    graph.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    return {"value": n_evals / (ms * 1e-3), "unit": "configs/s", "ms_per_step": ms, "steps": steps,
            "kernels": "sa_seg_fill_kernel + sa_product_kernel + sa_merge_kernel",
            "bytes_per_eval": 8, "GBps": 8 * n_evals / (ms * 1e-3) / 1e9,
            "note": "no configuration rows read: values from the local index; 8 B per evaluation written"}


def regret_leg(per_family: int):
    """Top-1 regret against measured runtimes: a small measured dataset of the
    library's kernel families (the paper's timing protocol), the correction
    trained on three quarters of each family's instances and evaluated on the
    rest; two ablations on the same split (the network's ranking alone, with
    and without the features computed from the static model's terms); the
    same with each family left out of training entirely; and the
    model-guided search run live on the held-out instances (the full sweep and
    the 8 survivors of each key timed again, wall clock compared)."""
    from paper_1701_08547_amd import correction, runtime_dataset

    t0 = time.perf_counter()
    data = runtime_dataset.build(per_family, seed=7)
    sur, rep = correction.run(data, epochs=150, seed=7, held_frac=0.25)
    a = rep["all"]
    out = {"instances": int(data["instance"].max()) + 1, "held_out": a["instances"],
           "regret_plain": a["regret_plain"], "regret_corrected": a["regret_corrected"],
           "regret_diff_ci": a["regret_diff_ci"],
           "spearman_plain": a["spearman_plain"], "spearman_corrected": a["spearman_corrected"],
           "paper_pruned_fraction": a.get("pruned_fraction"),
           "regret_paper_pruned_plain": a.get("regret_pruned_plain"),
           "regret_paper_pruned_best": a.get("regret_pruned_best")}
    # does the static model carry the corrected key?  The same split, the
    # network ranking alone (trained on the centred log runtime), with and
    # without the features computed from the model's terms
    out["ablation"] = {}
    for name, kw in (("network_alone", {"key": "direct"}),
                     ("network_alone_without_model_features", {"key": "direct",
                                                               "drop": correction.MODEL_FEATURES})):
        _, ra = correction.run(data, epochs=150, seed=7, held_frac=0.25, **kw)
        out["ablation"][name] = {"regret": ra["all"]["regret_corrected"],
                                 "regret_ci": ra["all"]["regret_corrected_ci"],
                                 "spearman": ra["all"]["spearman_corrected"]}
    out["leave_one_family_out"] = correction.leave_one_family_out(data, epochs=150, seed=7)
    out["live_search_k8"] = correction.live_search(data, rep["keys"], k=8)
    out["seconds"] = time.perf_counter() - t0
    return sur, out


def corrected_leg(arch, var, cfg, n_var, n_evals, sur, steps: int) -> dict:
    """The fused corrected pass (occupancy, score, features, MLP, top-8 on
    ln score + Delta) on the same workload: configurations per second and
    its dense-contraction rate against the bf16 MFMA peak."""
    import numpy as np
    import torch

    from paper_1701_08547_amd import api

    dev = cfg["seg"].device
    if sur is None:
        from paper_1701_08547_amd import correction

        sur = api.Surrogate(correction.init_params(0), np.zeros(24, np.float32), np.ones(24, np.float32), dev)
    outs = {"occ": torch.empty(n_evals, dtype=torch.int32, device=dev),
            "score": torch.empty(n_evals, dtype=torch.float32, device=dev),
            "idx": torch.empty((n_var, K), dtype=torch.int32, device=dev),
            "val": torch.empty((n_var, K), dtype=torch.float32, device=dev)}
    ws = api.Workspace(api.workspace_bytes(n_var, n_evals, K), dev)

    def step():
        api.score(arch, var, cfg, k=K, outputs=outs, workspace=ws, mlp=sur)

    step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    tflops = MLP_FLOP_PER_EVAL * n_evals / (ms * 1e-3) / 1e12
    return {"value": n_evals / (ms * 1e-3), "unit": "configs/s", "ms_per_step": ms, "steps": steps,
            "kernels": "sa_corrected_kernel + sa_merge_kernel",
            "roofline": {"bound": "mfma", "achieved": tflops, "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": tflops / MFMA_BF16_PEAK_TFLOPS, "traffic": None,
                         "note": "39,168 algorithmic FLOP per evaluation (24->128->128->1; the padding of the inputs "
                                 "to 32 is not counted); "
                                 "bound by LDS reads first (the GELU table and the weight tiles, about 245 KiB per 64 evaluations), vector issue second; the matrix cores are about a third busy (SQ counters)"}}


if __name__ == "__main__":
    main()
