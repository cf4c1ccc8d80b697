"""GPU parity of planned batches (persistent kernel over workgroup items,
split-segment merge, graph capture, autotuner) against the CPU oracle."""
import sys

import numpy as np
import pytest

import oracle
from paper_1701_08547_amd import api, workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)


def say(*a):
    print("[gpu-plan]", *a, flush=True)
    sys.stdout.flush()


def check(ref, got, rows=None):
    if got.get("occ") is not None:
        assert np.array_equal(ref["occ"], got["occ"])
    if got.get("score") is not None:
        assert np.array_equal(ref["score32"].view(np.uint32), got["score"].view(np.uint32))
    ridx, rval = ref["idx"], ref["val"]
    gidx, gval = got["idx"], got["val"]
    if rows is not None:
        gidx, gval = gidx[rows], gval[rows]
    assert np.array_equal(ridx, gidx), np.flatnonzero((ridx != gidx).any(1))[:10]
    assert np.array_equal(rval.view(np.uint32), gval.view(np.uint32))


def run_plan(batch, k, shape, arch=None, **kw):
    a = arch or oracle.arch_cdna4()
    var, cfg = api.device_batch(batch)
    plan = api.Plan(batch.seg, k=k, shape=shape)
    say("plan", batch.name, "shape", plan.shape, "items", plan.n_items, "splits", plan.n_splits)
    out = plan.score(a, var, cfg, **kw)
    torch.cuda.synchronize()
    return {key: (None if t is None else t.cpu().numpy()) for key, t in out.items()}


SIZES = [0, 1, 5, 63, 64, 65, 255, 256, 257, 1000, 4095, 4096, 4097, 10000, 0, 3, 20000, 1, 70000, 0]


@pytest.mark.parametrize("items", [1, 2, 4])
@pytest.mark.parametrize("wpb", [4, 8, 16])
def test_plan_shapes_ragged(items, wpb):
    b = workloads.custom_batch(40 + items * wpb, SIZES, with_grid=True, name="plan-ragged")
    ref = oracle.run(oracle.arch_cdna4(), b.variants, b.configs(), k=8)
    check(ref, run_plan(b, 8, (1024, items, wpb)))


@pytest.mark.parametrize("tile", [256, 2048, 8192])
def test_plan_tiles_and_no_grid(tile):
    b = workloads.custom_batch(50 + tile, SIZES, with_grid=False, name="plan-nogrid")
    ref = oracle.run(oracle.arch_cdna4(), b.variants, b.configs(), k=16)
    check(ref, run_plan(b, 16, (tile, 4, 4)))


@pytest.mark.parametrize("shape", [(1024, 2, 4), (256, 4, 16)])
def test_plan_unaligned_columns(shape):
    """Columns at an odd offset (not 16-byte aligned) send the planned pass
    down its masked path, where a split item's 256-row blocks are dealt to
    its waves in turn (some waves get none): results equal the oracle's."""
    b = workloads.custom_batch(14, [700, 5000, 33, 20000, 300], with_grid=True, name="plan-unaligned")
    a = oracle.arch_cdna4()
    ref = oracle.run(a, b.variants, b.configs(), k=8)
    var, cfg = api.device_batch(b)
    for key in ("block", "unroll", "regs", "grid"):
        big = torch.empty(cfg[key].numel() + 1, dtype=torch.int32, device=cfg[key].device)
        big[1:] = cfg[key]
        cfg[key] = big[1:]
    plan = api.Plan(b.seg, k=8, shape=shape)
    say("plan unaligned", shape, "items", plan.n_items, "splits", plan.n_splits)
    out = plan.score(a, var, cfg)
    torch.cuda.synchronize()
    check(ref, {key: t.cpu().numpy() for key, t in out.items()})


def test_plan_optional_outputs_and_occupancy_only():
    b = workloads.custom_batch(61, SIZES, with_grid=True, name="plan-outputs")
    ref = oracle.run(oracle.arch_cdna4(), b.variants, b.configs(), k=8)
    got = run_plan(b, 8, (1024, 4, 8), want_score=False, want_occ=False)
    assert np.array_equal(ref["idx"], got["idx"])
    got = run_plan(b, 8, (1024, 4, 8), want_topk=False)
    assert np.array_equal(ref["occ"], got["occ"])
    assert np.array_equal(ref["score32"].view(np.uint32), got["score"].view(np.uint32))


def test_plan_topk_keys():
    g = np.random.default_rng(23)
    sizes = np.array(SIZES + [50000], np.int64)
    seg = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(seg[-1])
    keys = (g.standard_normal(n) * 10).astype(np.float32)
    keys[g.random(n) < 0.05] = np.inf
    keys[g.random(n) < 0.02] = np.nan
    keys[g.random(n) < 0.2] = np.float32(0.5)
    ridx, rval = oracle.topk(keys, seg, 8)
    plan = api.Plan(seg, k=8, shape=(1024, 2, 4))
    idx, val = plan.topk(torch.from_numpy(keys).cuda(), torch.from_numpy(seg).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(ridx, idx.cpu().numpy())
    assert np.array_equal(rval.view(np.uint32), val.cpu().numpy().view(np.uint32))


def test_plan_c1_full():
    b = workloads.c1()
    ref = oracle.run(oracle.arch_cdna4(), b.variants, b.configs(), k=8)
    check(ref, run_plan(b, 8, (4096, 4, 4)))


def test_plan_graph_capture_replays():
    """sa_plan_score captured in a HIP graph: every replay equals the eager
    result (eager work and synchronisation between replays)."""
    b = workloads.custom_batch(71, SIZES, with_grid=True, name="plan-graph")
    a = oracle.arch_cdna4()
    var, cfg = api.device_batch(b)
    plan = api.Plan(b.seg, k=8, shape=(1024, 4, 4))
    ws = api.Workspace(plan.workspace_bytes, "cuda")
    eager = plan.score(a, var, cfg, workspace=ws)
    torch.cuda.synchronize()
    eager = {k: v.clone() for k, v in eager.items()}
    outs = {k: torch.empty_like(v) for k, v in eager.items()}
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.score(a, var, cfg, outputs=outs, workspace=ws)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.score(a, var, cfg, outputs=outs, workspace=ws)
    for r in range(3):
        for t in outs.values():
            t.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for key in eager:
            assert torch.equal(eager[key].view(torch.int32), outs[key].view(torch.int32)), (r, key)


def test_plan_item_queue_across_launches_and_replays():
    """A plan with far more workgroup items than resident workgroups takes
    its items from the ticket queue in its table.  The queue must be back at
    zero after every launch whatever kernel took it: the scoring pass, the
    top-k pass over keys (another kernel, another grid) and replays of a
    captured graph, interleaved, each equal to the oracle."""
    g = np.random.default_rng(5)
    sizes = g.integers(1, 400, 40000)
    sizes[::97] = g.integers(2000, 9000, sizes[::97].size)  # some segments cut into several items
    b = workloads.custom_batch(91, sizes, with_grid=True, name="plan-queue")
    a = oracle.arch_cdna4()
    var, cfg = api.device_batch(b)
    plan = api.Plan(b.seg, k=8, shape=(256, 1, 4))
    say("queue plan items", plan.n_items, "splits", plan.n_splits, "evaluations", b.n_evals)
    assert plan.n_items > 8 * 256  # more than any grid of this shape resides
    ref = oracle.run(a, b.variants, b.configs(), k=8, want_occ=True, want_f32=True, want_f64=False)
    ws = api.Workspace(plan.workspace_bytes, "cuda")
    outs = {"occ": torch.empty(b.n_evals, dtype=torch.int32, device="cuda"),
            "score": torch.empty(b.n_evals, dtype=torch.float32, device="cuda"),
            "idx": torch.empty((b.n_var, 8), dtype=torch.int32, device="cuda"),
            "val": torch.empty((b.n_var, 8), dtype=torch.float32, device="cuda")}

    def host(o):
        return {key: t.cpu().numpy() for key, t in o.items()}

    for r in range(2):
        plan.score(a, var, cfg, outputs=outs, workspace=ws)
        torch.cuda.synchronize()
        check(ref, host(outs))
        idx, val = plan.topk(outs["score"], cfg["seg"], workspace=ws)
        torch.cuda.synchronize()
        check({"idx": ref["idx"], "val": ref["val"]}, {"idx": idx.cpu().numpy(), "val": val.cpu().numpy()})
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.score(a, var, cfg, outputs=outs, workspace=ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.score(a, var, cfg, outputs=outs, workspace=ws)
    for r in range(3):
        for t in outs.values():
            t.fill_(-7)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        check(ref, host(outs))
        idx, val = plan.topk(outs["score"], cfg["seg"], workspace=ws)  # eager, between replays
        torch.cuda.synchronize()
        assert np.array_equal(idx.cpu().numpy(), ref["idx"])


def test_autotuner_picks_a_valid_shape():
    b = workloads.custom_batch(81, [5000, 64, 300000, 7, 20000, 0], with_grid=True, name="plan-tune")
    a = oracle.arch_cdna4()
    var, cfg = api.device_batch(b)
    shape, ms = api.autotune(a, var, cfg, k=8, reps=2)
    say("autotuned", shape, ms)
    assert shape[0] in (1024, 2048, 4096, 8192) and shape[1] in (1, 2, 4) and shape[2] in (4, 8, 16)
    assert 0 < ms < 1000
    ref = oracle.run(a, b.variants, b.configs(), k=8)
    check(ref, run_plan(b, 8, shape))


def test_plan_c2_full():
    """10,000 variants with log-uniform search spaces in [64, 262,144]
    (315,504,608 evaluations), top-16, one planned launch at the shape the
    autotuner picks for it, compared in full with the oracle: occupancy and
    binary32 score bits of every evaluation, top-16 indices and values of
    every variant."""
    b = workloads.c2()
    say("c2 evaluations", b.n_evals)
    a = oracle.arch_cdna4()
    var, cfg = api.device_batch(b)
    out_t = {"idx": torch.empty((b.n_var, 16), dtype=torch.int32, device="cuda"),
             "val": torch.empty((b.n_var, 16), dtype=torch.float32, device="cuda")}
    shape, _ = api.autotune(a, var, cfg, k=16, reps=2, outputs=out_t, want_score=False, want_occ=False)
    say("c2 autotuned shape", shape)
    for sh in (shape, (4096, 4, 4)) if tuple(shape) != (4096, 4, 4) else (shape,):
        plan = api.Plan(b.seg, k=16, shape=sh)
        out = plan.score(a, var, cfg)
        torch.cuda.synchronize()
        got = {key: t.cpu().numpy() for key, t in out.items()}
        del out, plan
        ref = oracle.run(a, b.variants, b.configs(), k=16, want_occ=True, want_f32=True, want_f64=False)
        check(ref, got)
        del ref, got
    del var, cfg
    torch.cuda.empty_cache()


def test_plan_c1_every_autotuner_shape():
    """The benchmark workload (1,000 variants x 16,384 configurations, top-8,
    the device's own descriptor) compared in full with the oracle at each of
    the 36 shapes the autotuner chooses from and at the one it picks here:
    whichever launch configuration bench.py ends up timing is covered."""
    a = api.arch_default(0)
    b = workloads.c1(n_cu=a["n_cu"])
    ref = oracle.run(a, b.variants, b.configs(), k=8)
    var, cfg = api.device_batch(b)
    picked, _ = api.autotune(a, var, cfg, k=8, reps=2)
    shapes = [(t, i, w) for t in (1024, 2048, 4096, 8192) for i in (1, 2, 4) for w in (4, 8, 16)]
    assert tuple(picked) in shapes
    for shape in shapes + [tuple(picked)]:
        say("c1 shape", shape)
        plan = api.Plan(b.seg, k=8, shape=shape)
        ws = api.Workspace(plan.workspace_bytes, "cuda")
        o = plan.score(a, var, cfg, workspace=ws)
        torch.cuda.synchronize()
        check(ref, {key: t.cpu().numpy() for key, t in o.items()})
        del o, ws, plan
    torch.cuda.empty_cache()


@pytest.mark.parametrize("k,shape", [(1, (1024, 1, 4)), (33, (2048, 2, 8)), (64, (1024, 4, 16)), (64, (8192, 1, 4))])
def test_plan_k_extremes(k, shape):
    """k from 1 to the maximum on ragged segments (empty ones, and ones split
    over several workgroup items): with 16 waves and k = 64 a workgroup's
    merge runs 1,024 keys through the selection buffer."""
    b = workloads.custom_batch(90 + k, SIZES, with_grid=True, name="plan-k")
    ref = oracle.run(oracle.arch_cdna4(), b.variants, b.configs(), k=k)
    check(ref, run_plan(b, k, shape))
