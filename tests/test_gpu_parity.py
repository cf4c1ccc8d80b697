"""GPU parity: the gfx950 library (through its C ABI) against the CPU oracle
on the same seeded inputs.

Bar: occupancy, top-k indices and selected values bit-exact; binary32 scores
bit-identical to the oracle's binary32 sequence and within 1e-5 relative of
its binary64 reference.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1701_08547_amd import api, workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

REL_TOL = 1e-5


def say(*a):
    print("[gpu-parity]", *a, flush=True)
    sys.stdout.flush()


def gpu_run(arch, batch, k, *, tile=None, want_score=True, want_occ=True, want_topk=True):
    var, cfg = api.device_batch(batch)
    if tile:
        api.set_tile(tile)
    try:
        out = api.score(arch, var, cfg, k=k, want_score=want_score, want_occ=want_occ, want_topk=want_topk)
        torch.cuda.synchronize()
    finally:
        api.set_tile(0)
    return {key: (None if t is None else t.cpu().numpy()) for key, t in out.items()}


def assert_parity(ref, got, k_checked=True, score_checked=True, occ_checked=True):
    if occ_checked:
        assert np.array_equal(ref["occ"], got["occ"]), "occupancy differs at %s" % np.flatnonzero(ref["occ"] != got["occ"])[:10]
    if score_checked:
        s32, g = ref["score32"], got["score"]
        bad = np.flatnonzero(s32.view(np.uint32) != g.view(np.uint32))
        assert bad.size == 0, "binary32 scores differ at %s: %s vs %s" % (bad[:5], s32[bad[:5]], g[bad[:5]])
        fin = np.isfinite(ref["score64"])
        assert np.array_equal(fin, np.isfinite(g))
        rel = np.abs(g[fin].astype(np.float64) - ref["score64"][fin]) / np.maximum(np.abs(ref["score64"][fin]), 1e-300)
        assert rel.size == 0 or rel.max() <= REL_TOL, rel.max()
    if k_checked:
        assert np.array_equal(ref["idx"], got["idx"]), "top-k indices differ in rows %s" % np.flatnonzero((ref["idx"] != got["idx"]).any(1))[:10]
        assert np.array_equal(ref["val"].view(np.uint32), got["val"].view(np.uint32))


def both(batch, k, arch=None, tile=None, **kw):
    a = arch or oracle.arch_cdna4()
    say("case", batch.name, "n_var", batch.n_var, "n_evals", batch.n_evals, "k", k, "tile", tile)
    ref = oracle.run(a, batch.variants, batch.configs(), k=k)
    got = gpu_run(a, batch, k, tile=tile, **kw)
    return ref, got


def test_device_descriptor():
    a = api.arch_default(0)
    say("device descriptor", a)
    api.arch_validate(a)
    assert a["wave_size"] == 64
    assert a["n_cu"] > 0


def test_c0_full():
    ref, got = both(workloads.c0(), 8)
    assert_parity(ref, got)


RAGGED = [0, 1, 5, 63, 64, 65, 255, 256, 257, 1000, 4095, 4096, 4097, 10000, 0, 3, 20000, 1]


@pytest.mark.parametrize("tile", [1024, 2048, 4096])
@pytest.mark.parametrize("grid", [True, False])
def test_ragged_segments_span_tiles(tile, grid):
    b = workloads.custom_batch(11 + tile, RAGGED, with_grid=grid, name="ragged")
    ref, got = both(b, 8, tile=tile)
    assert_parity(ref, got)


@pytest.mark.parametrize("k", [1, 2, 16, 63, 64])
def test_k_range(k):
    b = workloads.custom_batch(20 + k, [3, 64, 130, 5000, 9000], with_grid=True, name="krange")
    ref, got = both(b, k, tile=1024)
    assert_parity(ref, got)


def test_edge_values_corpus():
    """Illegal and boundary configurations and variants: occupancy 0 and
    score +inf exactly where the oracle says, never selected."""
    sets = dict(block=[-5, 0, 1, 63, 64, 65, 100, 192, 1024, 1025, 1 << 20],
                unroll=[-1, 0, 1, 3, 8, 64, 65],
                regs=[-1, 0, 1, 8, 9, 20, 64, 65, 96, 168, 256, 512, 513],
                grid=[-1, 0, 1, 255, 256, 1000, 2048, 262144, 262145])
    b = workloads.custom_batch(5, [50, 700, 3000, 64, 1, 2500, 900, 4100], with_grid=True, value_sets=sets,
                               name="edges")
    v = b.variants
    v["lds"][:] = np.array([0, 1, 511, 512, 513, 5376, 163840, 163841], np.int32)
    v["n_fp"][1] = -1          # invalid count
    v["n_bar"][2] = (1 << 14) + 1
    v["div"][3] = np.float32(np.nan)
    v["div"][4] = np.float32(1.0)
    v["n_reg"][5] = 100
    v["n_ld"][6] = (1 << 24) - 1
    ref, got = both(b, 16, tile=1024)
    assert_parity(ref, got)
    assert (ref["occ"] == 0).any() and (ref["occ"] > 0).any()


def test_ties_break_to_lower_index():
    sets = dict(block=[256], unroll=[4], regs=[64], grid=[512])
    b = workloads.custom_batch(7, [10, 300, 5000, 2], with_grid=True, value_sets=sets, name="ties")
    ref, got = both(b, 8, tile=1024)
    assert_parity(ref, got)
    assert got["idx"][2].tolist() == list(range(8))


def test_occupancy_entry_point():
    b = workloads.custom_batch(3, RAGGED, with_grid=True, name="occ")
    a = oracle.arch_cdna4()
    say("case sa_occupancy", b.n_evals)
    ref = oracle.run(a, b.variants, b.configs(), k=0, want_f32=False, want_f64=False)
    var, cfg = api.device_batch(b)
    occ = api.occupancy(a, var, cfg)
    torch.cuda.synchronize()
    assert np.array_equal(ref["occ"], occ.cpu().numpy())


def test_outputs_optional():
    b = workloads.custom_batch(4, [100, 5000, 7], with_grid=False, name="optional")
    a = oracle.arch_cdna4()
    ref = oracle.run(a, b.variants, b.configs(), k=8)
    got = gpu_run(a, b, 8, want_score=False, want_occ=False)
    assert np.array_equal(ref["idx"], got["idx"])
    got = gpu_run(a, b, 8, want_topk=False)
    assert_parity(ref, got, k_checked=False)


@pytest.mark.parametrize("gpu", ["fermi", "kepler", "maxwell", "pascal"])
def test_paper_descriptors(gpu):
    """The same kernels under the paper's NVIDIA descriptors (warp 32, one
    register pool, no allocation rounding)."""
    sets = dict(block=list(range(32, 1025, 32)) + [1, 31, 1025], regs=[0, 8, 16, 20, 21, 22, 31, 32, 33, 63, 64,
                                                                        128, 255, 256],
                grid=[14, 13, 24, 56, 100, 1000])
    b = workloads.custom_batch(30, [4000, 3000, 5], with_grid=True, value_sets=sets, name="paper-" + gpu)
    b.variants["lds"][:] = np.array([0, 3072, 8192], np.int32)
    ref, got = both(b, 8, arch=oracle.arch_paper(gpu), tile=1024)
    assert_parity(ref, got)


def test_topk_entry_point_keys():
    g = np.random.default_rng(17)
    sizes = np.array(RAGGED + [30000, 2], np.int64)
    seg = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(seg[-1])
    keys = (g.standard_normal(n) * 100).astype(np.float32)
    keys[g.random(n) < 0.05] = np.inf
    keys[g.random(n) < 0.02] = -np.inf
    keys[g.random(n) < 0.02] = np.nan
    keys[g.random(n) < 0.3] = np.float32(1.5)  # ties
    keys[g.random(n) < 0.05] = np.float32(-0.0)  # signed zeros tie with +0
    keys[g.random(n) < 0.05] = np.float32(0.0)
    for k in (1, 8, 33):
        say("case sa_topk", n, "k", k)
        ridx, rval = oracle.topk(keys, seg, k)
        api.set_tile(1024)
        try:
            idx, val = api.topk(torch.from_numpy(keys).cuda(), torch.from_numpy(seg).cuda(), k)
            torch.cuda.synchronize()
        finally:
            api.set_tile(0)
        assert np.array_equal(ridx, idx.cpu().numpy())
        assert np.array_equal(rval.view(np.uint32), val.cpu().numpy().view(np.uint32))


def test_unaligned_columns_take_the_masked_path():
    """Columns that are not 16-byte aligned (views at an odd offset) give the
    same results through the scalar path."""
    b = workloads.custom_batch(12, [700, 5000, 33], with_grid=True, name="unaligned")
    a = oracle.arch_cdna4()
    ref = oracle.run(a, b.variants, b.configs(), k=8)
    var, cfg = api.device_batch(b)
    for key in ("block", "unroll", "regs", "grid"):
        big = torch.empty(cfg[key].numel() + 1, dtype=torch.int32, device=cfg[key].device)
        big[1:] = cfg[key]
        cfg[key] = big[1:]
    say("case unaligned", b.n_evals)
    out = api.score(a, var, cfg, k=8)
    torch.cuda.synchronize()
    got = {key: t.cpu().numpy() for key, t in out.items()}
    assert_parity(ref, got)


def test_empty_batches():
    a = oracle.arch_cdna4()
    b = workloads.custom_batch(1, [0, 0, 0], with_grid=True, name="empty")
    ref, got = both(b, 4)
    assert (got["idx"] == -1).all() and np.isinf(got["val"]).all()


def test_determinism():
    b = workloads.custom_batch(9, [70000, 3, 12345], with_grid=True, name="determinism")
    a = oracle.arch_cdna4()
    r1 = gpu_run(a, b, 16)
    r2 = gpu_run(a, b, 16)
    for key in ("occ", "score", "idx", "val"):
        assert r1[key].tobytes() == r2[key].tobytes()


def test_c1_full_size_bench_configuration():
    """The benchmark workload (1,000 variants x 16,384 configurations, top-8)
    in the launch configuration the benchmark times, compared in full."""
    b = workloads.c1()
    ref, got = both(b, 8)
    assert_parity(ref, got)
