"""GPU parity of product-space scoring (sa_score_product): the same
occupancy, scores and top-k as sa_score on the materialised rows, bit for
bit, and as the oracle on small spaces."""
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
    print("[gpu-product]", *a, flush=True)
    sys.stdout.flush()


def materialise(space: dict, n_var: int):
    """Rows of the product (block slowest, grid fastest), repeated per variant."""
    dims = [d for d in api.PRODUCT_DIMS if space.get(d) is not None]
    grids = np.meshgrid(*[np.asarray(space[d], np.int32) for d in dims], indexing="ij")
    cols = {d: np.tile(g.reshape(-1), n_var).astype(np.int32) for d, g in zip(dims, grids)}
    S = api.product_size(space)
    seg = (np.arange(n_var + 1, dtype=np.int64) * S)
    return seg, cols


def run_both(arch, v, space, k):
    n_var = int(v["n_fp"].shape[0])
    seg, cols = materialise(space, n_var)
    b = workloads.Batch(v, seg, cols["block"], cols["unroll"], cols["regs"], cols.get("grid"), "product")
    var, cfg = api.device_batch(b)
    ref = api.score(arch, var, cfg, k=k)
    got = api.score_product(arch, var, space, k=k)
    torch.cuda.synchronize()
    return b, ref, got


def assert_same(ref, got):
    for key in ("occ", "idx"):
        assert np.array_equal(ref[key].cpu().numpy(), got[key].cpu().numpy()), key
    for key in ("score", "val"):
        assert np.array_equal(ref[key].cpu().numpy().view(np.uint32), got[key].cpu().numpy().view(np.uint32)), key


SPACE_GRID = {"block": [64, 96, 128, 192, 256, 512, 1024, 1100, 0], "unroll": [1, 2, 5],
              "regs": [0, 16, 24, 64, 128, 256, 512, 513], "grid": [256, 300, 1024, 0]}
SPACE_NOGRID = {"block": list(range(32, 1025, 32)), "unroll": [1, 2, 3, 4, 5], "regs": [16, 32, 48, 200]}


@pytest.mark.parametrize("k", [1, 8, 16])
def test_product_matches_materialised_with_grid(k):
    arch = oracle.arch_cdna4()
    v = workloads.variant_features(37, 901)
    b, ref, got = run_both(arch, v, SPACE_GRID, k)
    say("grid space", api.product_size(SPACE_GRID), "evaluations", b.n_evals)
    assert_same(ref, got)


def test_product_matches_oracle_no_grid():
    arch = oracle.arch_cdna4()
    v = workloads.variant_features(9, 902)
    b, ref, got = run_both(arch, v, SPACE_NOGRID, 8)
    assert_same(ref, got)
    o = oracle.run(arch, b.variants, b.configs(), k=8, want_f64=False)
    assert np.array_equal(o["occ"], got["occ"].cpu().numpy())
    assert np.array_equal(o["score32"].view(np.uint32), got["score"].cpu().numpy().view(np.uint32))
    assert np.array_equal(o["idx"], got["idx"].cpu().numpy())


def test_product_single_values_and_spans():
    """Lists of one value (no division), and spaces whose segments straddle
    wave-tiles at odd offsets."""
    arch = oracle.arch_cdna4()
    v = workloads.variant_features(23, 903)
    assert_same(*run_both(arch, v, {"block": [256], "unroll": [4], "regs": [64]}, 4)[1:])
    odd = {"block": [64, 128, 256], "unroll": [1, 2, 3, 4, 5], "regs": list(range(8, 520, 8))[:7],
           "grid": list(range(256, 256 * 12, 256))}
    assert api.product_size(odd) == 1155
    assert_same(*run_both(arch, v, odd, 8)[1:])


def test_product_outputs_optional():
    arch = oracle.arch_cdna4()
    v = workloads.variant_features(5, 904)
    var = api.device_batch(workloads.Batch(v, np.zeros(6, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32),
                                           np.zeros(0, np.int32), None, "p"))[0]
    full = api.score_product(arch, var, SPACE_GRID, k=8)
    only_k = api.score_product(arch, var, SPACE_GRID, k=8, want_score=False, want_occ=False)
    only_occ = api.score_product(arch, var, SPACE_GRID, want_score=False, want_topk=False)
    torch.cuda.synchronize()
    assert np.array_equal(full["idx"].cpu().numpy(), only_k["idx"].cpu().numpy())
    assert np.array_equal(full["occ"].cpu().numpy(), only_occ["occ"].cpu().numpy())


def test_product_full_size_benchmark_space():
    """1,000 variants over the benchmark's 16 x 8 x 32 x 4 product: every
    output equal to the planned pass over the materialised rows."""
    arch = api.arch_default(0)
    b = workloads.c1(n_cu=arch["n_cu"])
    space = {"block": workloads.BLOCK_VALUES, "unroll": workloads.UNROLL_VALUES, "regs": workloads.REG_VALUES,
             "grid": (workloads.GRID_MULTIPLIERS * arch["n_cu"]).astype(np.int32)}
    assert api.product_size(space) == 16384
    seg, cols = materialise(space, b.n_var)
    assert np.array_equal(seg, b.seg)
    for d in api.PRODUCT_DIMS:
        assert np.array_equal(cols[d], getattr(b, d)), d   # the benchmark batch is this product
    var, cfg = api.device_batch(b)
    plan = api.Plan(b.seg, k=8)
    ref = plan.score(arch, var, cfg)
    got = api.score_product(arch, var, space, k=8)
    torch.cuda.synchronize()
    assert_same(ref, got)
    del var, cfg, ref, got
    torch.cuda.empty_cache()


def test_product_maximum_space_and_k():
    """The largest space (64 values in each of the four lists, 2^24
    configurations) with k = 64: equal to the materialised pass."""
    arch = oracle.arch_cdna4()
    v = workloads.variant_features(1, 905)
    g = np.random.default_rng(905)
    space = {"block": np.sort(g.choice(np.arange(1, 1100), 64, replace=False)).astype(np.int32),
             "unroll": np.arange(1, 65, dtype=np.int32),
             "regs": np.sort(g.choice(np.arange(0, 530), 64, replace=False)).astype(np.int32),
             "grid": (np.arange(1, 65) * 97).astype(np.int32)}
    assert api.product_size(space) == 1 << 24
    b, ref, got = run_both(arch, v, space, 64)
    say("maximum space", b.n_evals, "legal top-64 of", int((ref["idx"].cpu().numpy() >= 0).sum()))
    assert_same(ref, got)
    del ref, got
    torch.cuda.empty_cache()


def test_product_empty_and_limits():
    arch = oracle.arch_cdna4()
    v = workloads.variant_features(0, 906)
    var = api.device_batch(workloads.Batch(v, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32),
                                           np.zeros(0, np.int32), None, "p"))[0]
    out = api.score_product(arch, var, SPACE_GRID, k=8)
    torch.cuda.synchronize()
    assert out["idx"].shape == (0, 8) and out["occ"].numel() == 0
    v = workloads.variant_features(2, 907)
    var = api.device_batch(workloads.Batch(v, np.zeros(3, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32),
                                           np.zeros(0, np.int32), None, "p"))[0]
    with pytest.raises(api.SAError):
        api.score_product(arch, var, {"block": list(range(1, 66)), "unroll": [1], "regs": [0]}, k=8)


@pytest.mark.parametrize("gpu", ["fermi", "kepler", "maxwell", "pascal"])
def test_product_paper_descriptors(gpu):
    """The paper's own GPUs (32-lane warps, their register files, shared
    memory and block limits): the product pass equals the materialised pass
    and the oracle."""
    arch = oracle.arch_paper(gpu)
    v = workloads.variant_features(11, 910)
    space = {"block": [32, 64, 96, 128, 192, 256, 512, 1024, 2048], "unroll": [1, 2, 4, 8],
             "regs": [0, 16, 24, 32, 63, 64, 128, 255, 256], "grid": [13, 26, 100, 1000]}
    b, ref, got = run_both(arch, v, space, 8)
    assert_same(ref, got)
    o = oracle.run(arch, b.variants, b.configs(), k=8, want_f64=False)
    assert np.array_equal(o["occ"], got["occ"].cpu().numpy())
    assert np.array_equal(o["score32"].view(np.uint32), got["score"].cpu().numpy().view(np.uint32))
    assert np.array_equal(o["idx"], got["idx"].cpu().numpy())
