"""GPU parity of the paper's search-space reduction (Sec. III-C, IV-C)
against the oracle: the kept block sizes per variant (T* by full occupancy,
then the intensity half-range rule) and the top-k restricted to them."""
import sys

import numpy as np
import pytest

import oracle
from oracle import paper
from paper_1701_08547_amd import api, workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)


def say(*a):
    print("[gpu-suggest]", *a, flush=True)
    sys.stdout.flush()


def oracle_kept(arch, v):
    ws = arch["wave_size"]
    t_star = paper.suggested_threads(arch, range(ws, arch["max_threads_per_block"] + 1, ws))
    inten = paper.intensity(float(v["n_fp"]), float(v["n_ld"] + v["n_st"]))
    return set(paper.rule(t_star, inten))


def variants_both_sides(n, seed):
    g = np.random.default_rng(seed)
    v = workloads.variant_features(n, 500 + seed)
    mem = v["n_ld"] + v["n_st"]
    # a third exactly at the threshold (intensity 4.0 -> lower half), a third above
    k = n // 3
    v["n_fp"][:k] = 4 * np.maximum(1, mem[:k])
    v["n_fp"][k:2 * k] = 4 * np.maximum(1, mem[k:2 * k]) + g.integers(1, 50, k)
    return v


@pytest.mark.parametrize("name", ["cdna4", "fermi", "kepler", "maxwell", "pascal"])
def test_kept_masks_match_oracle(name):
    arch = oracle.arch_cdna4() if name == "cdna4" else oracle.arch_paper(name)
    v = variants_both_sides(300, 1)
    b = workloads.Batch(v, np.zeros(301, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32),
                        np.zeros(0, np.int32), None, "suggest")
    var, _ = api.device_batch(b)
    kept = api.suggest(arch, var).cpu().numpy().view(np.uint64)
    ws = arch["wave_size"]
    for i in range(300):
        vi = {k2: a[i] for k2, a in v.items()}
        want = oracle_kept(arch, vi)
        got = {ws * (j + 1) for j in range(64) if (int(kept[i]) >> j) & 1}
        assert got == want, (name, i, sorted(got), sorted(want))
    say(name, "kept sizes e.g.", sorted({ws * (j + 1) for j in range(64) if (int(kept[0]) >> j) & 1}))


@pytest.mark.parametrize("with_grid", [True, False])
def test_restricted_topk_matches_oracle(with_grid):
    arch = oracle.arch_cdna4()
    b = workloads.custom_batch(71 if with_grid else 72, [1, 500, 4096, 0, 9000, 65], with_grid=with_grid)
    b.variants.update({k2: a for k2, a in variants_both_sides(b.n_var, 2).items() if k2 in ("n_fp", "n_ld", "n_st")})
    var, cfg = api.device_batch(b)
    got = api.score_suggested(arch, var, cfg, k=8, want_score=True)
    torch.cuda.synchronize()
    ref = oracle.run(arch, b.variants, b.configs(), k=0)
    s32 = ref["score32"]
    assert np.array_equal(got["score"].cpu().numpy().view(np.uint32), s32.view(np.uint32))
    idx = got["idx"].cpu().numpy()
    val = got["val"].cpu().numpy()
    for vv in range(b.n_var):
        lo, hi = int(b.seg[vv]), int(b.seg[vv + 1])
        kept = oracle_kept(arch, {k2: a[vv] for k2, a in b.variants.items()})
        keys = [(s32[e], e - lo) for e in range(lo, hi) if int(b.block[e]) in kept and np.isfinite(s32[e])]
        keys.sort()
        want = [j for _, j in keys[:8]] + [-1] * (8 - min(8, len(keys)))
        assert idx[vv].tolist() == want, (vv, idx[vv], want)
        wv = [s for s, _ in keys[:8]] + [np.inf] * (8 - min(8, len(keys)))
        assert np.array_equal(val[vv].astype(np.float32).view(np.uint32), np.array(wv, np.float32).view(np.uint32))
