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


def _headroom(arch, T, R=None):
    b = torch.from_numpy(np.asarray(T, np.int32)).cuda()
    r = None if R is None else torch.from_numpy(np.asarray(R, np.int32)).cuda()
    rs, ss = api.headroom(arch, b, r)
    torch.cuda.synchronize()
    return rs.cpu().numpy(), ss.cpu().numpy()


def test_headroom_table7(golden):
    """R* and S* of Table VII from the GPU: every reproducible [R^u : R*] row
    at each suggested thread count, and S* (bytes) at the smallest suggested
    thread count for the rows with occupancy 1."""
    t7 = golden("paper_tables.json")["table7_suggested"]
    rows = [r for r in t7["rows"] if not (r["kernel"] == "matvec2d" and r["gpu"] in ("kepler", "maxwell"))]
    assert len(rows) == 14
    for r in rows:
        a = oracle.arch_paper(r["gpu"])
        ts = t7["t_star"][r["gpu"]]
        rs, ss = _headroom(a, ts, [r["R_u"]] * len(ts))
        assert rs.tolist() == [r["R_star"]] * len(ts), (r, rs)
        if r["occ"] == 1.0:
            assert int(ss[ts.index(min(ts))]) == r["S_star"], (r, ss)


@pytest.mark.parametrize("name", ["cdna4", "fermi", "kepler", "maxwell", "pascal"])
def test_headroom_matches_oracle(name):
    """Every block size from -1 to the limit plus a wave, against the
    oracle's searches over Eqs. 1-5 (registers by scan, LDS by bisection);
    out-of-range rows give 0."""
    a = oracle.arch_cdna4() if name == "cdna4" else oracle.arch_paper(name)
    ws, tmax, rmax = a["wave_size"], a["max_threads_per_block"], a["max_vgprs_per_thread"]
    g = a["vgpr_granule"]
    r_set = sorted({0, 1, g - 1 if g > 1 else 0, g, 16, 21, 32, 40, 63, 64, 65, rmax - 1, rmax, rmax + 1, -1})
    Ts = list(range(-1, tmax + ws + 1))
    T = np.repeat(np.array(Ts, np.int32), len(r_set))
    R = np.tile(np.array(r_set, np.int32), len(Ts))
    rs, ss = _headroom(a, T, R)
    rs0, ss0 = _headroom(a, Ts)
    rfull, sfull = {}, {}
    for t in Ts:
        ok = 1 <= t <= tmax
        rfull[t] = paper.max_registers_at_full(a, t) if ok else 0
        sfull[t] = paper.max_shared_at_full(a, t) if ok else 0
    for i, (t, r) in enumerate(zip(T.tolist(), R.tolist())):
        valid = 1 <= t <= tmax and 0 <= r <= rmax
        want_r = max(0, rfull[t] - r) if valid else 0
        want_s = sfull[t] if valid else 0
        assert (int(rs[i]), int(ss[i])) == (want_r, want_s), (name, t, r, rs[i], ss[i], want_r, want_s)
    assert rs0.tolist() == [rfull[t] for t in Ts]
    assert ss0.tolist() == [sfull[t] for t in Ts]
    say(name, "R* at T = 4 waves:", rfull[4 * ws], "S*:", sfull[4 * ws])
