"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: the expected values are the
paper's printed tables (Table VII's T*, R*, S*, occ*; Table V's modal
occupancies; Table VI's intensities with the preferences stated in Sec. IV-B;
the pruning percentages of Sec. IV-C), hand-worked cases, an independent
residency simulator, exact rational arithmetic, a plain sort, and invariants.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import exact, paper, placement

GPUS = ("fermi", "kepler", "maxwell", "pascal")


# ------------------------------------------------------------ paper pins


def test_table1_descriptor_matches_paper(golden):
    """The oracle's paper descriptors carry Table I's limits and Table II's IPCs."""
    t1 = golden("paper_tables.json")["table1_gpus"]
    t2 = golden("paper_tables.json")["table2_ipc"]
    for g in GPUS:
        a, row, ipc = oracle.arch_paper(g), t1[g], t2[g]
        assert a["n_cu"] == row["mp"]
        assert a["wave_size"] == row["T_W"]
        assert a["max_waves_per_cu"] == row["W_mp"] == row["T_mp"] // row["T_W"]
        assert a["max_blocks_per_cu"] == row["B_mp"]
        assert a["max_threads_per_block"] == row["T_B"]
        assert a["vgprs_per_simd_lane"] * row["T_W"] == row["R_fs"]
        assert a["max_vgprs_per_thread"] == row["R_T"]
        assert a["lds_per_cu"] == a["max_lds_per_block"] == row["S_B"]
        assert a["cpi_fp"] == 1.0 / ipc["FPIns32"] and a["cpi_int"] == 1.0 / ipc["IntAdd32"]
        assert a["cpi_mem"] == 1.0 / ipc["LdSt"] and a["cpi_ctrl"] == 1.0 / ipc["Ctrl"]
        assert a["cpi_reg"] == 1.0 / ipc["Regs"]


@pytest.mark.parametrize("gpu", GPUS)
def test_suggested_threads_table7(golden, gpu):
    """T*: the thread counts reaching occupancy 1 (Eqs. 2-3) are exactly the
    ones Table VII prints for each GPU."""
    want = golden("paper_tables.json")["table7_suggested"]["t_star"][gpu]
    assert paper.suggested_threads(oracle.arch_paper(gpu)) == want


def _reproducible_register_rows(rows):
    # R^u + R* sums to 31 on two MatVec2D rows where every other row of that
    # GPU sums to 32: a misprint, excluded.
    return [r for r in rows if not (r["kernel"] == "matvec2d" and r["gpu"] in ("kepler", "maxwell"))]


def test_register_headroom_table7(golden):
    """R* = (largest registers per thread at occupancy 1) - R^u, clipped at 0,
    for every reproducible row of Table VII (Eq. 4 register path)."""
    t7 = golden("paper_tables.json")["table7_suggested"]
    rows = _reproducible_register_rows(t7["rows"])
    assert len(rows) == 14
    for r in rows:
        a = oracle.arch_paper(r["gpu"])
        for T in t7["t_star"][r["gpu"]]:
            assert paper.register_headroom(a, T, r["R_u"]) == r["R_star"], (r, T)


def test_register_limit_is_file_over_threads(golden):
    """The largest full-occupancy register count is R_fs / T_mp (Table I)."""
    t1 = golden("paper_tables.json")["table1_gpus"]
    for g in GPUS:
        a = oracle.arch_paper(g)
        T = paper.suggested_threads(a)[0]
        assert paper.max_registers_at_full(a, T) == t1[g]["R_fs"] // t1[g]["T_mp"]


def test_shared_memory_headroom_table7(golden):
    """S* (bytes) for every row of Table VII with occ* = 1: the largest shared
    memory per block that keeps occupancy 1 at the smallest suggested thread
    count, S_sm / B_mp (Eq. 5)."""
    t7 = golden("paper_tables.json")["table7_suggested"]
    rows = [r for r in t7["rows"] if r["occ"] == 1.0]
    assert len(rows) == 12
    for r in rows:
        a = oracle.arch_paper(r["gpu"])
        T = min(t7["t_star"][r["gpu"]])
        assert paper.max_shared_at_full(a, T) == r["S_star"], r


def test_fermi_bicg_three_quarter_occupancy(golden):
    """Table VII's BiCG/Fermi row: S = 8192 bytes gives occupancy .75 at a
    suggested thread count (192 threads: 6 blocks of 6 warps = 36/48)."""
    row = [r for r in golden("paper_tables.json")["table7_suggested"]["rows"]
           if r["kernel"] == "bicg" and r["gpu"] == "fermi"][0]
    a = oracle.arch_paper("fermi")
    occs = {T: oracle.occupancy(a, T, 0, row["S_star"]) / a["max_waves_per_cu"]
            for T in paper.suggested_threads(a)}
    assert row["occ"] in occs.values()
    assert occs[192] == 0.75


def test_table5_modal_occupancies_attainable(golden):
    """Every modal occupancy of Table V lies in the image of Eqs. 1-3 on its
    GPU (some thread count and some number of resident blocks reach it)."""
    modes = golden("paper_tables.json")["table5_mode_occupancy"]
    for g in GPUS:
        a = oracle.arch_paper(g)
        attain = set()
        for T in range(32, 1025, 32):
            for b in range(1, a["max_blocks_per_cu"] + 1):
                S = a["lds_per_cu"] // b  # shared memory that admits exactly b blocks
                attain.add(100.0 * oracle.occupancy(a, T, 0, S) / a["max_waves_per_cu"])
        for m in modes[g]:
            assert min(abs(m - x) for x in attain) <= 0.011, (g, m)


def test_intensity_rule_direction(golden):
    """Sec. III-C rule on Table VI's intensities: > 4.0 -> upper thread range,
    else lower, matching the preferences Sec. IV-B reports."""
    for r in golden("paper_tables.json")["table6_intensity"]["rows"]:
        t_star = paper.suggested_threads(oracle.arch_paper(r["gpu"]))
        kept = paper.rule(t_star, r["intensity"])
        assert len(kept) == len(t_star) // 2
        if r["prefers"] == "upper":
            assert kept == t_star[-len(kept):]
        else:
            assert kept == t_star[:len(kept)]


def test_pruning_percentages(golden):
    """Sec. IV-C: 5,120 variants; 4 of 32 thread counts -> 640 (87.5 %);
    5 of 32 -> 84 %; with the rule 2 of 32 -> 93.8 %, on every GPU."""
    s = golden("paper_tables.json")["search_space"]
    total = paper.space_size(*s["dims"].values())
    assert total == s["total"]
    n_tc = s["dims"]["TC"]
    assert len(range(32, 1025, 32)) == n_tc
    for g in GPUS:
        t_star = paper.suggested_threads(oracle.arch_paper(g))
        reduced = total // n_tc * len(t_star)
        pct = 100.0 * (1 - reduced / total)
        if len(t_star) == 4:
            assert reduced == s["reduced_kepler_atax"] and pct == s["pct_four_threads"]
        else:
            assert round(pct) == s["pct_five_threads"]
        for inten in (1.0, 10.0):
            kept = paper.rule(t_star, inten)
            pct_rule = 100.0 * (1 - total // n_tc * len(kept) / total)
            assert round(pct_rule, 1) == s["pct_with_rule"]


# ------------------------------------------------------------ CDNA4 hand cases


def test_cdna4_hand_worked_occupancy(golden):
    a = oracle.arch_cdna4()
    for c in golden("cdna4_hand_cases.json")["occupancy"]:
        assert oracle.occupancy(a, c["T"], c["R"], c["S"]) == c["W"], c


def test_cdna4_hand_worked_scores(golden):
    a = oracle.arch_cdna4()
    sc = golden("cdna4_hand_cases.json")["scores"]
    v = sc["variant"]
    for r in sc["rows"]:
        assert oracle.score_f64(a, v, r["T"], r["U"], r["R"], r["G"]) == r["score"], r
        assert float(oracle.score_f32(a, v, r["T"], r["U"], r["R"], r["G"])) == r["score"], r
        assert float(exact.score(a, v, r["T"], r["U"], r["R"], r["G"])) == r["score"], r


def test_tie_in_hand_cases_breaks_to_lower_index(golden):
    """Two configurations with the same score: the lower index is selected."""
    a = oracle.arch_cdna4()
    sc = golden("cdna4_hand_cases.json")["scores"]
    rows = sc["rows"][:2]
    assert rows[0]["score"] == rows[1]["score"]
    keys = np.array([oracle.score_f32(a, sc["variant"], r["T"], r["U"], r["R"], r["G"]) for r in rows] * 2,
                    dtype=np.float32)
    idx, val = oracle.topk(keys, np.array([0, 4]), 3)
    assert idx.tolist() == [[0, 1, 2]]


# ------------------------------------------------------------ special cases and invariants


def test_eq6_special_case():
    """d = 0, U = 1, no barriers, saturated occupancy, no grid: the score is
    Eq. 6 exactly, sum of CPI x count."""
    a = oracle.arch_cdna4()
    g = np.random.default_rng(7)
    for _ in range(200):
        v = dict(n_fp=int(g.integers(0, 5000)), n_int=int(g.integers(0, 5000)), n_ld=int(g.integers(0, 500)),
                 n_st=int(g.integers(0, 500)), n_br=int(g.integers(0, 500)), n_bar=0,
                 n_reg=int(g.integers(0, 500)), lds=0, div=0.0)
        T = int(g.choice([64, 128, 256, 512]))
        want = (a["cpi_fp"] * v["n_fp"] + a["cpi_int"] * v["n_int"] + a["cpi_mem"] * (v["n_ld"] + v["n_st"])
                + a["cpi_ctrl"] * v["n_br"] + a["cpi_reg"] * v["n_reg"])
        assert oracle.score_f64(a, v, T, 1, 32) == want
        assert float(oracle.score_f32(a, v, T, 1, 32)) == pytest.approx(want, rel=1e-6)


def _random_variant(g, lds_choices=(0, 256, 512, 5376, 20000, 40960, 65536)):
    return dict(n_fp=int(g.poisson(200)), n_int=int(g.poisson(150)), n_ld=int(g.poisson(40)),
                n_st=int(g.poisson(10)), n_br=int(g.poisson(12)), n_bar=int(g.integers(0, 5)),
                n_reg=int(g.integers(0, 3)), lds=int(g.choice(lds_choices)),
                div=float(np.float32(g.random() * 0.5)))


def test_closed_form_matches_residency_simulator():
    """Eqs. 1-5 (closed form) equal block-by-block placement, for CDNA4 and
    the paper's four GPUs, over thread counts at and around wave boundaries,
    register counts at and around granule boundaries, LDS sizes at and around
    granule and pool boundaries."""
    Ts = [1, 32, 33, 63, 64, 65, 96, 100, 128, 192, 256, 320, 384, 448, 512, 576, 640, 768, 960, 1024, 1025]
    Rs = [0, 1, 7, 8, 9, 16, 20, 24, 32, 33, 48, 63, 64, 65, 72, 73, 80, 96, 100, 128, 168, 170, 255, 256, 257,
          384, 511, 512, 513]
    for name, a in [("cdna4", oracle.arch_cdna4())] + [(g, oracle.arch_paper(g)) for g in GPUS]:
        pool = a["lds_per_cu"]
        Ss = [0, 1, 511, 512, 513, 1280, 1281, 5376, 6144, 6400, 6401, 8192, 11520, 20000, pool // 3, pool // 2,
              pool - 1, pool, pool + 1]
        for T in Ts:
            for R in Rs:
                for S in Ss:
                    assert oracle.active_blocks(a, T, R, S) == placement.resident_blocks(a, T, R, S), (name, T, R, S)


def test_occupancy_invariants():
    a = oracle.arch_cdna4()
    g = np.random.default_rng(11)
    for _ in range(3000):
        T = int(g.integers(1, 1025))
        R = int(g.integers(0, 513))
        S = int(g.integers(0, 163841))
        W = oracle.occupancy(a, T, R, S)
        B = oracle.active_blocks(a, T, R, S)
        W_B = -(-T // 64)
        assert W == B * W_B
        assert 0 <= W <= a["max_waves_per_cu"]  # capped by the waves-per-SIMD limit
        # never rises when registers or LDS per block rise
        assert oracle.occupancy(a, T, min(512, R + int(g.integers(1, 64))), S) <= W
        assert oracle.occupancy(a, T, R, min(163840, S + int(g.integers(1, 8192)))) <= W
        if B > 0:
            if S > 0:
                g_l = a["lds_granule"]
                assert B * (-(-S // g_l) * g_l) <= a["lds_per_cu"]
            if R > 0:
                wv = min(8, 512 // (-(-R // 8) * 8))
                assert B * W_B <= 4 * wv
            # one more block never fits
            assert placement.resident_blocks(a, T, R, S) == B
    # not monotone in T
    assert oracle.occupancy(a, 192, 0, 0) == 30 and oracle.occupancy(a, 256, 0, 0) == 32


def test_illegal_configurations_are_zero_and_infinite():
    a = oracle.arch_cdna4()
    v = dict(n_fp=200, n_int=150, n_ld=40, n_st=10, n_br=12, n_bar=2, n_reg=0, lds=0, div=0.25)
    bad = [dict(T=0), dict(T=1025), dict(R=-1), dict(R=513), dict(U=0), dict(U=65), dict(G=0),
           dict(G=262145), dict(T=1024, R=256)]
    for b in bad:
        c = dict(T=256, U=2, R=64, G=None)
        c.update(b)
        assert oracle.occupancy(a, c["T"], c["R"], 0, c["U"], c["G"]) == 0, b
        assert math.isinf(oracle.score_f64(a, v, c["T"], c["U"], c["R"], c["G"]))
        assert math.isinf(float(oracle.score_f32(a, v, c["T"], c["U"], c["R"], c["G"])))
    for field, val in [("n_fp", -1), ("n_ld", 2 ** 24), ("n_bar", 2 ** 14 + 1), ("div", 1.5), ("div", float("nan")),
                       ("lds", 163841)]:
        w = dict(v)
        w[field] = val
        assert math.isinf(oracle.score_f64(a, w, 256, 2, 64)), field
        valid = field == "lds"
        assert oracle.occupancy(a, 256, 64, w["lds"], 2, None, valid) == 0, field


def test_score_invariants():
    a = oracle.arch_cdna4()
    g = np.random.default_rng(3)
    for _ in range(2000):
        v = _random_variant(g)
        T = int(g.choice([64, 128, 192, 256, 320, 512, 768, 1024]))
        R = int(g.choice([0, 16, 64, 96, 128, 256]))
        G = None if g.random() < 0.5 else int(g.choice([256, 512, 1000, 2048]))
        U = int(g.integers(1, 8))
        s = oracle.score_f64(a, v, T, U, R, G)
        s32 = float(oracle.score_f32(a, v, T, U, R, G))
        occ = oracle.occupancy(a, T, R, v["lds"], U, G)
        assert math.isinf(s) == (occ == 0) == math.isinf(s32)
        if occ == 0:
            continue
        # non-increasing in U
        assert oracle.score_f64(a, v, T, U + 1, R, G) <= s
        assert float(oracle.score_f32(a, v, T, U + 1, R, G)) <= s32
        # score >= issue cost E' (the latency and grid factors are >= 1)
        e = oracle.score_f64(a, v, T, U, R, None) if occ * U >= 32 else None
        if e is not None:
            assert s >= e
        # doubling every count doubles the score exactly (both precisions)
        w = dict(v)
        for f in ("n_fp", "n_int", "n_ld", "n_st", "n_br", "n_bar", "n_reg"):
            w[f] = 2 * v[f]
        assert oracle.score_f64(a, w, T, U, R, G) == 2 * s
        assert float(oracle.score_f32(a, w, T, U, R, G)) == 2 * s32


def test_scores_against_exact_rationals():
    """binary64 within 1e-15 and binary32 within 1e-5 relative (and 16 ulp) of
    the exact rational score, for CDNA4 and the paper's GPUs."""
    g = np.random.default_rng(5)
    archs = [oracle.arch_cdna4()] + [oracle.arch_paper(x) for x in GPUS]
    for i in range(1500):
        a = archs[i % len(archs)]
        v = _random_variant(g, lds_choices=(0, 256, 1024, 4096, 12288))
        v["div"] = float(np.float32(g.random() * 0.5))
        T = int(g.integers(1, 1025))
        U = int(g.integers(1, 9))
        R = int(g.choice([0, 8, 16, 21, 32, 40, 64, 96, 128, 200]))
        G = None if g.random() < 0.4 else int(g.integers(1, 5000))
        ex = exact.score(a, v, T, U, R, G)
        s64 = oracle.score_f64(a, v, T, U, R, G)
        s32 = oracle.score_f32(a, v, T, U, R, G)
        if ex is None:
            assert math.isinf(s64) and math.isinf(float(s32))
            continue
        exf = float(ex)
        assert abs(s64 - exf) <= 1e-15 * abs(exf)
        assert abs(float(s32) - exf) <= 1e-5 * abs(exf)
        assert abs(float(s32) - exf) <= 16 * float(np.spacing(np.float32(exf)))


# ------------------------------------------------------------ selection


def _brute_topk(keys, seg, k):
    idx = np.full((len(seg) - 1, k), -1, np.int32)
    val = np.full((len(seg) - 1, k), np.inf, np.float32)
    for v in range(len(seg) - 1):
        ent = [(float(keys[e]), e - seg[v]) for e in range(seg[v], seg[v + 1]) if np.isfinite(keys[e])]
        ent.sort()
        for j, (s, i) in enumerate(ent[:k]):
            idx[v, j], val[v, j] = i, s
    return idx, val


def test_topk_matches_plain_sort_with_ties_and_short_segments():
    g = np.random.default_rng(9)
    for trial in range(30):
        sizes = g.choice([0, 1, 2, 3, 7, 8, 9, 31, 64, 65, 200], size=int(g.integers(1, 12)))
        seg = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        n = int(seg[-1])
        keys = g.choice(np.array([0.0, 0.5, 1.0, 1.5, 2.0, 3.25, np.inf], np.float32), size=n)  # many ties
        if trial % 2:
            keys = (g.random(n) * 10).astype(np.float32)
            keys[g.random(n) < 0.2] = np.inf
            keys[g.random(n) < 0.02] = np.nan
        k = int(g.choice([1, 2, 8, 16]))
        idx, val = oracle.topk(keys, seg, k)
        bidx, bval = _brute_topk(keys, seg, k)
        assert (idx == bidx).all() and np.array_equal(val, bval)


def test_run_topk_equals_topk_of_scores():
    from paper_1701_08547_amd import workloads

    a = oracle.arch_cdna4()
    b = workloads.custom_batch(1, [0, 1, 5, 64, 300, 1000], with_grid=True)
    out = oracle.run(a, b.variants, b.configs(), k=8)
    idx, val = oracle.topk(out["score32"], b.seg, 8)
    assert (idx == out["idx"]).all() and np.array_equal(val, out["val"])
    bidx, bval = _brute_topk(out["score32"], b.seg, 8)
    assert (idx == bidx).all()
    # scores agree with the scalar entry points
    for e in range(0, b.n_evals, 37):
        v = int(np.searchsorted(b.seg, e, side="right") - 1)
        vd = {f: b.variants[f][v] for f in b.variants}
        assert out["score32"][e] == oracle.score_f32(a, vd, b.block[e], b.unroll[e], b.regs[e], b.grid[e])
        assert out["occ"][e] == oracle.occupancy(a, b.block[e], b.regs[e], vd["lds"], b.unroll[e], b.grid[e])


def test_workload_shapes():
    from paper_1701_08547_amd import workloads

    b0 = workloads.c0()
    assert b0.n_var == 1 and b0.n_evals == 4096 and b0.grid is None
    assert b0.block[0] == 64 and b0.block[-1] == 1024 and b0.regs[1] == 32  # registers fastest
    v = workloads.variant_features(20000, 1)
    assert abs(v["n_fp"].mean() - 200) < 2 and abs(v["n_ld"].mean() - 40) < 1
    assert v["lds"].max() <= 65536 and (v["lds"] % 256 == 0).all()
    assert v["div"].dtype == np.float32 and v["div"].max() < 0.5
    s = workloads.loguniform_sizes(10000, 64, 262144, 2)
    assert s.min() >= 64 and s.max() <= 262144
