"""Host-side pieces of the measured-runtime dataset: launch rules, trip
counts, argument checks of the timing harness, the sampling of instances
and the static instruction mix read from the library's own assembly."""
import ctypes
import os

import numpy as np
import pytest

from paper_1701_08547_amd import api, asm_features, runtime_dataset as rd

FIXTURE = """\
_Zdemo:                                 ; @_Zdemo
; %bb.0:
\tv_mov_b32_e32 v1, 0
\tv_cmp_gt_i32_e32 vcc, s4, v0
\ts_and_saveexec_b64 s[2:3], vcc
\ts_cbranch_execz .LBB0_4
.LBB0_2:                                ; =>This Inner Loop Header: Depth=1
\tglobal_load_dword v5, v[2:3], off
\tv_fma_f32 v4, v5, v5, v4
\tv_add_u32_e32 v2, 4, v2
\tv_cmp_gt_u32_e32 vcc, s6, v2
\ts_and_saveexec_b64 s[8:9], vcc
; %bb.3:                                ;   in Loop: Header=BB0_2 Depth=1
\tds_write_b32 v0, v4
\tv_cvt_f32_i32_e32 v7, v2
\ts_or_b64 exec, exec, s[8:9]
\ts_barrier
\ts_cbranch_scc1 .LBB0_2
.LBB0_4:
\tglobal_store_dword v[0:1], v4, off
\ts_endpgm
.Lfunc_end0:
"""


def test_fixture_mix():
    km = asm_features.parse(FIXTURE)["_Zdemo"]
    assert km.outside == dict(n_fp=0, n_int=1, n_ld=0, n_st=1, n_br=1, n_bar=0, n_reg=1)
    assert km.loops == [dict(n_fp=1, n_int=3, n_ld=1, n_st=1, n_br=1, n_bar=1, n_reg=0)]
    # six vector instructions in the loop, two after the in-loop exec mask
    assert km.loop_vec == [6] and km.loop_div == [2]
    c = km.counts([10])
    assert c["n_fp"] == 10 and c["n_int"] == 31 and c["n_st"] == 11 and c["n_bar"] == 10
    assert km.divergence([10]) == pytest.approx(2 / 6)
    with pytest.raises(ValueError):
        km.counts([1, 2])


def test_categories():
    cat = asm_features.category
    assert cat("v_pk_fma_f16") == "n_fp" and cat("v_exp_f32_e32") == "n_fp" and cat("v_cmp_lt_f32_e64") == "n_fp"
    assert cat("v_cvt_f32_u32_e32") == "n_int" and cat("v_lshl_add_u64") == "n_int"
    assert cat("v_cndmask_b32_e64") == "n_int"
    assert cat("ds_read_b128") == "n_ld" and cat("buffer_load_dwordx4") == "n_ld"
    assert cat("global_atomic_add_f32") == "n_st" and cat("ds_write2_b32") == "n_st"
    assert cat("s_cbranch_execz") == "n_br" and cat("s_barrier") == "n_bar"
    assert cat("v_accvgpr_write_b32") == "n_reg" and cat("scratch_load_dword") == "n_reg"
    assert cat("s_add_u32") is None and cat("s_waitcnt") is None and cat("s_load_dword") is None


@pytest.fixture(scope="module")
def kernels():
    path = os.path.join(os.path.dirname(api.LIB_PATH), "sa_runtime_gfx950.s")
    if not os.path.exists(path):
        from paper_1701_08547_amd import build

        build.build_runtime_asm()
    return asm_features.runtime_kernels(path)


def test_families_have_the_documented_loops(kernels):
    assert len(kernels) == 24
    for (fam, u), km in kernels.items():
        assert len(km.loops) == (2 if fam == "reduce" else 1), (fam, u)
        assert km.regs > 0
        assert km.lds == (4096 if fam == "reduce" else 0)
        # the main loop's float work grows with the unroll factor
        assert km.loops[0]["n_fp"] >= u
    for fam in rd.FAMILIES:
        assert kernels[(fam, 8)].loops[0]["n_ld"] > kernels[(fam, 1)].loops[0]["n_ld"]
    assert kernels[("reduce", 1)].loops[1]["n_bar"] == 1


def test_launch_rules_and_trips():
    L = api.lib()
    assert L.sa_rt_grid(0, 1680, 64, 1, 256) == 27 * 2
    assert L.sa_rt_grid(0, 1000, 64, 1, 256) == -1      # not a multiple of 840
    assert L.sa_rt_trips(0, 1680, 64, 7, 54, 0) == 120
    G = L.sa_rt_grid(1, 8192, 256, 4, 256)
    units = 8190 * (-(-8190 // 4))
    assert G == min(-(-units // 256), 256 * 8)
    assert L.sa_rt_trips(1, 8192, 256, 4, G, 0) == -(-units // (G * 256))
    assert L.sa_rt_grid(2, 1 << 28, 1024, 8, 256) == 256 * 2
    assert L.sa_rt_trips(2, 1 << 28, 1024, 8, 512, 0) == (1 << 28) // (512 * 1024 * 8)
    assert L.sa_rt_trips(2, 1 << 20, 960, 1, 10, 1) == 10    # 960 -> 1024: ten halvings
    assert L.sa_rt_trips(2, 1 << 20, 960, 1, 10, 2) == -1
    assert L.sa_rt_grid(3, 100, 64, 1, 256) == -1
    assert L.sa_rt_grid(2, 100, 64, 9, 256) == -1
    assert L.sa_rt_buffer_floats(0, 840, 0) == 840 * 840 and L.sa_rt_buffer_floats(2, 99, 2) == 1


def test_measure_argument_errors():
    L = api.lib()
    T = np.array([64], np.int32)
    U = np.array([1], np.int32)
    ms = np.zeros(1, np.float32)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    fake = ctypes.c_void_p(256)
    assert L.sa_rt_measure(0, 1680, fake, fake, fake, p(T), p(U), 1, 256, 1, 65, 5, p(ms), None) == -1
    assert L.sa_rt_measure(0, 1680, fake, fake, fake, p(T), p(U), 1, 256, 1, 10, 11, p(ms), None) == -1
    assert L.sa_rt_measure(0, 1680, fake, None, fake, p(T), p(U), 1, 256, 1, 10, 5, p(ms), None) == -1
    assert L.sa_rt_measure(0, 1680, fake, fake, fake, None, p(U), 1, 256, 1, 10, 5, p(ms), None) == -1
    assert b"buffer" in L.sa_rt_last_error() or b"NULL" in L.sa_rt_last_error()


def test_instance_sampling():
    a = rd.sample_instances(50, 0)
    b = rd.sample_instances(50, 0)
    assert a == b and len(a) == 150
    for fam, n in a:
        lo, hi = rd.SIZE_RANGE[fam]
        if fam == "matvec":
            assert n % 840 == 0 and 1680 <= n <= 32760
        else:
            assert lo <= n <= hi
    T, U = rd.config_grid()
    assert T.size == 128 and len(set(zip(T.tolist(), U.tolist()))) == 128


def test_parts_cover_and_assemble():
    inst = rd.sample_instances(3, 5)
    shares = [rd.select(inst, f, p, 2) for f in rd.FAMILIES for p in range(2)]
    assert sorted(i for s in shares for i in s) == list(range(len(inst)))
    mk = lambda idx: {"index": np.asarray(idx, np.int64),
                      "ms": np.arange(len(idx) * rd.N_CFG, dtype=np.float32).reshape(len(idx), rd.N_CFG) + 1000 * idx[0],
                      "n_cu": np.array([256]), "per_family": np.array([3]), "seed": np.array([5])}
    parts = [mk(s) for s in shares if s]
    rows = rd.assemble(parts[::-1])                  # any order of parts
    assert rows["ms"].size == len(inst) * rd.N_CFG
    assert rows["n"].tolist()[::rd.N_CFG] == [n for _, n in inst]
    assert rows["ms"][:rd.N_CFG].tolist() == parts[0]["ms"][0].tolist()
    direct = rd.static_rows(inst, 256)
    for f in rd.COUNT_FIELDS + ("block", "unroll", "grid", "regs"):
        assert np.array_equal(rows[f], direct[f])
    with pytest.raises(ValueError):
        rd.assemble([parts[0], parts[0]])
    other = dict(parts[1], seed=np.array([6]))
    with pytest.raises(ValueError):
        rd.assemble([parts[0], other])


def test_imix_static_side_and_comparison(tmp_path):
    from paper_1701_08547_amd import imix

    cs = imix.cases()
    assert len(cs) == 81 and len(set(cs)) == 81
    pred = imix.predicted(cs, 256)
    # a family's counted loads are at least one per element it reads
    mv = [p for p in pred if p["family"] == "matvec" and p["U"] == 1]
    for p in mv:
        assert p["static"]["vmem_rd"] * 64 >= p["n"] * p["n"]
    # a counter file that matches the static side exactly gives zero error
    path = tmp_path / "c.csv"
    with open(path, "w") as f:
        f.write('"Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value"\n')
        f.write('1,"void at::native::fill","SQ_INSTS_VALU",5\n')
        for i, p in enumerate(pred):
            kn = "void (anonymous namespace)::rt_%s<%d>(int)" % (p["family"], p["U"])
            for cn, cls in imix.COUNTERS.items():
                f.write('%d,"%s","%s",%d\n' % (i + 2, kn, cn, p["static"][cls]))
            f.write('%d,"%s","SQ_WAVES",%d\n' % (i + 2, kn, p["waves"]))
    rep = imix.compare(pred, imix.read_counters(str(path)))
    for fam, s in rep["summary"].items():
        assert s["waves_exact"]
        assert all(v["max_abs_error"] == 0.0 for k, v in s.items() if k != "waves_exact")
    with pytest.raises(ValueError):
        imix.compare(pred[:-1], imix.read_counters(str(path)))


def test_cpi_argument_errors():
    L = api.lib()
    p = ctypes.c_void_p(256)
    assert L.sa_rt_cpi(6, 3, p, p, None, None) == -1
    assert L.sa_rt_cpi(-1, 3, p, p, None, None) == -1
    assert L.sa_rt_cpi(0, 0, p, p, None, None) == -1
    assert L.sa_rt_cpi(0, 65, p, p, None, None) == -1
    assert L.sa_rt_cpi(0, 3, None, p, None, None) == -1
    assert L.sa_rt_cpi(0, 3, p, None, None, None) == -1
    assert b"NULL" in L.sa_rt_last_error()


def test_stream_argument_errors():
    """Invalid stream-ceiling arguments are refused before anything is
    launched (no GPU needed)."""
    L = api.lib()
    p = ctypes.c_void_p(4096)
    ms = ctypes.c_float(0.0)
    ok = (p, p, p, p, p, p)
    assert L.sa_rt_stream(0, *ok, 1, 0, 0, 3, ctypes.byref(ms), None) == -1
    assert L.sa_rt_stream(6, *ok, 1, 0, 0, 3, ctypes.byref(ms), None) == -1
    assert b"multiple of 4" in L.sa_rt_last_error()
    for items in (0, 3, 8):
        assert L.sa_rt_stream(64, *ok, items, 0, 0, 3, ctypes.byref(ms), None) == -1
    assert L.sa_rt_stream(64, *ok, 1, -1, 0, 3, ctypes.byref(ms), None) == -1
    assert L.sa_rt_stream(64, *ok, 1, 65, 0, 3, ctypes.byref(ms), None) == -1
    assert L.sa_rt_stream(64, *ok, 1, 0, 0, 0, ctypes.byref(ms), None) == -1
    assert L.sa_rt_stream(64, *ok, 1, 0, 0, 65, ctypes.byref(ms), None) == -1
    assert L.sa_rt_stream(64, p, p, None, p, p, p, 1, 0, 0, 3, ctypes.byref(ms), None) == -1
    assert b"NULL" in L.sa_rt_last_error()
    assert L.sa_rt_stream(64, p, p, p, p, p, ctypes.c_void_p(4100), 1, 0, 0, 3, ctypes.byref(ms), None) == -1
    assert b"aligned" in L.sa_rt_last_error()
    assert L.sa_rt_stream(64, *ok, 1, 0, 0, 3, None, None) == -1
    assert L.sa_rt_stream(64, *ok, 1, 0, 2, 3, ctypes.byref(ms), None) == -1
    assert b"nontemporal" in L.sa_rt_last_error()


def test_calibrated_descriptor_mapping():
    from paper_1701_08547_amd import calibration

    arch = {"cpi_" + c: 1.0 for c in calibration.CATEGORIES}
    meas = {c: (0.5 + i, 1.0) for i, c in enumerate(calibration.CATEGORIES)}
    a = calibration.calibrated_arch(arch, meas)
    assert a["cpi_fp"] == 0.5 and a["cpi_reg"] == 5.5 and a["cpi_sync"] == 4.5 / 4
    assert arch["cpi_fp"] == 1.0                      # the input is not modified
