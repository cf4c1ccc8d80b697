"""The C-ABI library builds, loads and exports every entry point that
include/sa.h declares; argument validation runs on the host before any HIP
call, so these tests need no GPU."""
import ctypes
import os
import re

import pytest

import oracle
from paper_1701_08547_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    inc = os.path.join(ROOT, "include")
    src = "".join(open(os.path.join(inc, h)).read() for h in sorted(os.listdir(inc)) if h.endswith(".h"))
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sa_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(api.LIB_PATH):
        from paper_1701_08547_amd import build

        build.build()
    return api.lib()


def test_every_declared_symbol_is_exported(L):
    declared = _header_functions()
    assert declared, "no declarations found"
    assert sorted(api.EXPORTED) == declared
    for name in declared:
        assert hasattr(L, name), name


def test_status_strings(L):
    for code, name in api.STATUS_NAMES.items():
        assert L.sa_status_string(code).decode() == name


def test_gfx950_constants_equal_oracle_descriptor(L):
    """The library and the oracle keep separate copies of the CDNA4
    constants; they must agree field by field."""
    lib_arch = api.arch_gfx950()
    ora = oracle.arch_cdna4()
    assert set(lib_arch) == set(ora)
    for f in ora:
        assert lib_arch[f] == ora[f], f
    api.arch_validate(lib_arch)


def test_paper_descriptors_are_supported(L):
    for g in ("fermi", "kepler", "maxwell", "pascal"):
        api.arch_validate(oracle.arch_paper(g))


@pytest.mark.parametrize("field,value", [("n_cu", 0), ("wave_size", 1), ("max_waves_per_cu", 65),
                                         ("max_unroll", 65), ("max_grid", 1 << 19), ("vgpr_granule", 0),
                                         ("cpi_fp", float("nan")), ("cpi_mem", -1.0), ("simd_per_cu", 33),
                                         ("max_threads_per_block", 65537)])
def test_invalid_descriptor_rejected(L, field, value):
    a = api.arch_gfx950()
    a[field] = value
    with pytest.raises(api.SAError) as e:
        api.arch_validate(a)
    assert e.value.status == -6


def test_table_size_limit(L):
    a = api.arch_gfx950()
    a["vgpr_granule"] = 1
    a["max_vgprs_per_thread"] = 1024  # 1025 x 17 > 16384 entries
    with pytest.raises(api.SAError):
        api.arch_validate(a)


def test_workspace_bytes(L):
    assert api.workspace_bytes(10, 0, 8) == 0
    assert api.workspace_bytes(10, 100, 0) == 0
    n = 16_384_000
    assert api.workspace_bytes(1000, n, 8) >= 2 * (n // 1024) * 8 * 8


def _null_args():
    a = api._arch_struct(api.arch_gfx950())
    v = api.SaVariants()
    c = api.SaConfigs()
    return a, v, c


def test_argument_errors_before_any_launch(L):
    a, v, c = _null_args()
    by = ctypes.byref
    # NULL arch
    assert L.sa_score(None, by(v), by(c), 1, 1, None, None, 8, None, None, None, None, 0, None) == -1
    # negative sizes
    assert L.sa_score(by(a), by(v), by(c), -1, 1, None, None, 8, None, None, None, None, 0, None) == -1
    # evaluations without variants
    assert L.sa_occupancy(by(a), by(v), by(c), 0, 5, None, None) == -1
    # NULL variant columns, then NULL seg
    assert L.sa_occupancy(by(a), by(v), by(c), 1, 5, None, None) == -1
    assert "variant" in L.sa_last_error().decode()
    v_ok = api.SaVariants(*([8] * 9))
    assert L.sa_occupancy(by(a), by(v_ok), by(c), 1, 5, None, None) == -1
    assert "seg" in L.sa_last_error().decode()
    # misaligned seg
    c.seg = 4
    assert L.sa_occupancy(by(a), by(v), by(c), 0, 0, None, None) == -2
    # k outside [1, 64]
    assert L.sa_topk(None, ctypes.c_void_p(8), 1, 0, 0, ctypes.c_void_p(16), None, None, 0, None) == -1
    assert L.sa_topk(None, ctypes.c_void_p(8), 1, 0, 65, ctypes.c_void_p(16), None, None, 0, None) == -1
    # workspace missing for a top-k over evaluations
    assert L.sa_topk(ctypes.c_void_p(256), ctypes.c_void_p(8), 1, 100, 8, ctypes.c_void_p(16), None, None, 0,
                     None) == -4
    # workspace too small / misaligned
    assert L.sa_topk(ctypes.c_void_p(256), ctypes.c_void_p(8), 1, 100, 8, ctypes.c_void_p(16), None,
                     ctypes.c_void_p(256), 8, None) == -4
    assert L.sa_topk(ctypes.c_void_p(256), ctypes.c_void_p(8), 1, 100, 8, ctypes.c_void_p(16), None,
                     ctypes.c_void_p(128), 1 << 20, None) == -2
    # corrected mode: the network's pointers are checked before any launch
    v2 = api.SaVariants(*([8] * 9))
    c2 = api.SaConfigs(8, 8, 8, 8, None)
    m_null = api.SaMlp(*([256] * 7 + [None]))
    assert L.sa_score(by(a), by(v2), by(c2), 1, 1, ctypes.c_void_p(8), None, 0, None, None, by(m_null),
                      None, 0, None) == -1
    assert "mlp" in L.sa_last_error().decode()
    m_odd = api.SaMlp(*([260] + [256] * 7))
    assert L.sa_score(by(a), by(v2), by(c2), 1, 1, ctypes.c_void_p(8), None, 0, None, None, by(m_odd),
                      None, 0, None) == -2


def test_tile_setter(L):
    with pytest.raises(api.SAError):
        api.set_tile(1000)
    with pytest.raises(api.SAError):
        api.set_tile(512)
    api.set_tile(2048)
    api.set_tile(0)


def test_no_device_is_reported(L):
    try:
        import torch

        has_gpu = torch.cuda.device_count() > 0
    except Exception:
        has_gpu = False
    if has_gpu:
        pytest.skip("a GPU is present")
    with pytest.raises(api.SAError) as e:
        api.arch_default(0)
    assert e.value.status == -3


def test_suggest_argument_errors(L):
    a = api.SaArch()
    assert L.sa_arch_gfx950(ctypes.byref(a)) == 0
    v = api.SaVariants(*([8] * 9))
    assert L.sa_suggest(ctypes.byref(a), ctypes.byref(v), 5, None, None) == -1
    assert L.sa_suggest(ctypes.byref(a), ctypes.byref(v), 5, ctypes.c_void_p(12), None) == -2
    assert L.sa_suggest(ctypes.byref(a), ctypes.byref(v), -1, ctypes.c_void_p(16), None) == -1
    assert L.sa_suggest(ctypes.byref(a), ctypes.byref(v), 0, None, None) == 0
    c = api.SaConfigs(8, 8, 8, 8, None)
    # no top-k output / k out of range
    assert L.sa_score_suggested(ctypes.byref(a), ctypes.byref(v), ctypes.byref(c), 1, 1, None, None, 8, None, None,
                                None, 0, None) == -1
    assert L.sa_score_suggested(ctypes.byref(a), ctypes.byref(v), ctypes.byref(c), 1, 1, None, None, 0,
                                ctypes.c_void_p(16), None, None, 0, None) == -1



def test_headroom_argument_errors(L):
    a = api.SaArch()
    assert L.sa_arch_gfx950(ctypes.byref(a)) == 0
    p = ctypes.c_void_p
    assert L.sa_headroom(ctypes.byref(a), None, None, 4, p(16), None, None) == -1      # block NULL
    assert L.sa_headroom(ctypes.byref(a), p(16), None, 4, None, None, None) == -1      # no output
    assert L.sa_headroom(ctypes.byref(a), p(16), None, -1, p(16), None, None) == -1    # negative n
    assert L.sa_headroom(ctypes.byref(a), p(18), None, 4, p(16), None, None) == -2     # misaligned
    assert L.sa_headroom(ctypes.byref(a), p(16), None, 4, None, p(22), None) == -2
    assert L.sa_headroom(ctypes.byref(a), None, None, 0, None, None, None) == 0        # empty
    bad = api.SaArch()
    ctypes.memmove(ctypes.byref(bad), ctypes.byref(a), ctypes.sizeof(a))
    bad.wave_size = 48
    assert L.sa_headroom(ctypes.byref(bad), p(16), None, 4, p(16), None, None) == -6   # descriptor rejected


def test_product_argument_errors(L):
    a = api.SaArch()
    assert L.sa_arch_gfx950(ctypes.byref(a)) == 0
    v = api.SaVariants(*([16] * 9))
    vals = (ctypes.c_int32 * 65)(*range(1, 66))
    p = ctypes.cast(vals, ctypes.c_void_p)
    out = ctypes.c_void_p(256)
    ok = api.SaProduct(2, 2, 2, 0, p, p, p, None)
    sc = lambda sp, **kw: L.sa_score_product(ctypes.byref(a), ctypes.byref(v), kw.get("n", 3),
                                             None if sp is None else ctypes.byref(sp), kw.get("score", out), None,
                                             kw.get("k", 8), kw.get("idx"), None, kw.get("ws"), kw.get("wsb", 0), None)
    assert sc(None) == -1
    assert sc(api.SaProduct(0, 2, 2, 0, p, p, p, None)) == -1            # empty block list
    assert sc(api.SaProduct(65, 2, 2, 0, p, p, p, None)) == -1           # too many values
    assert sc(api.SaProduct(2, 2, 2, -1, p, p, p, None)) == -1           # negative grid count
    assert sc(api.SaProduct(2, 2, 2, 2, p, p, p, None)) == -1            # grid list NULL
    assert sc(api.SaProduct(2, 2, 2, 0, p, None, p, None)) == -1        # unroll list NULL
    assert sc(ok, n=-1) == -1
    assert sc(ok, score=None) == -1                                     # no output
    assert sc(ok, n=0, score=None) == 0                                 # empty batch: nothing to write
    assert sc(ok, score=ctypes.c_void_p(258)) == -2                     # misaligned
    assert sc(ok, idx=out, k=0) == -1                                   # k outside [1, 64]
    assert sc(ok, idx=out, ws=None) == -4                               # top-k needs a workspace
    assert sc(ok, idx=out, ws=ctypes.c_void_p(256), wsb=8) == -4        # too small
    assert sc(ok, idx=out, ws=ctypes.c_void_p(128), wsb=1 << 20) == -2  # misaligned workspace
    assert sc(ok, n=0) == 0
    assert L.sa_product_workspace_bytes(3, 8, 8) > 0 and L.sa_product_workspace_bytes(0, 8, 8) == 0


def test_product_division_bound():
    """floor(x m / 2^32) with m = ceil(2^32 / n) is floor(x / n) for every
    x < 2^24 and 2 <= n <= 64 (the digit extraction of product spaces)."""
    import numpy as np

    x = np.arange(1 << 24, dtype=np.uint64)
    for n in range(2, 65):
        m = np.uint64(((1 << 32) + n - 1) // n)
        assert np.array_equal((x * m) >> np.uint64(32), x // np.uint64(n)), n


def test_pairwise_train_argument_errors(L):
    m = api.SaMlp(*([ctypes.c_void_p(256)] * 8))
    p = ctypes.c_void_p(256)
    call = lambda n, group: L.sa_surrogate_train_step_pairwise(ctypes.byref(m), p, p, p, 1, None, ctypes.c_float(1e-3),
                                                               p, p, n, group, None, p, 1 << 30, None)
    assert call(256, 1) == -1           # group below 2
    assert call(2048, 2048) == -1       # group above the maximum
    assert call(300, 128) == -1         # n not a multiple of the group
    assert b"group" in L.sa_last_error() or b"multiple" in L.sa_last_error()


def test_train_step_counter_arguments(L):
    """A host step number and a device step counter are exclusive; the
    counter must be 8-byte aligned.  Checked before any launch."""
    m = api.SaMlp(*([ctypes.c_void_p(256)] * 8))
    p = ctypes.c_void_p(256)
    call = lambda step, counter: L.sa_surrogate_train_step(ctypes.byref(m), p, p, p, step, counter,
                                                           ctypes.c_float(1e-3), p, p, 64, None, p, 1 << 30, None)
    assert call(0, None) == -1                        # no step number and no counter
    assert call(3, ctypes.c_void_p(4096)) == -1       # both
    assert call(0, ctypes.c_void_p(4100)) == -2       # counter misaligned
    assert b"step" in L.sa_last_error() or b"aligned" in L.sa_last_error()
