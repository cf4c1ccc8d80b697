"""CPU oracle of the static autotuning model -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_1701_08547_amd``) and never imports it; both sides meet only through
the seeded input generators, which hold none of the model's arithmetic.

Contents:
  * ``sa_oracle.c``  -- occupancy (Eqs. 1-5), binary64 and binary32 scores
    (Eq. 6 with divergence and latency-hiding factors), segmented top-k by
    full sort.  Loaded here through ctypes.
  * ``exact.py``     -- the same score in exact rational arithmetic, for tiny
    inputs (pins the rounding of the C code).
  * ``placement.py`` -- a block-by-block residency simulator (pins the closed
    form of the occupancy bounds).
  * ``paper.py``     -- the paper's own search-space reduction (suggested
    thread counts T*, register headroom R*, shared memory S*, the intensity
    rule), used to check the engine against the values the paper prints.
  * ``mlp.py``       -- binary64 forward/backward of the learned correction.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sa_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libsa_oracle.so")
_lock = threading.Lock()
_lib = None

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC"]


def compile_library(force: bool = False) -> str:
    """Build ``libsa_oracle.so`` next to its source with gcc (CPU only)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


ARCH_INT_FIELDS = (
    "n_cu", "wave_size", "max_threads_per_block", "max_waves_per_cu", "max_blocks_per_cu",
    "single_wave_exempt", "simd_per_cu", "vgprs_per_simd_lane", "vgpr_granule",
    "max_vgprs_per_thread", "lds_per_cu", "lds_granule", "max_lds_per_block", "w_sat",
    "max_unroll", "max_grid",
)
ARCH_FLOAT_FIELDS = ("cpi_fp", "cpi_int", "cpi_mem", "cpi_ctrl", "cpi_sync", "cpi_reg")


class OracleArch(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in ARCH_INT_FIELDS] + [(f, ctypes.c_float) for f in ARCH_FLOAT_FIELDS]


def arch_cdna4() -> dict:
    """CDNA4 (gfx950, MI355X) descriptor as the oracle reads the paper's
    Table I rows on that part: 256 CUs, wave64, 8 wave slots on each of 4
    SIMDs, a 512-register unified VGPR/AGPR file per SIMD lane (granule 8),
    160 KiB of LDS per CU allocated in 1,280-byte granules, at most 16
    multi-wave workgroups per CU (one-wave workgroups exempt).  The register,
    wave-slot, LDS-granule and workgroup-limit values were measured on the
    device by the residency probe (workgroups resident at once per CU for
    probe kernels of known register and LDS use).  Instruction weights follow Table II's convention (CPI = 1/IPC,
    FP32 IPC = lanes per CU) with 64 lanes per CU: 2^-6 for fp and int ops,
    2^-4 for memory, control and barrier, 2^-5 for register moves."""
    return dict(
        n_cu=256, wave_size=64, max_threads_per_block=1024, max_waves_per_cu=32,
        max_blocks_per_cu=16, single_wave_exempt=1, simd_per_cu=4, vgprs_per_simd_lane=512,
        vgpr_granule=8, max_vgprs_per_thread=512, lds_per_cu=163840, lds_granule=1280,
        max_lds_per_block=163840, w_sat=32, max_unroll=64, max_grid=262144,
        cpi_fp=2.0 ** -6, cpi_int=2.0 ** -6, cpi_mem=2.0 ** -4, cpi_ctrl=2.0 ** -4,
        cpi_sync=2.0 ** -4, cpi_reg=2.0 ** -5,
    )


def arch_paper(gpu: str) -> dict:
    """The paper's NVIDIA parts (Table I limits, Table II IPC -> CPI), in the
    oracle's descriptor: one register pool per SM with R_fs / T_W registers per
    lane and no allocation rounding, shared-memory pool S_sm = S_B (Sec.
    III-A, Eq. 5 text), no rounding of shared memory."""
    t = {
        #        mp, W_mp, B_mp, R_fs,  R_T, FP32, Int, MEM, CTRL, REG IPC
        "fermi": (14, 48, 8, 32768, 63, 32, 32, 16, 16, 16),
        "kepler": (13, 64, 16, 65536, 255, 192, 160, 32, 32, 32),
        "maxwell": (24, 64, 32, 65536, 255, 128, 64, 64, 64, 32),
        "pascal": (56, 64, 32, 65536, 255, 64, 32, 16, 16, 16),
    }[gpu]
    mp, wmp, bmp, rfs, rt, ipc_fp, ipc_int, ipc_mem, ipc_ctrl, ipc_reg = t
    return dict(
        n_cu=mp, wave_size=32, max_threads_per_block=1024, max_waves_per_cu=wmp,
        max_blocks_per_cu=bmp, single_wave_exempt=0, simd_per_cu=1,
        vgprs_per_simd_lane=rfs // 32, vgpr_granule=1, max_vgprs_per_thread=rt,
        lds_per_cu=49152, lds_granule=1, max_lds_per_block=49152, w_sat=wmp, max_unroll=64,
        max_grid=262144, cpi_fp=1.0 / ipc_fp, cpi_int=1.0 / ipc_int, cpi_mem=1.0 / ipc_mem,
        cpi_ctrl=1.0 / ipc_ctrl, cpi_sync=1.0 / ipc_ctrl, cpi_reg=1.0 / ipc_reg,
    )


def _to_struct(arch: dict) -> OracleArch:
    s = OracleArch()
    for f in ARCH_INT_FIELDS:
        setattr(s, f, int(arch[f]))
    for f in ARCH_FLOAT_FIELDS:
        setattr(s, f, float(arch[f]))
    return s


def lib():
    global _lib
    with _lock:
        if _lib is None:
            compile_library()
            L = ctypes.CDLL(_LIB_PATH)
            P = ctypes.POINTER
            i32, i64, f32, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double
            vp = ctypes.c_void_p
            L.oracle_occupancy.argtypes = [P(OracleArch), i32, i32, i32, vp, i32, i32]
            L.oracle_occupancy.restype = i32
            L.oracle_active_blocks.argtypes = [P(OracleArch), i32, i32, i32]
            L.oracle_active_blocks.restype = i32
            score_args = [P(OracleArch)] + [i32] * 8 + [f32, i32, i32, i32, vp]
            L.oracle_score_f64.argtypes = score_args
            L.oracle_score_f64.restype = f64
            L.oracle_score_f32.argtypes = score_args
            L.oracle_score_f32.restype = f32
            L.oracle_topk.argtypes = [vp, vp, i64, i32, vp, vp, i32]
            L.oracle_topk.restype = ctypes.c_int
            L.oracle_run.argtypes = [P(OracleArch)] + [vp] * 14 + [i64, vp, vp, vp, i32, vp, vp, i32]
            L.oracle_run.restype = ctypes.c_int
            L.oracle_terms.argtypes = [P(OracleArch)] + [i32] * 8 + [f32, i64, vp, vp, vp, vp, vp]
            L.oracle_terms.restype = None
            L.oracle_max_threads.argtypes = []
            L.oracle_max_threads.restype = ctypes.c_int
            _lib = L
    return _lib


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _grid_ptr(G):
    if G is None:
        return None
    box = ctypes.c_int32(int(G))
    return ctypes.byref(box)


def occupancy(arch: dict, T: int, R: int, S: int, U: int = 1, G=None, valid: bool = True) -> int:
    """W* (waves per CU) of one configuration; 0 when illegal."""
    a = _to_struct(arch)
    box = None if G is None else ctypes.c_int32(int(G))
    return int(lib().oracle_occupancy(ctypes.byref(a), int(T), int(U), int(R),
                                      None if box is None else ctypes.byref(box), int(S), int(bool(valid))))


def active_blocks(arch: dict, T: int, R: int, S: int) -> int:
    """B* of Eq. 1 for (T, R, S)."""
    a = _to_struct(arch)
    return int(lib().oracle_active_blocks(ctypes.byref(a), int(T), int(R), int(S)))


def _score(fn, arch, v, T, U, R, G):
    a = _to_struct(arch)
    box = None if G is None else ctypes.c_int32(int(G))
    return fn(ctypes.byref(a), int(v["n_fp"]), int(v["n_int"]), int(v["n_ld"]), int(v["n_st"]),
              int(v["n_br"]), int(v["n_bar"]), int(v.get("n_reg", 0)), int(v["lds"]),
              float(np.float32(v["div"])), int(T), int(U), int(R),
              None if box is None else ctypes.byref(box))


def score_f64(arch: dict, v: dict, T: int, U: int, R: int, G=None) -> float:
    return float(_score(lib().oracle_score_f64, arch, v, T, U, R, G))


def score_f32(arch: dict, v: dict, T: int, U: int, R: int, G=None) -> np.float32:
    return np.float32(_score(lib().oracle_score_f32, arch, v, T, U, R, G))


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def run(arch: dict, variants: dict, configs: dict, k: int = 0, *, want_occ=True, want_f32=True,
        want_f64=True, nthreads: int | None = None) -> dict:
    """Evaluate the model over a CSR batch.

    ``variants``: dict of per-variant arrays n_fp, n_int, n_ld, n_st, n_br,
    n_bar, n_reg (optional), lds (int32), div (float32).
    ``configs``: dict with ``seg`` (int64, n_var + 1) and per-eval ``block``,
    ``unroll``, ``regs`` (int32) and optional ``grid`` (int32 or None).
    Returns dict with occ (int32), score32 (float32), score64 (float64) and,
    when k > 0, idx (int32, n_var x k) and val (float32, n_var x k).
    """
    L = lib()
    a = _to_struct(arch)
    seg = _c(configs["seg"], np.int64)
    n_var = seg.shape[0] - 1
    n = int(seg[-1])
    cols = {c: _c(configs[c], np.int32) for c in ("block", "unroll", "regs")}
    grid = configs.get("grid")
    grid = None if grid is None else _c(grid, np.int32)
    vv = {f: _c(variants[f], np.int32) for f in ("n_fp", "n_int", "n_ld", "n_st", "n_br", "n_bar", "lds")}
    n_reg = variants.get("n_reg")
    vv["n_reg"] = None if n_reg is None else _c(n_reg, np.int32)
    div = _c(variants["div"], np.float32)
    out = {}
    out["occ"] = np.empty(n, np.int32) if want_occ else None
    out["score32"] = np.empty(n, np.float32) if want_f32 else None
    out["score64"] = np.empty(n, np.float64) if want_f64 else None
    if k > 0:
        out["idx"] = np.empty((n_var, k), np.int32)
        out["val"] = np.empty((n_var, k), np.float32)
    else:
        out["idx"] = out["val"] = None
    nt = max_threads() if nthreads is None else int(nthreads)
    rc = L.oracle_run(ctypes.byref(a), _ptr(vv["n_fp"]), _ptr(vv["n_int"]), _ptr(vv["n_ld"]),
                      _ptr(vv["n_st"]), _ptr(vv["n_br"]), _ptr(vv["n_bar"]), _ptr(vv["n_reg"]),
                      _ptr(vv["lds"]), _ptr(div), _ptr(seg), _ptr(cols["block"]), _ptr(cols["unroll"]),
                      _ptr(cols["regs"]), _ptr(grid), n_var, _ptr(out["occ"]), _ptr(out["score32"]),
                      _ptr(out["score64"]), int(k), _ptr(out["idx"]), _ptr(out["val"]), nt)
    if rc != 0:
        raise MemoryError("oracle_run failed to allocate scratch")
    return out


def topk(keys, seg, k: int, nthreads: int | None = None):
    """Segmented top-k by full sort: per segment the k smallest finite keys,
    ties broken by the smaller local index, padded with (-1, +inf)."""
    keys = _c(keys, np.float32)
    seg = _c(seg, np.int64)
    n_var = seg.shape[0] - 1
    idx = np.empty((n_var, k), np.int32)
    val = np.empty((n_var, k), np.float32)
    nt = max_threads() if nthreads is None else int(nthreads)
    rc = lib().oracle_topk(_ptr(keys), _ptr(seg), n_var, int(k), _ptr(idx), _ptr(val), nt)
    if rc != 0:
        raise MemoryError("oracle_topk failed to allocate scratch")
    return idx, val


TERM_NAMES = ("W_B", "G_W", "G_R", "G_S", "B", "W", "Eprime", "F", "score")


def terms(arch: dict, v: dict, T, U, R, G=None) -> dict:
    """Binary64 per-configuration terms of one variant (arrays)."""
    a = _to_struct(arch)
    T, U, R = (_c(x, np.int32) for x in (T, U, R))
    Gc = None if G is None else _c(G, np.int32)
    n = T.shape[0]
    out = np.empty((n, 9), np.float64)
    lib().oracle_terms(ctypes.byref(a), int(v["n_fp"]), int(v["n_int"]), int(v["n_ld"]), int(v["n_st"]),
                       int(v["n_br"]), int(v["n_bar"]), int(v.get("n_reg", 0)), int(v["lds"]),
                       float(np.float32(v["div"])), n, _ptr(T), _ptr(U), _ptr(R), _ptr(Gc), _ptr(out))
    return {k: out[:, i] for i, k in enumerate(TERM_NAMES)}


def features(arch: dict, v: dict, T, U, R, G=None) -> np.ndarray:
    """The learned correction's 24 binary32 features (see oracle/mlp.py)."""
    from . import mlp

    t = terms(arch, v, T, U, R, G)
    return mlp.features_from_terms(v, T, U, R, G, arch["n_cu"], t)
