"""Thin Python binding of the C ABI in ``include/sa.h`` (ctypes).

Argument marshalling only: tensors are checked for device, dtype and
contiguity and handed over as raw device pointers together with the current
torch stream; every step of the model runs in the gfx950 kernels of
``libsa.so``.  There is no CPU fallback: if the library is missing or no GPU
is present the calls raise.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsa.so")

ARCH_INT_FIELDS = (
    "n_cu", "wave_size", "max_threads_per_block", "max_waves_per_cu", "max_blocks_per_cu",
    "single_wave_exempt", "simd_per_cu", "vgprs_per_simd_lane", "vgpr_granule",
    "max_vgprs_per_thread", "lds_per_cu", "lds_granule", "max_lds_per_block", "w_sat",
    "max_unroll", "max_grid",
)
ARCH_FLOAT_FIELDS = ("cpi_fp", "cpi_int", "cpi_mem", "cpi_ctrl", "cpi_sync", "cpi_reg")
VARIANT_COLUMNS = ("n_fp", "n_int", "n_ld", "n_st", "n_br", "n_bar", "n_reg", "lds_bytes", "div")
CONFIG_COLUMNS = ("seg", "block", "unroll", "regs", "grid")
K_MAX = 64

SA_OK = 0
STATUS_NAMES = {0: "SA_OK", -1: "SA_ERR_ARG", -2: "SA_ERR_ALIGN", -3: "SA_ERR_NODEV", -4: "SA_ERR_WORKSPACE",
                -5: "SA_ERR_HIP", -6: "SA_ERR_UNSUPPORTED"}

# Every function the header declares (checked by the test suite).
EXPORTED = (
    "sa_status_string", "sa_last_error", "sa_arch_gfx950", "sa_arch_default_gfx950", "sa_arch_validate",
    "sa_workspace_bytes", "sa_occupancy", "sa_score", "sa_topk", "sa_set_tile",
    "sa_plan_create", "sa_plan_destroy", "sa_plan_device_bytes", "sa_plan_bind", "sa_plan_layout", "sa_plan_info", "sa_plan_score", "sa_plan_topk",
    "sa_plan_autotune_workspace_bytes", "sa_plan_autotune", "sa_features", "sa_surrogate_fwd",
    "sa_surrogate_train_workspace_bytes", "sa_surrogate_train_step", "sa_surrogate_train_step_pairwise",
    "sa_rt_last_error", "sa_rt_grid", "sa_rt_trips", "sa_rt_buffer_floats", "sa_rt_measure", "sa_rt_cpi",
    "sa_rt_stream", "sa_rt_residency",
    "sa_suggest", "sa_score_suggested", "sa_headroom", "sa_gen_configs",
    "sa_product_workspace_bytes", "sa_score_product", "sa_score_noalloc",
)
MLP_PARAMS = 20865
MLP_FLAT = 20992
N_FEAT = 24


class SaArch(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in ARCH_INT_FIELDS] + [(f, ctypes.c_float) for f in ARCH_FLOAT_FIELDS]


class SaVariants(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in VARIANT_COLUMNS]


class SaConfigs(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in CONFIG_COLUMNS]


class SaProduct(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in ("n_block", "n_unroll", "n_regs", "n_grid")] + \
               [(f, ctypes.c_void_p) for f in ("block", "unroll", "regs", "grid")]


class SaMlp(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in ("W1", "W2", "w3", "b1", "b2", "b3", "feat_mean", "feat_inv_std")]


class SaPlanShape(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("items_per_lane", ctypes.c_int32), ("waves_per_block", ctypes.c_int32)]


class SAError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))


_lock = threading.Lock()
_lib = None


def lib():
    """Load ``libsa.so`` (built by ``__graft_entry__.build()``)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError("libsa.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
            # torch ships its own HIP runtime under the same soname as the
            # system's: loading torch first makes the library bind to that one
            # runtime.  Loaded the other way round, torch would run on the
            # system runtime and find no device.
            _torch()
            L = ctypes.CDLL(LIB_PATH)
            P, vp = ctypes.POINTER, ctypes.c_void_p
            i32, i64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
            L.sa_status_string.argtypes = [i32]
            L.sa_status_string.restype = ctypes.c_char_p
            L.sa_last_error.argtypes = []
            L.sa_last_error.restype = ctypes.c_char_p
            L.sa_arch_gfx950.argtypes = [P(SaArch)]
            L.sa_arch_gfx950.restype = i32
            L.sa_arch_default_gfx950.argtypes = [ctypes.c_int, P(SaArch)]
            L.sa_arch_default_gfx950.restype = i32
            L.sa_arch_validate.argtypes = [P(SaArch)]
            L.sa_arch_validate.restype = i32
            L.sa_workspace_bytes.argtypes = [i64, i64, i32, i32]
            L.sa_workspace_bytes.restype = sz
            L.sa_occupancy.argtypes = [P(SaArch), P(SaVariants), P(SaConfigs), i64, i64, vp, vp]
            L.sa_occupancy.restype = i32
            L.sa_score.argtypes = [P(SaArch), P(SaVariants), P(SaConfigs), i64, i64, vp, vp, i32, vp, vp,
                                   P(SaMlp), vp, sz, vp]
            L.sa_score.restype = i32
            L.sa_score_noalloc.argtypes = [P(SaArch), P(SaVariants), P(SaConfigs), i64, i64, vp, vp, i32, vp, vp,
                                           P(SaMlp), vp]
            L.sa_score_noalloc.restype = i32
            L.sa_topk.argtypes = [vp, vp, i64, i64, i32, vp, vp, vp, sz, vp]
            L.sa_topk.restype = i32
            L.sa_set_tile.argtypes = [i32]
            L.sa_set_tile.restype = i32
            PS = P(SaPlanShape)
            L.sa_plan_create.argtypes = [vp, i64, i64, i32, PS, P(vp)]
            L.sa_plan_create.restype = i32
            L.sa_plan_destroy.argtypes = [vp]
            L.sa_plan_destroy.restype = i32
            L.sa_plan_device_bytes.argtypes = [vp]
            L.sa_plan_device_bytes.restype = sz
            L.sa_plan_bind.argtypes = [vp, vp, sz, vp]
            L.sa_plan_bind.restype = i32
            L.sa_plan_layout.argtypes = [vp, i64, i64, PS, P(i64), P(i64), P(i64), vp, vp, vp]
            L.sa_plan_layout.restype = i32
            L.sa_plan_info.argtypes = [vp, PS, P(i64), P(i64), P(sz)]
            L.sa_plan_info.restype = i32
            L.sa_plan_score.argtypes = [vp, P(SaArch), P(SaVariants), P(SaConfigs), vp, vp, vp, vp, vp, sz, vp]
            L.sa_plan_score.restype = i32
            L.sa_plan_topk.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp]
            L.sa_plan_topk.restype = i32
            L.sa_plan_autotune_workspace_bytes.argtypes = [vp, i64, i64, i32]
            L.sa_plan_autotune_workspace_bytes.restype = sz
            L.sa_plan_autotune.argtypes = [vp, i64, i64, i32, P(SaArch), P(SaVariants), P(SaConfigs), vp, vp, vp, vp,
                                           vp, sz, vp, i32, PS, P(ctypes.c_float)]
            L.sa_plan_autotune.restype = i32
            L.sa_features.argtypes = [P(SaArch), P(SaVariants), P(SaConfigs), i64, i64, vp, vp]
            L.sa_features.restype = i32
            L.sa_surrogate_fwd.argtypes = [P(SaMlp), vp, i64, vp, vp]
            L.sa_surrogate_fwd.restype = i32
            L.sa_surrogate_train_workspace_bytes.argtypes = [i64]
            L.sa_surrogate_train_workspace_bytes.restype = sz
            L.sa_surrogate_train_step.argtypes = [P(SaMlp), vp, vp, vp, i64, vp, ctypes.c_float, vp, vp, i64, vp, vp,
                                                  sz, vp]
            L.sa_surrogate_train_step.restype = i32
            L.sa_surrogate_train_step_pairwise.argtypes = [P(SaMlp), vp, vp, vp, i64, vp, ctypes.c_float, vp, vp,
                                                           i64, i32, vp, vp, sz, vp]
            L.sa_surrogate_train_step_pairwise.restype = i32
            L.sa_gen_configs.argtypes = [ctypes.c_uint64, i64, i64, i32, vp, vp, vp, vp, vp]
            L.sa_gen_configs.restype = i32
            L.sa_suggest.argtypes = [P(SaArch), P(SaVariants), i64, vp, vp]
            L.sa_suggest.restype = i32
            L.sa_score_suggested.argtypes = [P(SaArch), P(SaVariants), P(SaConfigs), i64, i64, vp, vp, i32, vp, vp,
                                             vp, sz, vp]
            L.sa_score_suggested.restype = i32
            L.sa_headroom.argtypes = [P(SaArch), vp, vp, i64, vp, vp, vp]
            L.sa_headroom.restype = i32
            L.sa_product_workspace_bytes.argtypes = [i64, i64, i32]
            L.sa_product_workspace_bytes.restype = sz
            L.sa_score_product.argtypes = [P(SaArch), P(SaVariants), i64, P(SaProduct), vp, vp, i32, vp, vp, vp, sz,
                                           vp]
            L.sa_score_product.restype = i32
            L.sa_rt_last_error.restype = ctypes.c_char_p
            L.sa_rt_grid.argtypes = [i32, i64, i32, i32, i32]
            L.sa_rt_grid.restype = i64
            L.sa_rt_trips.argtypes = [i32, i64, i32, i32, i64, i32]
            L.sa_rt_trips.restype = i64
            L.sa_rt_buffer_floats.argtypes = [i32, i64, i32]
            L.sa_rt_buffer_floats.restype = sz
            L.sa_rt_measure.argtypes = [i32, i64, vp, vp, vp, vp, vp, i32, i32, i32, i32, i32, vp, vp]
            L.sa_rt_measure.restype = i32
            L.sa_rt_cpi.argtypes = [i32, i32, vp, vp, vp, vp]
            L.sa_rt_cpi.restype = i32
            L.sa_rt_stream.argtypes = [i64, vp, vp, vp, vp, vp, vp, i32, i32, i32, i32, vp, vp]
            L.sa_rt_stream.restype = i32
            L.sa_rt_residency.argtypes = [i32, i32, i32, i32, i32, vp, P(i32), vp]
            L.sa_rt_residency.restype = i32
            _lib = L
    return _lib


def _check(status: int):
    if status != SA_OK:
        raise SAError(status, lib().sa_last_error().decode())


def _arch_struct(arch: dict) -> SaArch:
    s = SaArch()
    for f in ARCH_INT_FIELDS:
        setattr(s, f, int(arch[f]))
    for f in ARCH_FLOAT_FIELDS:
        setattr(s, f, float(arch[f]))
    return s


def _arch_dict(s: SaArch) -> dict:
    d = {f: int(getattr(s, f)) for f in ARCH_INT_FIELDS}
    d.update({f: float(getattr(s, f)) for f in ARCH_FLOAT_FIELDS})
    return d


def arch_gfx950() -> dict:
    """CDNA4 / MI355X descriptor constants (no device query)."""
    s = SaArch()
    _check(lib().sa_arch_gfx950(ctypes.byref(s)))
    return _arch_dict(s)


def arch_default(device: int = 0) -> dict:
    """CDNA4 descriptor with the limits HIP reports for `device`."""
    s = SaArch()
    _check(lib().sa_arch_default_gfx950(int(device), ctypes.byref(s)))
    return _arch_dict(s)


def arch_validate(arch: dict) -> None:
    s = _arch_struct(arch)
    _check(lib().sa_arch_validate(ctypes.byref(s)))


def workspace_bytes(n_variants: int, n_evals: int, k: int) -> int:
    return int(lib().sa_workspace_bytes(int(n_variants), int(n_evals), int(k), 0))


def set_tile(evals_per_wave: int) -> None:
    _check(lib().sa_set_tile(int(evals_per_wave)))


# ------------------------------------------------------------------ tensors


def _torch():
    import torch

    return torch


def _ptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.device.type != "cuda":
        raise ValueError("%s must be a device (cuda) tensor, got %s" % (name, t.device))
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return ctypes.c_void_p(t.data_ptr()) if t.numel() > 0 else ctypes.c_void_p(t.data_ptr() or None)


def _stream(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _variants_struct(v: dict) -> SaVariants:
    torch = _torch()
    s = SaVariants()
    for f in VARIANT_COLUMNS:
        key = f if f in v else ("lds" if f == "lds_bytes" else f)
        t = v.get(key)
        if t is None and f != "n_reg":
            raise ValueError("variant column %s missing" % f)
        setattr(s, f, _ptr(t, torch.float32 if f == "div" else torch.int32, f))
    return s


def _configs_struct(c: dict) -> SaConfigs:
    torch = _torch()
    s = SaConfigs()
    for f in CONFIG_COLUMNS:
        t = c.get(f)
        if t is None and f != "grid":
            raise ValueError("configuration column %s missing" % f)
        setattr(s, f, _ptr(t, torch.int64 if f == "seg" else torch.int32, f))
    return s


def _numel(t, n: int, name: str):
    """Raise unless tensor `t` (None allowed) holds exactly `n` elements: a
    mis-sized buffer would be read or written out of bounds on the device."""
    if t is not None and int(t.numel()) != int(n):
        raise ValueError("%s holds %d elements, expected %d" % (name, int(t.numel()), int(n)))


def _variant_sizes(variants: dict) -> int:
    """Number of variants, every per-variant column checked against it."""
    t = variants.get("n_fp")
    if t is None:
        raise ValueError("variant column n_fp missing")
    n_var = int(t.numel())
    for f in VARIANT_COLUMNS:
        _numel(variants.get(f if f in variants else ("lds" if f == "lds_bytes" else f)), n_var, "variant column " + f)
    return n_var


def _sizes(variants: dict, configs: dict):
    """(n_var, n_evals) of a batch, with every column's length checked: the
    per-variant columns against n_var = seg.numel() - 1 and the configuration
    columns against n_evals = block.numel().  seg's contents (monotone, last
    entry n_evals) are a documented precondition of the C ABI: checking them
    would read device memory."""
    for f in ("seg", "block"):
        if configs.get(f) is None:
            raise ValueError("configuration column %s missing" % f)
    n_var = int(configs["seg"].numel()) - 1
    if n_var < 0:
        raise ValueError("seg must hold n_var + 1 >= 1 offsets")
    n_evals = int(configs["block"].numel())
    if _variant_sizes(variants) != n_var:
        raise ValueError("variant columns hold %d variants, seg describes %d" % (_variant_sizes(variants), n_var))
    for f in ("unroll", "regs", "grid"):
        _numel(configs.get(f), n_evals, "configuration column " + f)
    return n_var, n_evals


def _check_outputs(o: dict, n_evals: int, n_var: int, k: int):
    _numel(o.get("occ"), n_evals, "occ")
    _numel(o.get("score"), n_evals, "score")
    _numel(o.get("idx"), n_var * k, "idx")
    _numel(o.get("val"), n_var * k, "val")


def occupancy(arch: dict, variants: dict, configs: dict, out=None, stream=None):
    """W* (active waves per CU, Eqs. 1-5) of every evaluation (int32)."""
    torch = _torch()
    n_var, n_evals = _sizes(variants, configs)
    if out is None:
        out = torch.empty(n_evals, dtype=torch.int32, device=configs["block"].device)
    _numel(out, n_evals, "out")
    a = _arch_struct(arch)
    _check(lib().sa_occupancy(ctypes.byref(a), ctypes.byref(_variants_struct(variants)),
                              ctypes.byref(_configs_struct(configs)), n_var, n_evals,
                              _ptr(out, torch.int32, "out"), _stream(stream)))
    return out


class Workspace:
    """Device workspace for sa_score / sa_topk (256-byte aligned torch buffer)."""

    def __init__(self, nbytes: int, device):
        torch = _torch()
        self.nbytes = int(nbytes)
        self.buf = torch.empty(max(self.nbytes + 256, 256), dtype=torch.uint8, device=device)
        base = self.buf.data_ptr()
        self.offset = (-base) % 256
        self.ptr = ctypes.c_void_p(base + self.offset) if self.nbytes > 0 else None


def score(arch: dict, variants: dict, configs: dict, k: int = 8, *, want_score: bool = True,
          want_occ: bool = True, want_topk: bool = True, outputs: dict | None = None,
          workspace: Workspace | None = None, stream=None, mlp: "Surrogate | None" = None) -> dict:
    """Occupancy, score and per-variant top-k in one pass (sa_score).

    Returns a dict with ``occ`` (int32[n_evals]), ``score`` (float32[n_evals]),
    ``idx`` (int32[n_var, k]) and ``val`` (float32[n_var, k]); entries not
    requested are None.  `outputs` may supply preallocated tensors.  With
    `mlp` (a Surrogate) the pass is the corrected one: ``score`` holds the
    corrected key z = ln(score) + Delta and the top-k ranks by z.
    """
    torch = _torch()
    n_var, n_evals = _sizes(variants, configs)
    dev = configs["seg"].device
    o = dict(outputs or {})
    if want_occ and o.get("occ") is None:
        o["occ"] = torch.empty(n_evals, dtype=torch.int32, device=dev)
    if want_score and o.get("score") is None:
        o["score"] = torch.empty(n_evals, dtype=torch.float32, device=dev)
    if want_topk:
        if o.get("idx") is None:
            o["idx"] = torch.empty((n_var, k), dtype=torch.int32, device=dev)
        if o.get("val") is None:
            o["val"] = torch.empty((n_var, k), dtype=torch.float32, device=dev)
        if workspace is None:
            workspace = Workspace(workspace_bytes(n_var, n_evals, k), dev)
    for key in ("occ", "score", "idx", "val"):
        o.setdefault(key, None)
    _check_outputs({key: o[key] for key, want in (("occ", want_occ), ("score", want_score), ("idx", want_topk),
                                                 ("val", want_topk)) if want}, n_evals, n_var, k)
    a = _arch_struct(arch)
    ws_ptr = workspace.ptr if (want_topk and workspace is not None) else None
    ws_bytes = workspace.nbytes if (want_topk and workspace is not None) else 0
    _check(lib().sa_score(ctypes.byref(a), ctypes.byref(_variants_struct(variants)),
                          ctypes.byref(_configs_struct(configs)), n_var, n_evals,
                          _ptr(o["score"] if want_score else None, torch.float32, "score"),
                          _ptr(o["occ"] if want_occ else None, torch.int32, "occ"), int(k) if want_topk else 0,
                          _ptr(o["idx"] if want_topk else None, torch.int32, "idx"),
                          _ptr(o["val"] if want_topk else None, torch.float32, "val"),
                          None if mlp is None else ctypes.byref(mlp.struct()), ws_ptr, ws_bytes, _stream(stream)))
    return o


def suggest(arch: dict, variants: dict, out=None, stream=None):
    """The paper's reduced search space per variant (sa_suggest): int64
    tensor whose bit j keeps the block size wave_size * (j + 1)."""
    torch = _torch()
    n_var = _variant_sizes(variants)
    if out is None:
        out = torch.zeros(n_var, dtype=torch.int64, device=variants["n_fp"].device)
    _numel(out, n_var, "kept")
    a = _arch_struct(arch)
    _check(lib().sa_suggest(ctypes.byref(a), ctypes.byref(_variants_struct(variants)), n_var,
                            _ptr(out, torch.int64, "kept"), _stream(stream)))
    return out


PRODUCT_DIMS = ("block", "unroll", "regs", "grid")


def product_size(space: dict) -> int:
    """Configurations per variant of a product space (grid optional)."""
    n = 1
    for d in PRODUCT_DIMS:
        if space.get(d) is not None:
            n *= len(space[d])
    return n


def score_product(arch: dict, variants: dict, space: dict, k: int = 8, *, want_score: bool = True,
                  want_occ: bool = True, want_topk: bool = True, outputs: dict | None = None,
                  workspace: "Workspace | None" = None, stream=None) -> dict:
    """sa_score over the product space `space` (dict of value lists for
    block, unroll, regs and optionally grid; block slowest, grid fastest)
    shared by every variant, without configuration rows (sa_score_product).
    Per-evaluation outputs are indexed v * S + i."""
    torch = _torch()
    n_var = _variant_sizes(variants)
    dev = variants["n_fp"].device
    S = product_size(space)
    n = n_var * S
    lists = {d: None if space.get(d) is None else np.ascontiguousarray(space[d], dtype=np.int32) for d in PRODUCT_DIMS}
    ps = SaProduct(*[0 if lists[d] is None else int(lists[d].size) for d in PRODUCT_DIMS],
                   *[None if lists[d] is None else lists[d].ctypes.data_as(ctypes.c_void_p) for d in PRODUCT_DIMS])
    o = dict(outputs or {})
    if want_occ and o.get("occ") is None:
        o["occ"] = torch.empty(n, dtype=torch.int32, device=dev)
    if want_score and o.get("score") is None:
        o["score"] = torch.empty(n, dtype=torch.float32, device=dev)
    if want_topk:
        if o.get("idx") is None:
            o["idx"] = torch.empty((n_var, k), dtype=torch.int32, device=dev)
        if o.get("val") is None:
            o["val"] = torch.empty((n_var, k), dtype=torch.float32, device=dev)
    if workspace is None and want_topk:
        workspace = Workspace(int(lib().sa_product_workspace_bytes(n_var, S, int(k))), dev)
    for key in ("occ", "score", "idx", "val"):
        o.setdefault(key, None)
    _check_outputs({key: o[key] for key, want in (("occ", want_occ), ("score", want_score), ("idx", want_topk),
                                                 ("val", want_topk)) if want}, n, n_var, k)
    a = _arch_struct(arch)
    _check(lib().sa_score_product(ctypes.byref(a), ctypes.byref(_variants_struct(variants)), n_var, ctypes.byref(ps),
                                  _ptr(o["score"] if want_score else None, torch.float32, "score"),
                                  _ptr(o["occ"] if want_occ else None, torch.int32, "occ"), int(k),
                                  _ptr(o["idx"] if want_topk else None, torch.int32, "idx"),
                                  _ptr(o["val"] if want_topk else None, torch.float32, "val"),
                                  workspace.ptr if workspace is not None else None,
                                  workspace.nbytes if workspace is not None else 0, _stream(stream)))
    return o


def headroom(arch: dict, block, regs=None, stream=None):
    """Registers per thread still free (R*) and LDS per workgroup (S*) at
    full occupancy for each row's block size (sa_headroom): two int32
    tensors."""
    torch = _torch()
    n = int(block.numel())
    _numel(regs, n, "regs")
    r_star = torch.empty(n, dtype=torch.int32, device=block.device)
    s_star = torch.empty(n, dtype=torch.int32, device=block.device)
    a = _arch_struct(arch)
    _check(lib().sa_headroom(ctypes.byref(a), _ptr(block, torch.int32, "block"), _ptr(regs, torch.int32, "regs"), n,
                             _ptr(r_star, torch.int32), _ptr(s_star, torch.int32), _stream(stream)))
    return r_star, s_star


def rt_stream(cols, outs, *, items: int = 1, blocks_per_cu: int = 0, nontemporal: bool = False, reps: int = 5,
              stream=None) -> float:
    """Median milliseconds of a pure stream of a scoring pass's traffic
    (sa_rt_stream): four int32 columns read, outs[0] = c0 + c1 and
    outs[1] = c2 ^ c3 written."""
    torch = _torch()
    n = int(cols[0].numel())
    if len(cols) != 4 or len(outs) != 2:
        raise ValueError("rt_stream takes four columns and two outputs")
    for i, t in enumerate(list(cols) + list(outs)):
        _numel(t, n, "stream buffer %d" % i)
    ms = ctypes.c_float(0.0)
    st = lib().sa_rt_stream(n, *[_ptr(c, torch.int32, "column") for c in cols],
                            *[_ptr(o, torch.int32, "output") for o in outs], int(items), int(blocks_per_cu),
                            int(bool(nontemporal)), int(reps), ctypes.byref(ms), _stream(stream))
    if st != 0:
        raise SAError(st, lib().sa_rt_last_error().decode())
    return float(ms.value)


def score_suggested(arch: dict, variants: dict, configs: dict, k: int = 8, *, want_score: bool = False,
                    want_occ: bool = False, workspace: Workspace | None = None, stream=None) -> dict:
    """Top-k by score within the paper's reduced search space (sa_score_suggested)."""
    torch = _torch()
    n_var, n_evals = _sizes(variants, configs)
    dev = configs["seg"].device
    o = {"occ": torch.empty(n_evals, dtype=torch.int32, device=dev) if want_occ else None,
         "score": torch.empty(n_evals, dtype=torch.float32, device=dev) if want_score else None,
         "idx": torch.empty((n_var, k), dtype=torch.int32, device=dev),
         "val": torch.empty((n_var, k), dtype=torch.float32, device=dev)}
    if workspace is None:
        workspace = Workspace(workspace_bytes(n_var, n_evals, k), dev)
    _check_outputs(o, n_evals, n_var, k)
    a = _arch_struct(arch)
    _check(lib().sa_score_suggested(ctypes.byref(a), ctypes.byref(_variants_struct(variants)),
                                    ctypes.byref(_configs_struct(configs)), n_var, n_evals,
                                    _ptr(o["score"], torch.float32, "score"), _ptr(o["occ"], torch.int32, "occ"),
                                    int(k), _ptr(o["idx"], torch.int32, "idx"), _ptr(o["val"], torch.float32, "val"),
                                    workspace.ptr, workspace.nbytes, _stream(stream)))
    return o


def topk(keys, seg, k: int, *, workspace: Workspace | None = None, stream=None):
    """Segmented top-k of float keys (sa_topk): (idx int32[n_var,k], val float32[n_var,k])."""
    torch = _torch()
    n_var = int(seg.numel()) - 1
    n_evals = int(keys.numel())
    idx = torch.empty((n_var, k), dtype=torch.int32, device=seg.device)
    val = torch.empty((n_var, k), dtype=torch.float32, device=seg.device)
    if workspace is None:
        workspace = Workspace(workspace_bytes(n_var, n_evals, k), seg.device)
    _check(lib().sa_topk(_ptr(keys, torch.float32, "keys"), _ptr(seg, torch.int64, "seg"), n_var, n_evals, int(k),
                         _ptr(idx, torch.int32, "idx"), _ptr(val, torch.float32, "val"), workspace.ptr,
                         workspace.nbytes, _stream(stream)))
    return idx, val


def device_batch(batch, device="cuda") -> tuple[dict, dict]:
    """Copy a ``workloads.Batch`` to device tensors: (variants, configs)."""
    torch = _torch()
    var = {}
    for f in ("n_fp", "n_int", "n_ld", "n_st", "n_br", "n_bar", "n_reg", "lds", "div"):
        a = batch.variants[f]
        var["lds_bytes" if f == "lds" else f] = torch.from_numpy(np.ascontiguousarray(a)).to(device)
    cfg = {"seg": torch.from_numpy(np.ascontiguousarray(batch.seg, dtype=np.int64)).to(device)}
    for f in ("block", "unroll", "regs", "grid"):
        a = getattr(batch, f)
        cfg[f] = None if a is None else torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(device)
    return var, cfg


# ------------------------------------------------------------------ plans


def _shape(shape):
    if shape is None:
        return None
    if isinstance(shape, SaPlanShape):
        return shape
    t, i, w = shape
    return SaPlanShape(int(t), int(i), int(w))


def _seg_host(seg) -> np.ndarray:
    if hasattr(seg, "detach"):
        seg = seg.detach().cpu().numpy()
    return np.ascontiguousarray(seg, dtype=np.int64)


def plan_layout(seg, shape=None) -> dict:
    """The decomposition a plan would use, computed on the host."""
    sh = _seg_host(seg)
    n_var, n_evals = sh.shape[0] - 1, int(sh[-1])
    ni, ns, nsl = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    s = _shape(shape)
    sp = ctypes.byref(s) if s is not None else None
    vp = sh.ctypes.data_as(ctypes.c_void_p)
    _check(lib().sa_plan_layout(vp, n_var, n_evals, sp, ctypes.byref(ni), ctypes.byref(ns), ctypes.byref(nsl),
                                None, None, None))
    wpb = (s.waves_per_block if s is not None else 4)
    items = np.zeros((ni.value, 3), np.int64)
    waves = np.zeros((ni.value, wpb, 4), np.int64)
    splits = np.zeros((ns.value, 3), np.int64)
    _check(lib().sa_plan_layout(vp, n_var, n_evals, sp, ctypes.byref(ni), ctypes.byref(ns), ctypes.byref(nsl),
                                items.ctypes.data_as(ctypes.c_void_p), waves.ctypes.data_as(ctypes.c_void_p),
                                splits.ctypes.data_as(ctypes.c_void_p)))
    return {"items": items, "waves": waves, "splits": splits, "n_slots": nsl.value, "wpb": wpb}


class Plan:
    """A persistent-kernel plan for one CSR layout (sa_plan_*): the host
    decomposition, bound to a device table this object allocates as a torch
    buffer on `device` (the library allocates nothing)."""

    def __init__(self, seg, k: int = 8, shape=None, device=None, stream=None):
        sh = _seg_host(seg)
        self.n_var, self.n_evals, self.k = sh.shape[0] - 1, int(sh[-1]), int(k)
        h = ctypes.c_void_p()
        s = _shape(shape)
        _check(lib().sa_plan_create(sh.ctypes.data_as(ctypes.c_void_p), self.n_var, self.n_evals, self.k,
                                    ctypes.byref(s) if s is not None else None, ctypes.byref(h)))
        self._h = h
        info_shape = SaPlanShape()
        ni, ns, wb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()
        _check(lib().sa_plan_info(self._h, ctypes.byref(info_shape), ctypes.byref(ni), ctypes.byref(ns),
                                  ctypes.byref(wb)))
        self.shape = (info_shape.tile, info_shape.items_per_lane, info_shape.waves_per_block)
        self.n_items, self.n_splits, self.workspace_bytes = ni.value, ns.value, wb.value
        torch = _torch()
        if device is None:
            device = seg.device if isinstance(seg, torch.Tensor) and seg.device.type == "cuda" else "cuda"
        self.table = Workspace(int(lib().sa_plan_device_bytes(self._h)), device)
        _check(lib().sa_plan_bind(self._h, self.table.ptr, self.table.nbytes, _stream(stream)))
        # the copy reads this plan's host memory: let it finish here, so that
        # closing the plan later never races it
        (_torch().cuda.current_stream() if stream is None else stream).synchronize()

    def close(self):
        if getattr(self, "_h", None):
            lib().sa_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def score(self, arch: dict, variants: dict, configs: dict, *, want_score=True, want_occ=True, want_topk=True,
              outputs: dict | None = None, workspace: Workspace | None = None, stream=None) -> dict:
        torch = _torch()
        dev = configs["seg"].device
        if _sizes(variants, configs) != (self.n_var, self.n_evals):
            raise ValueError("batch of %d variants / %d evaluations, plan made for %d / %d"
                             % (*_sizes(variants, configs), self.n_var, self.n_evals))
        o = dict(outputs or {})
        if want_occ and o.get("occ") is None:
            o["occ"] = torch.empty(self.n_evals, dtype=torch.int32, device=dev)
        if want_score and o.get("score") is None:
            o["score"] = torch.empty(self.n_evals, dtype=torch.float32, device=dev)
        if want_topk:
            if o.get("idx") is None:
                o["idx"] = torch.empty((self.n_var, self.k), dtype=torch.int32, device=dev)
            if o.get("val") is None:
                o["val"] = torch.empty((self.n_var, self.k), dtype=torch.float32, device=dev)
        if workspace is None:
            workspace = Workspace(self.workspace_bytes, dev)
        for key in ("occ", "score", "idx", "val"):
            o.setdefault(key, None)
        _check_outputs({key: o[key] for key, want in (("occ", want_occ), ("score", want_score), ("idx", want_topk),
                                                     ("val", want_topk)) if want}, self.n_evals, self.n_var, self.k)
        a = _arch_struct(arch)
        _check(lib().sa_plan_score(self._h, ctypes.byref(a), ctypes.byref(_variants_struct(variants)),
                                   ctypes.byref(_configs_struct(configs)),
                                   _ptr(o["score"] if want_score else None, torch.float32, "score"),
                                   _ptr(o["occ"] if want_occ else None, torch.int32, "occ"),
                                   _ptr(o["idx"] if want_topk else None, torch.int32, "idx"),
                                   _ptr(o["val"] if want_topk else None, torch.float32, "val"),
                                   workspace.ptr, workspace.nbytes, _stream(stream)))
        return o

    def topk(self, keys, seg, *, workspace: Workspace | None = None, stream=None):
        torch = _torch()
        _numel(keys, self.n_evals, "keys")
        _numel(seg, self.n_var + 1, "seg")
        idx = torch.empty((self.n_var, self.k), dtype=torch.int32, device=seg.device)
        val = torch.empty((self.n_var, self.k), dtype=torch.float32, device=seg.device)
        if workspace is None:
            workspace = Workspace(self.workspace_bytes, seg.device)
        _check(lib().sa_plan_topk(self._h, _ptr(keys, torch.float32, "keys"), _ptr(seg, torch.int64, "seg"),
                                  _ptr(idx, torch.int32, "idx"), _ptr(val, torch.float32, "val"), workspace.ptr,
                                  workspace.nbytes, _stream(stream)))
        return idx, val


def autotune(arch: dict, variants: dict, configs: dict, k: int = 8, reps: int = 3, outputs: dict | None = None,
             stream=None, want_score: bool = True, want_occ: bool = True):
    """Fastest plan shape for this batch (sa_plan_autotune): (shape, ms).
    Timed with the outputs a later scoring pass writes (per-evaluation score
    and occupancy only when asked for)."""
    torch = _torch()
    sh = _seg_host(configs["seg"])
    n_var, n_evals = sh.shape[0] - 1, int(sh[-1])
    dev = configs["seg"].device
    o = dict(outputs or {})
    if want_occ:
        o.setdefault("occ", torch.empty(n_evals, dtype=torch.int32, device=dev))
    if want_score:
        o.setdefault("score", torch.empty(n_evals, dtype=torch.float32, device=dev))
    o.setdefault("occ", None)
    o.setdefault("score", None)
    o.setdefault("idx", torch.empty((n_var, k), dtype=torch.int32, device=dev))
    o.setdefault("val", torch.empty((n_var, k), dtype=torch.float32, device=dev))
    if _sizes(variants, configs) != (n_var, n_evals):
        raise ValueError("configuration columns do not match seg")
    _check_outputs(o, n_evals, n_var, k)
    ws = Workspace(int(lib().sa_plan_autotune_workspace_bytes(sh.ctypes.data_as(ctypes.c_void_p), n_var, n_evals,
                                                              int(k))), dev)
    best = SaPlanShape()
    ms = ctypes.c_float()
    a = _arch_struct(arch)
    _check(lib().sa_plan_autotune(sh.ctypes.data_as(ctypes.c_void_p), n_var, n_evals, int(k), ctypes.byref(a),
                                  ctypes.byref(_variants_struct(variants)), ctypes.byref(_configs_struct(configs)),
                                  _ptr(o["score"], torch.float32), _ptr(o["occ"], torch.int32),
                                  _ptr(o["idx"], torch.int32), _ptr(o["val"], torch.float32), ws.ptr, ws.nbytes,
                                  _stream(stream), int(reps), ctypes.byref(best), ctypes.byref(ms)))
    return (best.tile, best.items_per_lane, best.waves_per_block), float(ms.value)


# ------------------------------------------------------------------ learned correction

# offsets of the flat fp32 parameter vector
FLAT_W1, FLAT_B1 = 0, 128 * 32
FLAT_W2 = FLAT_B1 + 128
FLAT_B2 = FLAT_W2 + 128 * 128
FLAT_W3 = FLAT_B2 + 128
FLAT_B3 = FLAT_W3 + 128


def features(arch: dict, variants: dict, configs: dict, out=None, stream=None):
    """The 24 features of every evaluation (float32 [n_evals, 24])."""
    torch = _torch()
    n_var, n_evals = _sizes(variants, configs)
    if out is None:
        out = torch.empty((n_evals, N_FEAT), dtype=torch.float32, device=configs["seg"].device)
    _numel(out, n_evals * N_FEAT, "out")
    a = _arch_struct(arch)
    _check(lib().sa_features(ctypes.byref(a), ctypes.byref(_variants_struct(variants)),
                             ctypes.byref(_configs_struct(configs)), n_var, n_evals, _ptr(out, torch.float32, "out"),
                             _stream(stream)))
    return out


def _feature_rows(feat) -> int:
    """Rows of a feature matrix, which must be (n, 24)."""
    if feat.dim() != 2 or int(feat.shape[1]) != N_FEAT:
        raise ValueError("features must have shape (n, %d), got %s" % (N_FEAT, tuple(feat.shape)))
    return int(feat.shape[0])


def flat_from_params(p: dict):
    """Pack a dict of numpy parameters (W1 128x32, b1, W2, b2, w3, b3) into the
    flat float32 layout."""
    flat = np.zeros(MLP_FLAT, np.float32)
    flat[FLAT_W1:FLAT_B1] = np.asarray(p["W1"], np.float32).reshape(-1)
    flat[FLAT_B1:FLAT_W2] = p["b1"]
    flat[FLAT_W2:FLAT_B2] = np.asarray(p["W2"], np.float32).reshape(-1)
    flat[FLAT_B2:FLAT_W3] = p["b2"]
    flat[FLAT_W3:FLAT_B3] = p["w3"]
    flat[FLAT_B3] = np.asarray(p["b3"]).reshape(-1)[0]
    return flat


def params_from_flat(flat) -> dict:
    f = np.asarray(flat, np.float32)
    return {"W1": f[FLAT_W1:FLAT_B1].reshape(128, 32).copy(), "b1": f[FLAT_B1:FLAT_W2].copy(),
            "W2": f[FLAT_W2:FLAT_B2].reshape(128, 128).copy(), "b2": f[FLAT_B2:FLAT_W3].copy(),
            "w3": f[FLAT_W3:FLAT_B3].copy(), "b3": f[FLAT_B3:FLAT_B3 + 1].copy()}


class Surrogate:
    """Device state of the learned correction: fp32 master weights and Adam
    moments (flat layout), the bf16 shadow the kernels read, and the
    feature normalisation."""

    def __init__(self, params: dict, mean, inv_std, device="cuda"):
        torch = _torch()
        self.device = torch.device(device)
        flat = flat_from_params(params)
        self.master = torch.from_numpy(flat).to(self.device)
        self.m = torch.zeros(MLP_FLAT, dtype=torch.float32, device=self.device)
        self.v = torch.zeros(MLP_FLAT, dtype=torch.float32, device=self.device)
        self.grad = torch.zeros(MLP_FLAT, dtype=torch.float32, device=self.device)
        self.mean = torch.as_tensor(np.asarray(mean, np.float32), device=self.device).contiguous()
        self.inv_std = torch.as_tensor(np.asarray(inv_std, np.float32), device=self.device).contiguous()
        self.step_count = 0
        # device-side step count for steps replayed from a captured graph
        self.steps_dev = torch.zeros(1, dtype=torch.int64, device=self.device)
        self.W1 = torch.empty((128, 32), dtype=torch.bfloat16, device=self.device)
        self.W2 = torch.empty((128, 128), dtype=torch.bfloat16, device=self.device)
        self.w3 = torch.empty(128, dtype=torch.bfloat16, device=self.device)
        self.b1 = torch.empty(128, dtype=torch.float32, device=self.device)
        self.b2 = torch.empty(128, dtype=torch.float32, device=self.device)
        self.b3 = torch.empty(1, dtype=torch.float32, device=self.device)
        self.refresh_shadow()
        self._ws = None

    def refresh_shadow(self):
        """bf16 shadow and biases from the master weights (round to nearest even)."""
        mst = self.master
        self.W1.copy_(mst[FLAT_W1:FLAT_B1].view(128, 32).to(self.W1.dtype))
        self.W2.copy_(mst[FLAT_W2:FLAT_B2].view(128, 128).to(self.W2.dtype))
        self.w3.copy_(mst[FLAT_W3:FLAT_B3].to(self.w3.dtype))
        self.b1.copy_(mst[FLAT_B1:FLAT_W2])
        self.b2.copy_(mst[FLAT_B2:FLAT_W3])
        self.b3.copy_(mst[FLAT_B3:FLAT_B3 + 1])

    def struct(self) -> SaMlp:
        p = lambda t: ctypes.c_void_p(t.data_ptr())
        return SaMlp(p(self.W1), p(self.W2), p(self.w3), p(self.b1), p(self.b2), p(self.b3), p(self.mean),
                     p(self.inv_std))

    def forward(self, feat, out=None, stream=None):
        torch = _torch()
        n = _feature_rows(feat)
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=feat.device)
        _numel(out, n, "out")
        m = self.struct()
        _check(lib().sa_surrogate_fwd(ctypes.byref(m), _ptr(feat, torch.float32, "feat"), n,
                                      _ptr(out, torch.float32, "out"), _stream(stream)))
        return out

    def reserve(self, n: int):
        """Allocate the training workspace for batches of up to n rows now
        (before a graph capture, which must not allocate it)."""
        need = int(lib().sa_surrogate_train_workspace_bytes(int(n)))
        if need and (self._ws is None or self._ws.nbytes < need):
            self._ws = Workspace(need, self.device)

    def train_step(self, feat, target, lr: float = 1e-3, stream=None, group: int = 0, device_counter: bool = False):
        """One Adam step on the batch; returns the batch loss (0-d device
        tensor).  group = 0: squared error against `target` (the residual);
        group > 0: pairwise ranking loss over groups of `group` consecutive
        rows with `target` the measured log runtime
        (sa_surrogate_train_step_pairwise).  device_counter: Adam's step
        number comes from (and advances) `steps_dev` on the device, so the
        call can be captured in a graph and replayed; set steps_dev from
        step_count before the first such step."""
        torch = _torch()
        n = _feature_rows(feat)
        _numel(target, n, "target")
        self.reserve(n)
        ws_ptr, ws_bytes = (self._ws.ptr, self._ws.nbytes) if self._ws is not None else (None, 0)
        m = self.struct()
        step = 0 if device_counter else self.step_count + 1
        counter = _ptr(self.steps_dev, torch.int64, "steps_dev") if device_counter else None
        common = (ctypes.byref(m), _ptr(self.master, torch.float32), _ptr(self.m, torch.float32),
                  _ptr(self.v, torch.float32), step, counter, float(lr), _ptr(feat, torch.float32, "feat"),
                  _ptr(target, torch.float32, "target"), n)
        if group > 0:
            _check(lib().sa_surrogate_train_step_pairwise(*common, int(group), _ptr(self.grad, torch.float32), ws_ptr,
                                                          ws_bytes, _stream(stream)))
        else:
            _check(lib().sa_surrogate_train_step(*common, _ptr(self.grad, torch.float32), ws_ptr, ws_bytes,
                                                 _stream(stream)))
        if not device_counter:
            # with the device counter the step happens when the stream (or a
            # graph replay) runs it: the caller advances step_count then
            self.step_count += 1
        return self.grad[MLP_PARAMS]

    def params(self) -> dict:
        return params_from_flat(self.master.cpu().numpy())

    def state_dict(self) -> dict:
        return {"master": self.master.cpu().numpy(), "m": self.m.cpu().numpy(), "v": self.v.cpu().numpy(),
                "step": self.step_count, "mean": self.mean.cpu().numpy(), "inv_std": self.inv_std.cpu().numpy()}

    @classmethod
    def from_state(cls, st: dict, device="cuda"):
        s = cls(params_from_flat(st["master"]), st["mean"], st["inv_std"], device)
        torch = _torch()
        s.m.copy_(torch.from_numpy(np.asarray(st["m"], np.float32)))
        s.v.copy_(torch.from_numpy(np.asarray(st["v"], np.float32)))
        s.step_count = int(st["step"])
        return s
