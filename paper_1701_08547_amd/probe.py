"""Residency probe of the device limits behind the occupancy bound (Sec.
III-A, Eqs. 1-5; the per-multiprocessor limits of Table I).

``residency`` runs the library's probe kernels (sa_rt_residency) and
reduces their per-workgroup records on the host: records of one compute
unit (same XCC, shader engine, array and CU id) are [start, end) intervals,
and the largest number of them that overlap is the number of workgroups the
unit held at once.  W* of the probe is that count times the waves per
workgroup, the quantity Eq. 2 predicts.
"""
from __future__ import annotations

import ctypes

import numpy as np

# (block rounded up to 64, vgprs) pairs the library has probe kernels for
PROBES = {64: (16, 24, 64, 72, 80, 128, 256, 512), 128: (16, 64, 256), 192: (16, 96, 168), 256: (64, 128),
          320: (16, 96, 168), 384: (16, 128), 448: (16,), 512: (80,), 576: (16,), 640: (16,), 768: (16,), 960: (16,),
          1024: (64, 128)}


def cu_key(hw_id: np.ndarray, xcc_id: np.ndarray) -> np.ndarray:
    """One key per compute unit: XCC id and the CU, array and shader-engine
    fields of HW_ID (bits 8..15)."""
    return (np.asarray(xcc_id, np.int64) & 0xF) * 256 + ((np.asarray(hw_id, np.int64) >> 8) & 0xFF)


def max_overlap(start: np.ndarray, end: np.ndarray) -> int:
    """Largest number of [start, end) intervals containing one point (an
    interval that ends when another starts does not overlap it)."""
    if len(start) == 0:
        return 0
    t = np.concatenate([np.asarray(end, np.int64), np.asarray(start, np.int64)])
    d = np.concatenate([-np.ones(len(end), np.int64), np.ones(len(start), np.int64)])
    order = np.lexsort((d, t))  # by time, ends (-1) before starts (+1)
    return int(np.cumsum(d[order]).max())


def concurrency(records: np.ndarray) -> dict:
    """Per-CU largest overlap of a probe's records (int64 [n, 4]: start, end,
    HW_ID, XCC_ID)."""
    r = np.asarray(records, np.int64).reshape(-1, 4)
    keys = cu_key(r[:, 2], r[:, 3])
    per_cu = {}
    for k in np.unique(keys):
        m = keys == k
        per_cu[int(k)] = max_overlap(r[m, 0], r[m, 1])
    vals = np.array(sorted(per_cu.values()), np.int64)
    if len(vals) == 0:
        return {"cus": 0, "max": 0, "mode": 0, "per_cu": per_cu}
    uniq, counts = np.unique(vals, return_counts=True)
    return {"cus": len(per_cu), "max": int(vals.max()), "mode": int(uniq[np.argmax(counts)]),
            "min": int(vals.min()), "per_cu": per_cu}


def residency(block: int, vgprs: int, lds_bytes: int, n_cu: int, spin_us: int = 200, device="cuda") -> dict:
    """Run one probe (enough workgroups to fill every CU twice over) and
    reduce it: the workgroups one CU held at once (largest and most common
    over the CUs), the CUs seen, and HIP's occupancy API for the same
    kernel."""
    import torch

    from . import api

    waves = -(-int(block) // 64)
    n_blocks = int(n_cu) * 2 * (32 // waves + 1)
    rec = torch.zeros((n_blocks, 4), dtype=torch.int64, device=device)
    api_nb = ctypes.c_int32(-1)
    st = api.lib().sa_rt_residency(int(block), int(vgprs), int(lds_bytes), n_blocks, int(spin_us),
                                   ctypes.c_void_p(rec.data_ptr()), ctypes.byref(api_nb), api._stream(None))
    if st != 0:
        raise api.SAError(st, api.lib().sa_rt_last_error().decode())
    torch.cuda.synchronize()
    c = concurrency(rec.cpu().numpy())
    c.update({"block": int(block), "vgprs": int(vgprs), "lds_bytes": int(lds_bytes), "waves_per_block": waves,
              "n_blocks": n_blocks, "api_blocks_per_cu": int(api_nb.value)})
    return c
