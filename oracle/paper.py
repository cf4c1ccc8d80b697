"""The paper's rule-based search-space reduction -- TEST INFRASTRUCTURE ONLY.

Sec. III-C and Sec. IV-C: from the occupancy model the static analyser
suggests the thread counts that reach full theoretical occupancy (T*), how
many more registers per thread (R*) and how much shared memory per block (S*)
keep that occupancy, and then keeps the upper or the lower half of T*
depending on whether the kernel's intensity (floating-point operations per
memory operation, Sec. IV-B) exceeds 4.0.  Everything here is built on the
C oracle's occupancy of Eqs. 1-5, so checking these against the values the
paper prints (Table VII and the pruning percentages of Sec. IV-C) pins that
engine.
"""
from __future__ import annotations

import math

from . import occupancy


def full(arch: dict, T: int, R: int = 0, S: int = 0) -> bool:
    return occupancy(arch, T, R, S) == arch["max_waves_per_cu"]


def suggested_threads(arch: dict, candidates=range(32, 1025, 32)) -> list[int]:
    """T*: thread counts at which occupancy is 1 when registers and shared
    memory do not limit (Eqs. 2-3)."""
    return [T for T in candidates if full(arch, T)]


def max_registers_at_full(arch: dict, T: int) -> int:
    """Largest registers per thread that keeps occupancy 1 at T threads."""
    best = 0
    for R in range(1, arch["max_vgprs_per_thread"] + 1):
        if full(arch, T, R):
            best = R
    return best


def register_headroom(arch: dict, T: int, R_used: int) -> int:
    """R* of Table VII: registers that could still be added, clipped at 0."""
    return max(0, max_registers_at_full(arch, T) - R_used)


def max_shared_at_full(arch: dict, T: int) -> int:
    """Largest shared memory per block that keeps occupancy 1 at T threads
    (binary search; occupancy never rises with S)."""
    if not full(arch, T):
        return 0
    lo, hi = 0, arch["max_lds_per_block"]
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if full(arch, T, 0, mid):
            lo = mid
        else:
            hi = mid - 1
    return lo


def intensity(n_fp: float, n_mem: float) -> float:
    """Floating-point operations per memory operation."""
    return n_fp / max(1.0, n_mem)


def rule(t_star: list[int], inten: float, threshold: float = 4.0) -> list[int]:
    """Keep the upper half of T* when intensity > threshold, else the lower
    half; an odd-length list drops its median (each half has floor(n/2))."""
    h = len(t_star) // 2
    return list(t_star[len(t_star) - h:]) if inten > threshold else list(t_star[:h])


def space_size(*dims: int) -> int:
    return math.prod(dims)
