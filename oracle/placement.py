"""Block-by-block residency simulator -- TEST INFRASTRUCTURE ONLY.

An independent formulation of the occupancy bound (Sec. III-A, Eqs. 1-5):
instead of the closed-form minimum of per-resource bounds, it places blocks
one at a time on a model of one compute unit -- wave slots and register file
per SIMD partition, a shared-memory pool, block slots -- and counts how many
fit.  Used only on small grids of (T, R, S), where it is cheap.
"""
from __future__ import annotations


def _round_up(x: int, g: int) -> int:
    return -(-x // g) * g


def resident_blocks(arch: dict, T: int, R: int, S: int, limit: int = 4096) -> int:
    """Largest number of blocks of T threads, R registers per thread and S
    bytes of shared memory that one CU holds at once."""
    if T < 1 or T > arch["max_threads_per_block"] or R < 0 or S < 0:
        return 0
    if R > arch["max_vgprs_per_thread"] or S > arch["max_lds_per_block"]:
        return 0
    waves_per_block = -(-T // arch["wave_size"])
    regs_per_wave = _round_up(R, arch["vgpr_granule"]) if R > 0 else 0
    lds_per_block = _round_up(S, arch["lds_granule"]) if S > 0 else 0
    p = arch["simd_per_cu"]
    simds = [[arch["max_waves_per_cu"] // p, arch["vgprs_per_simd_lane"]] for _ in range(p)]
    lds_free = arch["lds_per_cu"]
    counted = not (waves_per_block == 1 and arch["single_wave_exempt"])
    blocks = 0
    while blocks < limit:
        if counted and blocks >= arch["max_blocks_per_cu"]:
            break
        if lds_per_block > lds_free:
            break
        trial = [list(s) for s in simds]
        placed = 0
        for _ in range(waves_per_block):
            fits = [s for s in trial if s[0] > 0 and s[1] >= regs_per_wave]
            if not fits:
                break
            best = max(fits, key=lambda s: (s[0], s[1]))
            best[0] -= 1
            best[1] -= regs_per_wave
            placed += 1
        if placed < waves_per_block:
            break
        simds = trial
        lds_free -= lds_per_block
        blocks += 1
    return blocks


def resident_waves(arch: dict, T: int, R: int, S: int) -> int:
    return resident_blocks(arch, T, R, S) * (-(-T // arch["wave_size"]) if T >= 1 else 0)
