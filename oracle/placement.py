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
    bytes of shared memory that one CU holds at once.

    Blocks arrive one at a time.  A block of at most simd_per_cu waves needs
    that many distinct partitions with a free wave slot and room for one
    wave's registers; its waves take the least loaded of them.  A larger block
    needs ceil(W_B / simd_per_cu) free slots (and registers) on every
    partition, and its waves are dealt round-robin over the partitions,
    continuing where the previous large block stopped."""
    if T < 1 or T > arch["max_threads_per_block"] or R < 0 or S < 0:
        return 0
    if R > arch["max_vgprs_per_thread"] or S > arch["max_lds_per_block"]:
        return 0
    waves_per_block = -(-T // arch["wave_size"])
    regs_per_wave = _round_up(R, arch["vgpr_granule"]) if R > 0 else 0
    lds_per_block = _round_up(S, arch["lds_granule"]) if S > 0 else 0
    p = arch["simd_per_cu"]
    slots = [arch["max_waves_per_cu"] // p] * p
    regs = [arch["vgprs_per_simd_lane"]] * p
    lds_free = arch["lds_per_cu"]
    counted = not (waves_per_block == 1 and arch["single_wave_exempt"])
    need = -(-waves_per_block // p)
    nxt = 0  # round-robin position for blocks larger than the partition count
    blocks = 0
    while blocks < limit:
        if counted and blocks >= arch["max_blocks_per_cu"]:
            break
        if lds_per_block > lds_free:
            break
        if waves_per_block <= p:
            fits = [i for i in range(p) if slots[i] > 0 and regs[i] >= regs_per_wave]
            if len(fits) < waves_per_block:
                break
            fits.sort(key=lambda i: (-slots[i], -regs[i], i))
            for i in fits[:waves_per_block]:
                slots[i] -= 1
                regs[i] -= regs_per_wave
        else:
            if any(slots[i] < need or regs[i] < need * regs_per_wave for i in range(p)):
                break
            for _ in range(waves_per_block):
                slots[nxt] -= 1
                regs[nxt] -= regs_per_wave
                nxt = (nxt + 1) % p
        lds_free -= lds_per_block
        blocks += 1
    return blocks


def resident_waves(arch: dict, T: int, R: int, S: int) -> int:
    return resident_blocks(arch, T, R, S) * (-(-T // arch["wave_size"]) if T >= 1 else 0)
