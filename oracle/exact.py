"""Exact rational evaluation of the score -- TEST INFRASTRUCTURE ONLY.

Evaluates the cost model (Eq. 6 of Sec. III-B with the divergence weight of
Sec. II-A and the latency-hiding / grid-tail factor discussed with Eq. 2) in
``fractions.Fraction`` arithmetic, given the active blocks B* from the
residency simulator.  It pins the rounding of the C oracle's binary64 and
binary32 paths on tiny inputs; it is never timed.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from . import placement


def _frac32(x) -> Fraction:
    return Fraction(float(np.float32(x)))


def score(arch: dict, v: dict, T: int, U: int, R: int, G=None):
    """Exact score as a Fraction, or None when the configuration is illegal."""
    counts = [v["n_fp"], v["n_int"], v["n_ld"], v["n_st"], v["n_br"], v.get("n_reg", 0)]
    if any(c < 0 or c >= 2 ** 24 for c in counts) or not (0 <= v["n_bar"] <= 2 ** 14):
        return None
    d = np.float32(v["div"])
    if not (0.0 <= d <= 1.0):
        return None
    if U < 1 or U > arch["max_unroll"]:
        return None
    if G is not None and (G < 1 or G > arch["max_grid"]):
        return None
    B = placement.resident_blocks(arch, T, R, v["lds"])
    if B == 0:
        return None
    W_B = -(-T // arch["wave_size"])
    c = {k: _frac32(arch[k]) for k in ("cpi_fp", "cpi_int", "cpi_mem", "cpi_ctrl", "cpi_sync", "cpi_reg")}
    O_fl = c["cpi_fp"] * v["n_fp"] + c["cpi_int"] * v["n_int"]
    O_mem = c["cpi_mem"] * (v["n_ld"] + v["n_st"])
    O_ctrl = c["cpi_ctrl"] * v["n_br"] / U + c["cpi_sync"] * v["n_bar"] * W_B
    O_reg = c["cpi_reg"] * v.get("n_reg", 0)
    E = (O_fl + O_mem + O_ctrl + O_reg) * (1 + Fraction(float(d)))
    x = B * W_B * U
    hide = max(arch["w_sat"], x)
    if G is None:
        F = Fraction(hide, x)
    else:
        cap = arch["n_cu"] * B
        rounds = -(-G // cap)
        F = Fraction(rounds * cap * hide, G * x)
    return E * F
