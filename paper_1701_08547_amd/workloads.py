"""Seeded synthetic inputs for the static autotuning model.

This module only draws random numbers and lays them out; it holds none of the
model's arithmetic, so both the GPU path and the CPU oracle may take their
inputs from it.

The paper's own workloads (Orio-generated variants of atax, BiCG, ex14FJ and
MatVec2D on NVIDIA GPUs, Sec. IV-A, Table IV) are not available; these
generators stand in for them with the shapes of its search spaces
(Sec. III-C, Table III: thread counts, block counts, unroll factors) and with
per-variant instruction mixes whose mean intensity (fp ops per memory op) sits
at the paper's 4.0 threshold.

Every stream is ``numpy.random.default_rng(SeedSequence([170108547,
config_id, stream]))`` with stream 0 = variant features, 1 = search-space
sizes, 2 = configuration rows.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SEED_ROOT = 170108547

BLOCK_VALUES = np.arange(64, 1025, 64, dtype=np.int32)      # 16 thread counts
UNROLL_VALUES = np.arange(1, 9, dtype=np.int32)             # 8 unroll factors
REG_VALUES = np.arange(16, 513, 16, dtype=np.int32)         # 32 register counts
GRID_MULTIPLIERS = np.array([1, 2, 4, 8], dtype=np.int32)   # grid = CUs x {1,2,4,8}

VARIANT_FIELDS = ("n_fp", "n_int", "n_ld", "n_st", "n_br", "n_bar", "n_reg", "lds", "div")


def rng(config_id: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([SEED_ROOT, int(config_id), int(stream)]))


@dataclass
class Batch:
    """A CSR batch: per-variant SoA columns and per-evaluation SoA columns."""

    variants: dict      # field -> np.ndarray[n_var]  (int32; div float32)
    seg: np.ndarray     # int64[n_var + 1]
    block: np.ndarray   # int32[n_evals]
    unroll: np.ndarray  # int32[n_evals]
    regs: np.ndarray    # int32[n_evals]
    grid: np.ndarray | None  # int32[n_evals] or None
    name: str = ""

    @property
    def n_var(self) -> int:
        return int(self.seg.shape[0] - 1)

    @property
    def n_evals(self) -> int:
        return int(self.seg[-1])

    def configs(self) -> dict:
        return dict(seg=self.seg, block=self.block, unroll=self.unroll, regs=self.regs, grid=self.grid)


def variant_features(n_var: int, config_id: int) -> dict:
    """Per-variant instruction mix: fp Poisson(200), int Poisson(150), loads
    Poisson(40), stores Poisson(10), branches Poisson(12), barriers U{0..4},
    register moves 0, LDS 256 * U{0..256} bytes, divergence U[0, 0.5)."""
    g = rng(config_id, 0)
    v = {
        "n_fp": g.poisson(200, n_var),
        "n_int": g.poisson(150, n_var),
        "n_ld": g.poisson(40, n_var),
        "n_st": g.poisson(10, n_var),
        "n_br": g.poisson(12, n_var),
        "n_bar": g.integers(0, 5, n_var),
        "n_reg": np.zeros(n_var),
        "lds": 256 * g.integers(0, 257, n_var),
        "div": g.random(n_var, dtype=np.float32) * np.float32(0.5),
    }
    out = {k: np.ascontiguousarray(a, dtype=np.int32) for k, a in v.items() if k != "div"}
    out["div"] = np.ascontiguousarray(v["div"], dtype=np.float32)
    return out


def product_space(with_grid: bool, n_cu: int = 256):
    """Full product of the configuration value sets, row-major: block
    slowest, then unroll, registers, grid fastest."""
    cols = [BLOCK_VALUES, UNROLL_VALUES, REG_VALUES]
    if with_grid:
        cols.append((GRID_MULTIPLIERS * n_cu).astype(np.int32))
    mesh = np.meshgrid(*cols, indexing="ij")
    flat = [np.ascontiguousarray(m.reshape(-1), dtype=np.int32) for m in mesh]
    return flat if with_grid else flat + [None]


def product_batch(n_var: int, config_id: int, with_grid: bool, n_cu: int = 256, name: str = "") -> Batch:
    """n_var variants, each with the full product space materialised."""
    T, U, R, G = product_space(with_grid, n_cu)
    m = T.shape[0]
    seg = (np.arange(n_var + 1, dtype=np.int64) * m).astype(np.int64)
    tile = lambda a: None if a is None else np.ascontiguousarray(np.tile(a, n_var))
    return Batch(variant_features(n_var, config_id), seg, tile(T), tile(U), tile(R), tile(G), name)


def c0() -> Batch:
    """One variant x 4,096 configurations (block x unroll x registers)."""
    return product_batch(1, 0, with_grid=False, name="c0")


def c1(n_cu: int = 256, n_var: int = 1000) -> Batch:
    """1,000 variants x 16,384 configurations (block x unroll x registers x
    grid), 16,384,000 evaluations."""
    return product_batch(n_var, 1, with_grid=True, n_cu=n_cu, name="c1")


def loguniform_sizes(n_var: int, lo: int, hi: int, config_id: int) -> np.ndarray:
    g = rng(config_id, 1)
    s = np.floor(np.exp(g.uniform(np.log(lo), np.log(hi + 1), n_var)))
    return np.clip(s, lo, hi).astype(np.int64)


def random_rows(n: int, config_id: int, with_grid: bool, n_cu: int = 256, stream: int = 2):
    """n configuration rows, each column drawn i.i.d. from its value set."""
    g = rng(config_id, stream)
    T = BLOCK_VALUES[g.integers(0, BLOCK_VALUES.size, n)]
    U = UNROLL_VALUES[g.integers(0, UNROLL_VALUES.size, n)]
    R = REG_VALUES[g.integers(0, REG_VALUES.size, n)]
    G = (GRID_MULTIPLIERS[g.integers(0, GRID_MULTIPLIERS.size, n)] * n_cu).astype(np.int32) if with_grid else None
    c = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.int32)
    return c(T), c(U), c(R), c(G)


def uneven_batch(n_var: int, lo: int, hi: int, config_id: int, with_grid: bool = True, n_cu: int = 256,
                 name: str = "") -> Batch:
    """Variants with search-space sizes log-uniform in [lo, hi], rows i.i.d."""
    sizes = loguniform_sizes(n_var, lo, hi, config_id)
    seg = np.zeros(n_var + 1, dtype=np.int64)
    np.cumsum(sizes, out=seg[1:])
    T, U, R, G = random_rows(int(seg[-1]), config_id, with_grid, n_cu)
    return Batch(variant_features(n_var, config_id), seg, T, U, R, G, name)


def c2(n_cu: int = 256, n_var: int = 10000) -> Batch:
    """10,000 variants with search spaces log-uniform in [64, 262,144]."""
    return uneven_batch(n_var, 64, 262144, 2, True, n_cu, name="c2")


def custom_batch(seed: int, sizes, with_grid: bool = True, n_cu: int = 256, value_sets: dict | None = None,
                 name: str = "custom") -> Batch:
    """Test batch: explicit segment sizes, rows drawn from `value_sets`
    (dict of column -> candidate values, defaults to the standard sets)."""
    sizes = np.asarray(sizes, dtype=np.int64)
    n_var = sizes.shape[0]
    seg = np.zeros(n_var + 1, dtype=np.int64)
    np.cumsum(sizes, out=seg[1:])
    n = int(seg[-1])
    g = rng(1000 + int(seed), 2)
    vs = dict(block=BLOCK_VALUES, unroll=UNROLL_VALUES, regs=REG_VALUES,
              grid=(GRID_MULTIPLIERS * n_cu).astype(np.int32))
    if value_sets:
        vs.update({k: np.asarray(v, dtype=np.int32) for k, v in value_sets.items()})
    col = lambda name: np.ascontiguousarray(vs[name][g.integers(0, len(vs[name]), n)], dtype=np.int32)
    T, U, R = col("block"), col("unroll"), col("regs")
    G = col("grid") if with_grid else None
    return Batch(variant_features(n_var, 1000 + int(seed)), seg, T, U, R, G, name)


# ---------------------------------------------------------------- streamed batches

# SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) read at an arbitrary
# position: the same counter-based definition the device generator
# (sa_gen_configs) implements, so any row of a streamed batch can be rebuilt
# here for spot checks.
_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_at(seed: int, k) -> np.ndarray:
    """Output number k (array) of the SplitMix64 sequence seeded with `seed`."""
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (k + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _pick(u: np.ndarray, n: int) -> np.ndarray:
    return (((u >> np.uint64(32)) * np.uint64(n)) >> np.uint64(32)).astype(np.int64)


def streamed_rows(seed: int, e_idx, n_cu: int = 256, with_grid: bool = True):
    """(T, U, R, G) of global evaluations `e_idx`, as the device generates them."""
    e = np.asarray(e_idx, dtype=np.uint64) * np.uint64(4)
    T = (64 * (_pick(splitmix64_at(seed, e), 16) + 1)).astype(np.int32)
    U = (_pick(splitmix64_at(seed, e + np.uint64(1)), 8) + 1).astype(np.int32)
    R = (16 * (_pick(splitmix64_at(seed, e + np.uint64(2)), 32) + 1)).astype(np.int32)
    G = (n_cu << _pick(splitmix64_at(seed, e + np.uint64(3)), 4)).astype(np.int32) if with_grid else None
    return T, U, R, G


@dataclass
class StreamedBatch:
    """A batch whose rows are generated on the device chunk by chunk."""

    variants: dict
    seg: np.ndarray     # int64[n_var + 1]
    seed: int
    n_cu: int
    name: str = ""

    @property
    def n_var(self) -> int:
        return int(self.seg.shape[0] - 1)

    @property
    def n_evals(self) -> int:
        return int(self.seg[-1])

    def subset(self, vids) -> Batch:
        """Variants `vids` with their rows rebuilt on the host (local CSR)."""
        vids = np.asarray(vids, dtype=np.int64)
        sizes = self.seg[vids + 1] - self.seg[vids]
        seg = np.zeros(vids.size + 1, dtype=np.int64)
        np.cumsum(sizes, out=seg[1:])
        idx = np.concatenate([np.arange(self.seg[v], self.seg[v + 1], dtype=np.int64) for v in vids]) \
            if vids.size else np.zeros(0, np.int64)
        T, U, R, G = streamed_rows(self.seed, idx, self.n_cu)
        var = {k: np.ascontiguousarray(a[vids]) for k, a in self.variants.items()}
        return Batch(var, seg, T, U, R, G, self.name + "-subset")


def c4(n_cu: int = 256, n_var: int = 100000) -> StreamedBatch:
    """100,000 variants with search spaces log-uniform in [256, 1,048,576]
    (about 1.26e10 evaluations), rows generated on the device."""
    sizes = loguniform_sizes(n_var, 256, 1 << 20, 4)
    seg = np.zeros(n_var + 1, dtype=np.int64)
    np.cumsum(sizes, out=seg[1:])
    seed = int(np.random.SeedSequence([SEED_ROOT, 4, 2]).generate_state(1, np.uint64)[0])
    return StreamedBatch(variant_features(n_var, 4), seg, seed, n_cu, "c4")
