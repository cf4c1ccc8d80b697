"""The Python binding checks every buffer's length before it hands raw
pointers to the C ABI: a mis-sized tensor raises ValueError before any
library call, so a kernel never reads or writes past a buffer.  The checks
use only tensor metadata, so these tests run on host tensors without a GPU."""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp
from paper_1701_08547_amd import api, workloads


@pytest.fixture(scope="module")
def batch():
    b = workloads.custom_batch(3, [5, 0, 17], with_grid=True, name="sizes")
    var = {("lds_bytes" if f == "lds" else f): torch.from_numpy(np.ascontiguousarray(b.variants[f]))
           for f in ("n_fp", "n_int", "n_ld", "n_st", "n_br", "n_bar", "n_reg", "lds", "div")}
    cfg = {"seg": torch.from_numpy(np.ascontiguousarray(b.seg, dtype=np.int64))}
    for f in ("block", "unroll", "regs", "grid"):
        cfg[f] = torch.from_numpy(np.ascontiguousarray(getattr(b, f), dtype=np.int32))
    return var, cfg


def _short(t):
    return t[:-1].contiguous()


@pytest.mark.parametrize("col", ["unroll", "regs", "grid"])
def test_configuration_column_lengths(batch, col):
    var, cfg = batch
    bad = dict(cfg, **{col: _short(cfg[col])})
    with pytest.raises(ValueError, match=col):
        api.score(oracle.arch_cdna4(), var, bad, k=8)
    with pytest.raises(ValueError, match=col):
        api.occupancy(oracle.arch_cdna4(), var, bad)
    with pytest.raises(ValueError, match=col):
        api.features(oracle.arch_cdna4(), var, bad)


@pytest.mark.parametrize("col", ["n_int", "n_bar", "lds_bytes", "div", "n_reg"])
def test_variant_column_lengths(batch, col):
    var, cfg = batch
    bad = dict(var, **{col: _short(var[col])})
    with pytest.raises(ValueError, match=col):
        api.score(oracle.arch_cdna4(), bad, cfg, k=8)
    with pytest.raises(ValueError, match=col):
        api.suggest(oracle.arch_cdna4(), bad)
    with pytest.raises(ValueError, match=col):
        api.score_product(oracle.arch_cdna4(), bad, {"block": [64, 128], "unroll": [1], "regs": [32]}, k=4)


def test_seg_against_variant_count(batch):
    var, cfg = batch
    bad = dict(cfg, seg=cfg["seg"][:-1].contiguous())
    with pytest.raises(ValueError, match="variants"):
        api.score(oracle.arch_cdna4(), var, bad, k=8)


@pytest.mark.parametrize("out", ["occ", "score", "idx", "val"])
def test_output_lengths(batch, out):
    var, cfg = batch
    n_var, n_evals = cfg["seg"].numel() - 1, cfg["block"].numel()
    sizes = {"occ": n_evals, "score": n_evals, "idx": n_var * 8, "val": n_var * 8}
    dtype = torch.int32 if out in ("occ", "idx") else torch.float32
    with pytest.raises(ValueError, match=out):
        api.score(oracle.arch_cdna4(), var, cfg, k=8, outputs={out: torch.empty(sizes[out] - 1, dtype=dtype)})
    with pytest.raises(ValueError, match="out"):
        api.occupancy(oracle.arch_cdna4(), var, cfg, out=torch.empty(n_evals + 1, dtype=torch.int32))


def test_feature_and_target_shapes():
    s = api.Surrogate(mlp.init_params(seed=0), np.zeros(24, np.float32), np.ones(24, np.float32), device="cpu")
    with pytest.raises(ValueError, match="shape"):
        s.forward(torch.zeros((4, 23)))
    with pytest.raises(ValueError, match="shape"):
        s.forward(torch.zeros(96))
    with pytest.raises(ValueError, match="out"):
        s.forward(torch.zeros((4, 24)), out=torch.zeros(3))
    with pytest.raises(ValueError, match="target"):
        s.train_step(torch.zeros((4, 24)), torch.zeros(5))
    with pytest.raises(ValueError, match="shape"):
        s.train_step(torch.zeros((4, 25)), torch.zeros(4))


def test_headroom_and_stream_lengths():
    with pytest.raises(ValueError, match="regs"):
        api.headroom(oracle.arch_cdna4(), torch.zeros(4, dtype=torch.int32), torch.zeros(3, dtype=torch.int32))
    cols = [torch.zeros(8, dtype=torch.int32) for _ in range(4)]
    outs = [torch.zeros(8, dtype=torch.int32), torch.zeros(7, dtype=torch.int32)]
    with pytest.raises(ValueError, match="stream buffer 5"):
        api.rt_stream(cols, outs)
