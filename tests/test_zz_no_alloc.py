"""sa_score_noalloc, the allocation-free variant of sa_score for callers that
cannot allocate: through the C ABI, its outputs equal sa_score's (bit for
bit: the same kernels on the same inputs) on two calls in a row, the second
with a smaller input, for the plain and the corrected pass; a problem beyond
its fixed scratch is refused before any launch."""
import ctypes

import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_1701_08547_amd import api, workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)


def _outputs(n_var, n_evals, k):
    return {"occ": torch.full((n_evals,), -7, dtype=torch.int32, device="cuda"),
            "score": torch.full((n_evals,), -7.0, dtype=torch.float32, device="cuda"),
            "idx": torch.full((n_var, k), -7, dtype=torch.int32, device="cuda"),
            "val": torch.full((n_var, k), -7.0, dtype=torch.float32, device="cuda")}


def _noalloc(arch, var, cfg, k, sur=None):
    n_var, n_evals = api._sizes(var, cfg)
    o = _outputs(n_var, n_evals, k)
    a = api._arch_struct(arch)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    st = api.lib().sa_score_noalloc(ctypes.byref(a), ctypes.byref(api._variants_struct(var)),
                                    ctypes.byref(api._configs_struct(cfg)), n_var, n_evals, p(o["score"]), p(o["occ"]),
                                    k, p(o["idx"]), p(o["val"]), None if sur is None else ctypes.byref(sur.struct()),
                                    api._stream(None))
    assert st == 0, api.lib().sa_last_error().decode()
    return o


def _same(a, b):
    for key in ("occ", "score", "idx", "val"):
        x, y = a[key].cpu().numpy(), b[key].cpu().numpy()
        assert np.array_equal(x.view(np.uint32) if x.dtype == np.float32 else x,
                              y.view(np.uint32) if y.dtype == np.float32 else y), key


@pytest.mark.parametrize("corrected", [False, True])
def test_noalloc_equals_sa_score_on_two_calls(corrected):
    arch = oracle.arch_cdna4()
    sur = None
    if corrected:
        sur = api.Surrogate(mlp.init_params(seed=3), np.zeros(24, np.float32), np.ones(24, np.float32))
    big = workloads.custom_batch(21, [70000, 5, 0, 33000, 1, 9000], with_grid=True, name="noalloc-big")
    small = workloads.custom_batch(22, [300, 4100, 2], with_grid=False, name="noalloc-small")
    for b, k in ((big, 16), (small, 5)):
        var, cfg = api.device_batch(b)
        print("noalloc", "corrected" if corrected else "plain", b.n_var, b.n_evals, k, flush=True)
        got = _noalloc(arch, var, cfg, k, sur)
        want = api.score(arch, var, cfg, k=k, mlp=sur, outputs=_outputs(b.n_var, b.n_evals, k))
        torch.cuda.synchronize()
        _same(got, want)
        if not corrected:
            ref = oracle.run(arch, b.variants, b.configs(), k=k)
            assert np.array_equal(got["idx"].cpu().numpy(), ref["idx"])


def test_noalloc_refuses_beyond_its_scratch():
    arch = oracle.arch_cdna4()
    L = api.lib()
    # 2^28 corrected evaluations at k = 64 would need 2^28 / 1024 x 2 x 64 x 8 bytes = 256 MiB of slots
    var = {f: torch.zeros(1, dtype=torch.float32 if f == "div" else torch.int32, device="cuda")
           for f in api.VARIANT_COLUMNS}
    cfg = {"seg": torch.zeros(2, dtype=torch.int64, device="cuda")}
    for f in ("block", "unroll", "regs"):
        cfg[f] = torch.zeros(4, dtype=torch.int32, device="cuda")
    cfg["grid"] = None
    sur = api.Surrogate(mlp.init_params(seed=3), np.zeros(24, np.float32), np.ones(24, np.float32))
    idx = torch.zeros(64, dtype=torch.int32, device="cuda")
    a = api._arch_struct(arch)
    st = L.sa_score_noalloc(ctypes.byref(a), ctypes.byref(api._variants_struct(var)),
                            ctypes.byref(api._configs_struct(cfg)), 1, 1 << 28, None, None, 64,
                            ctypes.c_void_p(idx.data_ptr()), None, ctypes.byref(sur.struct()), None)
    assert st == -4
    assert "allocation-free" in L.sa_last_error().decode()
