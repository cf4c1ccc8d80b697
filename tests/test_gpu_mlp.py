"""GPU parity of the learned correction against its binary64 oracle.

Bars (derived from the arithmetic: the GPU rounds h1, h2 and x to bfloat16
exactly as the oracle does, so the only differences are binary32 rounding of
the accumulations and of GELU, and bfloat16 ties decided differently):
  * features: binary32 values within 4e-6 relative of the oracle's rounded
    binary64 features (ln E', 1/F, ln score within 2e-5: they start from the
    binary32 score, itself within 1e-5 of binary64), the indicator exact;
  * forward: |Delta_gpu - Delta_oracle| <= 2^-7 (1 + |Delta|);
  * one training step: gradients within 2e-2 relative L2 per tensor and
    cosine >= 0.999; the loss within 2^-6 relative; Adam on the returned
    gradients within binary32 rounding of the binary64 update.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_1701_08547_amd import api, workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

NAMES = ("W1", "b1", "W2", "b2", "w3", "b3")


def say(*a):
    print("[gpu-mlp]", *a, flush=True)
    sys.stdout.flush()


def oracle_features(batch, arch):
    rows = []
    for v in range(batch.n_var):
        lo, hi = int(batch.seg[v]), int(batch.seg[v + 1])
        vv = {k: a[v] for k, a in batch.variants.items()}
        G = None if batch.grid is None else batch.grid[lo:hi]
        if hi > lo:
            rows.append(oracle.features(arch, vv, batch.block[lo:hi], batch.unroll[lo:hi], batch.regs[lo:hi], G))
    return np.concatenate(rows) if rows else np.zeros((0, 24), np.float32)


def legal_mask(batch, arch):
    return np.isfinite(oracle.run(arch, batch.variants, batch.configs(), k=0)["score64"])


def feature_batch(seed, sizes, with_grid=True):
    return workloads.custom_batch(seed, sizes, with_grid=with_grid, name="feat%d" % seed)


def norm_stats(f):
    mean = f.mean(0).astype(np.float32)
    sd = f.std(0)
    inv = np.where(sd > 0, 1.0 / np.maximum(sd, 1e-12), 1.0).astype(np.float32)
    return mean, inv


def surrogate(seed, f):
    mean, inv = norm_stats(f)
    p = mlp.init_params(seed=seed)
    return p, mean, inv, api.Surrogate(p, mean, inv)


@pytest.mark.parametrize("with_grid", [True, False])
def test_features_match_oracle(with_grid):
    arch = oracle.arch_cdna4()
    b = feature_batch(1 if with_grid else 2, [1, 63, 64, 65, 1000, 0, 4097], with_grid)
    say("features", b.n_var, b.n_evals, "grid", with_grid)
    var, cfg = api.device_batch(b)
    got = api.features(arch, var, cfg).cpu().numpy()
    ref = oracle_features(b, arch)
    ok = legal_mask(b, arch)
    assert ok.sum() > 100
    g, r = got[ok].astype(np.float64), ref[ok].astype(np.float64)
    tol = np.full(24, 4e-6)
    tol[[20, 21, 22]] = 2e-5
    err = np.abs(g - r) / np.maximum(1.0, np.abs(r))
    worst = err.max(0)
    assert np.all(worst <= tol), dict(zip(mlp.FEATURES, worst))
    assert np.array_equal(g[:, 23], r[:, 23])
    # illegal rows are flagged by an infinite ln score
    assert np.all(np.isinf(got[~ok][:, 22]))


def test_features_paper_descriptor():
    arch = oracle.arch_paper("kepler")
    b = feature_batch(3, [300, 17])
    var, cfg = api.device_batch(b)
    got = api.features(arch, var, cfg).cpu().numpy()
    ref = oracle_features(b, arch)
    ok = legal_mask(b, arch)
    err = np.abs(got[ok].astype(np.float64) - ref[ok]) / np.maximum(1.0, np.abs(ref[ok]))
    assert err.max() <= 2e-5


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000, 20001])
def test_forward_matches_oracle(n):
    arch = oracle.arch_cdna4()
    b = feature_batch(10 + n % 7, [3 * n + 64])
    ok = legal_mask(b, arch)
    f = oracle_features(b, arch)[ok][:n]
    assert f.shape[0] == n
    p, mean, inv, s = surrogate(5, f)
    say("forward n", n)
    got = s.forward(torch.from_numpy(f).cuda()).cpu().numpy().astype(np.float64)
    x = mlp.normalise(f, mean, inv)
    want = mlp.forward(p, x)["delta"]
    err = np.abs(got - want) / (1.0 + np.abs(want))
    assert err.max() <= 2 ** -7, (err.max(), int(err.argmax()))
    # the inputs are not all alike: the network does discriminate rows
    assert n < 10 or np.std(want) > 1e-3


def test_forward_trained_scale_weights():
    """Weights several times larger than at initialisation (a trained net)."""
    arch = oracle.arch_cdna4()
    b = feature_batch(21, [5000])
    f = oracle_features(b, arch)[legal_mask(b, arch)]
    mean, inv = norm_stats(f)
    p = mlp.init_params(seed=9)
    for k in ("W1", "W2", "w3"):
        p[k] = (p[k] * 3.0).astype(np.float32)
    p["b1"] = np.linspace(-0.5, 0.5, 128).astype(np.float32)
    p["b2"] = np.linspace(0.3, -0.3, 128).astype(np.float32)
    p["b3"] = np.array([0.25], np.float32)
    s = api.Surrogate(p, mean, inv)
    got = s.forward(torch.from_numpy(f).cuda()).cpu().numpy().astype(np.float64)
    want = mlp.forward(p, mlp.normalise(f, mean, inv))["delta"]
    assert (np.abs(got - want) / (1.0 + np.abs(want))).max() <= 2 ** -7


def test_weights_not_16_byte_aligned():
    """Weight arrays 8- but not 16-byte aligned take the element-by-element
    staging: Delta (sa_surrogate_fwd) and the corrected pass's keys and
    selections (sa_score with the network) equal those of aligned arrays
    bit for bit."""
    arch = oracle.arch_cdna4()
    b = feature_batch(23, [3000, 700, 5000])
    f = oracle_features(b, arch)[legal_mask(b, arch)]
    p, mean, inv, s = surrogate(6, f)
    feat = torch.from_numpy(f).cuda()
    var, cfg = api.device_batch(b)
    want_d = s.forward(feat).cpu().numpy()
    want = api.score(arch, var, cfg, k=8, mlp=s)
    for name in ("W1", "W2"):
        t = getattr(s, name)
        u = torch.empty(t.numel() + 4, dtype=t.dtype, device=t.device)[4:].view(t.shape)
        u.copy_(t)
        assert u.data_ptr() % 16 == 8
        setattr(s, name, u)
    say("unaligned weights", s.W1.data_ptr() % 16, s.W2.data_ptr() % 16)
    got_d = s.forward(feat).cpu().numpy()
    got = api.score(arch, var, cfg, k=8, mlp=s)
    torch.cuda.synchronize()
    assert np.array_equal(want_d.view(np.uint32), got_d.view(np.uint32))
    for key in ("score", "idx", "val", "occ"):
        assert np.array_equal(want[key].cpu().numpy(), got[key].cpu().numpy()), key


def _grads_flat(grad):
    g = api.params_from_flat(grad)
    return {k: np.asarray(g[k], np.float64).reshape(-1) for k in NAMES}


@pytest.mark.parametrize("n", [1, 100, 256, 1000, 70000])
def test_train_step_gradients_and_adam(n):
    arch = oracle.arch_cdna4()
    b = feature_batch(30 + n % 11, [3 * n + 64])
    f = oracle_features(b, arch)[legal_mask(b, arch)][:n]
    assert f.shape[0] == n
    p, mean, inv, s = surrogate(7, f)
    rng = np.random.default_rng(n)
    target = (0.3 * np.tanh(f[:, 22] - f[:, 22].mean()) + 0.05 * rng.standard_normal(n)).astype(np.float32)
    say("train step n", n)
    lr = 1e-3
    master0 = s.master.cpu().numpy().copy()
    loss = float(s.train_step(torch.from_numpy(f).cuda(), torch.from_numpy(target).cuda(), lr=lr).item())
    torch.cuda.synchronize()
    grad = s.grad.cpu().numpy()
    x = mlp.normalise(f, mean, inv)
    ref_loss, ref_g, _ = mlp.loss_and_grads(p, x, target)
    assert abs(loss - ref_loss) <= 2 ** -6 * ref_loss, (loss, ref_loss)
    got = _grads_flat(grad)
    for k in NAMES:
        r = np.asarray(ref_g[k], np.float64).reshape(-1)
        g = got[k]
        nr = np.linalg.norm(r)
        if nr == 0:
            assert np.all(g == 0), k
            continue
        rel = np.linalg.norm(g - r) / nr
        cos = float(g @ r) / (np.linalg.norm(g) * nr)
        assert rel <= 2e-2 and cos >= 0.999, (k, rel, cos)
    # padding columns of W1 stay exactly zero
    W1 = s.master.cpu().numpy()[: 128 * 32].reshape(128, 32)
    assert np.all(W1[:, 24:] == 0)
    # Adam applied to the GPU's own gradients, in binary64
    g_used = api.params_from_flat(grad)
    new = mlp.adam_step(api.params_from_flat(master0), {k: np.asarray(g_used[k], np.float64) for k in NAMES}, {},
                        lr=lr)
    cur = api.params_from_flat(s.master.cpu().numpy())
    for k in NAMES:
        d = np.abs(np.asarray(cur[k], np.float64) - np.asarray(new[k], np.float64))
        tol = 2e-7 + 2 ** -22 * np.abs(np.asarray(new[k], np.float64))
        assert np.all(d <= tol), (k, d.max())
    # the bf16 shadow the kernels read is the master rounded to nearest even
    w2 = s.W2.float().cpu().numpy().astype(np.float64).reshape(-1)
    assert np.array_equal(w2, mlp.bf16(cur["W2"].reshape(-1)))


def test_adam_over_consecutive_steps():
    """Six consecutive training steps (t = 1..6, squared error and then the
    pairwise loss): before each step the device state (master, m, v) is read,
    and after it the update must equal Adam's binary64 definition at that t,
    fed with the gradient the step returned.  Catches beta1/beta2 mixed up and
    a bias correction that does not follow t."""
    arch = oracle.arch_cdna4()
    b = feature_batch(71, [9000])
    f = oracle_features(b, arch)[legal_mask(b, arch)][:2048]
    assert f.shape[0] == 2048
    p, mean, inv, s = surrogate(13, f)
    rng = np.random.default_rng(5)
    target = (0.4 * np.tanh(f[:, 22] - f[:, 22].mean()) + 0.05 * rng.standard_normal(f.shape[0])).astype(np.float32)
    ft, tt = torch.from_numpy(f).cuda(), torch.from_numpy(target).cuda()
    lr = 2e-3
    for t in range(1, 7):
        group = 0 if t <= 3 else 64
        master0, m0, v0 = (x.cpu().numpy().astype(np.float64) for x in (s.master, s.m, s.v))
        say("adam step", t, "group", group)
        s.train_step(ft, tt, lr=lr, group=group)
        torch.cuda.synchronize()
        grad = s.grad.cpu().numpy().astype(np.float64)
        state = {"t": t - 1}
        for k, vals in (("m_", m0), ("v_", v0)):
            for name, arr in api.params_from_flat(vals).items():
                state[k + name] = np.asarray(arr, np.float64)
        new = mlp.adam_step(api.params_from_flat(master0), {k: np.asarray(x, np.float64) for k, x in
                                                             api.params_from_flat(grad).items()}, state, lr=lr)
        assert state["t"] == t and s.step_count == t
        cur = api.params_from_flat(s.master.cpu().numpy())
        m1 = api.params_from_flat(s.m.cpu().numpy())
        v1 = api.params_from_flat(s.v.cpu().numpy())
        for k in NAMES:
            want = np.asarray(new[k], np.float64)
            d = np.abs(np.asarray(cur[k], np.float64) - want)
            assert np.all(d <= 2e-7 + 2 ** -22 * np.abs(want)), (t, k, d.max())
            # binary32 moments: a few roundings of each term, and the binary32
            # constants 0.9f and 1 - 0.999f (the latter 1.3e-5 below 0.001)
            g = np.asarray(api.params_from_flat(grad)[k], np.float64)
            mp, vp = (np.asarray(api.params_from_flat(x)[k], np.float64) for x in (m0, v0))
            m_tol = 2 ** -20 * (0.9 * np.abs(mp) + 0.1 * np.abs(g)) + 1e-30
            v_tol = 2 ** -20 * 0.999 * vp + 2e-5 * 1e-3 * g * g + 1e-30
            assert np.all(np.abs(np.asarray(m1[k], np.float64) - state["m_" + k]) <= m_tol), (t, k)
            assert np.all(np.abs(np.asarray(v1[k], np.float64) - state["v_" + k]) <= v_tol), (t, k)
        # the update moved the weights at every step (the loss has a gradient)
        assert np.abs(np.asarray(cur["W2"], np.float64) - api.params_from_flat(master0)["W2"]).max() > 0


def test_training_reduces_loss():
    arch = oracle.arch_cdna4()
    b = feature_batch(40, [6000])
    f = oracle_features(b, arch)[legal_mask(b, arch)][:4096]
    p, mean, inv, s = surrogate(11, f)
    # a smooth function of the static features to be learned
    target = (0.5 * np.sin(f[:, 9] * 6.0) + 0.3 * f[:, 17] - 0.2 * f[:, 21]).astype(np.float32)
    target -= target.mean()
    ft, tt = torch.from_numpy(f).cuda(), torch.from_numpy(target).cuda()
    losses = [float(s.train_step(ft, tt, lr=3e-3).item()) for _ in range(200)]
    say("loss", losses[0], losses[-1])
    assert losses[-1] < 0.2 * losses[0]
    # the trained forward still matches the oracle on the final weights
    got = s.forward(ft).cpu().numpy().astype(np.float64)
    want = mlp.forward(s.params(), mlp.normalise(f, mean, inv))["delta"]
    assert (np.abs(got - want) / (1.0 + np.abs(want))).max() <= 2 ** -7


def test_surrogate_errors():
    f = torch.zeros((4, 24), device="cuda")
    s = api.Surrogate(mlp.init_params(seed=0), np.zeros(24, np.float32), np.ones(24, np.float32))
    assert s.forward(f[:0]).shape[0] == 0  # n = 0 is a no-op
    with pytest.raises(api.SAError):
        s.train_step(f[:0], torch.zeros(0, device="cuda"))
    with pytest.raises(api.SAError):
        s.train_step(f, torch.zeros(4, device="cuda"), lr=0.0)
    with pytest.raises(api.SAError):
        s.train_step(f, torch.zeros(4, device="cuda"), lr=float("nan"))


@pytest.mark.parametrize("n,group", [(256, 128), (1024, 128), (96, 32), (4096, 128)])
def test_pairwise_train_step_gradients(n, group):
    """The pairwise ranking loss (groups of consecutive rows, targets the log
    runtimes): loss and every gradient against the oracle's binary64
    definition on the same bf16 network."""
    arch = oracle.arch_cdna4()
    b = feature_batch(50 + n % 13, [3 * n + 64])
    f = oracle_features(b, arch)[legal_mask(b, arch)][:n]
    assert f.shape[0] == n
    p, mean, inv, s = surrogate(9, f)
    rng = np.random.default_rng(n + group)
    # measured times loosely following the plain key, with ties
    y = np.round(f[:, 22] + 0.7 * rng.standard_normal(n), 1).astype(np.float32)
    say("pairwise step n", n, "group", group)
    loss = float(s.train_step(torch.from_numpy(f).cuda(), torch.from_numpy(y).cuda(), lr=1e-3, group=group).item())
    torch.cuda.synchronize()
    x = mlp.normalise(f, mean, inv)
    ref_loss, ref_g, _ = mlp.ranking_loss_and_grads(p, x, f[:, 22].astype(np.float64), y, group)
    assert abs(loss - ref_loss) <= 2 ** -6 * ref_loss, (loss, ref_loss)
    got = _grads_flat(s.grad.cpu().numpy())
    for k in NAMES:
        r = np.asarray(ref_g[k], np.float64).reshape(-1)
        g = got[k]
        if k == "b3":
            # every pair moves its two keys oppositely: dL/db3 = sum of dL/dz = 0
            assert abs(r[0]) < 1e-12 and abs(g[0]) <= 1e-6, (r, g)
            continue
        nr = np.linalg.norm(r)
        rel = np.linalg.norm(g - r) / nr
        cos = float(g @ r) / (np.linalg.norm(g) * nr)
        assert rel <= 2e-2 and cos >= 0.999, (k, rel, cos)


def test_pairwise_training_orders_groups():
    """Training on the ranking loss alone lowers it and raises the rank
    correlation of z with the measured order."""
    arch = oracle.arch_cdna4()
    b = feature_batch(60, [9000])
    f = oracle_features(b, arch)[legal_mask(b, arch)][:4096]
    p, mean, inv, s = surrogate(13, f)
    rng = np.random.default_rng(3)
    # "measured" order: the plain key plus a smooth function of other features
    y = (f[:, 22] + 1.5 * np.sin(3.0 * f[:, 10]) + 0.01 * rng.standard_normal(f.shape[0])).astype(np.float32)
    ft, yt = torch.from_numpy(f).cuda(), torch.from_numpy(y).cuda()
    losses = [float(s.train_step(ft, yt, lr=3e-3, group=128).item()) for _ in range(150)]
    torch.cuda.synchronize()
    assert losses[-1] < 0.8 * losses[0], (losses[0], losses[-1])
    d = torch.empty(f.shape[0], device="cuda")
    s.forward(ft, out=d)
    z = f[:, 22] + d.cpu().numpy()
    rho_plain = np.mean([mlp.spearman(f[i:i + 128, 22], y[i:i + 128]) for i in range(0, 4096, 128)])
    rho_z = np.mean([mlp.spearman(z[i:i + 128], y[i:i + 128]) for i in range(0, 4096, 128)])
    say("pairwise training: loss", losses[0], "->", losses[-1], "spearman", rho_plain, "->", rho_z)
    assert rho_z > rho_plain + 0.05


def test_training_and_inference_forward_agree():
    """The training step's forward (exact-erf GELU by A&S 7.1.26, 16x16x16
    MFMAs) and the inference forward (GELU chords from the LDS table,
    16x16x32 MFMAs) compute the same network: with the inference Delta as
    the target, the loss a training step reports is the mean squared gap
    between the two, and its gradient for b3 is twice the mean gap.  Both
    stay within the bf16 band the oracle comparisons claim."""
    arch = oracle.arch_cdna4()
    b = feature_batch(73, [9000])
    f = oracle_features(b, arch)[legal_mask(b, arch)][:4096]
    p, mean, inv, s = surrogate(17, f)
    ft = torch.from_numpy(f).cuda()
    d_inf = s.forward(ft)
    torch.cuda.synchronize()
    rms_delta = float(d_inf.pow(2).mean().sqrt().item())
    mse_gap = float(s.train_step(ft, d_inf.clone(), lr=1e-30).item())
    torch.cuda.synchronize()
    mean_gap = float(s.grad[api.FLAT_B3].item()) / 2.0
    say("train/infer gap: rms %.3g mean %.3g (rms Delta %.3g)" % (mse_gap ** 0.5, mean_gap, rms_delta))
    assert mse_gap ** 0.5 <= 2 ** -9 * (1.0 + rms_delta)
    assert abs(mean_gap) <= 2 ** -10 * (1.0 + rms_delta)


def test_graph_captured_epochs_equal_eager_steps():
    """correction.train with each epoch's steps captured in one HIP graph
    (Adam's step number from the device counter) leaves the same weights, the
    same Adam moments and the same losses as the same steps issued one by
    one with host step numbers; squared error and the pairwise loss."""
    from paper_1701_08547_amd import correction

    arch = oracle.arch_cdna4()
    b = feature_batch(77, [30000])
    f = oracle_features(b, arch)[legal_mask(b, arch)][:9216]
    assert f.shape[0] == 9216
    mean, inv = norm_stats(f)
    g = np.random.default_rng(8)
    ft = torch.from_numpy(f).cuda()
    for group in (0, 64):
        tgt = (0.3 * np.tanh(f[:, 22] - f[:, 22].mean()) + 0.05 * g.standard_normal(f.shape[0])).astype(np.float32)
        tt = torch.from_numpy(tgt).cuda()
        runs = {}
        for graph in (False, True):
            say("train epochs, group", group, "graph", graph)
            sur, losses = correction.train(ft, tt, mean, inv, epochs=3, batch=2048, lr=2e-3, seed=5, group=group,
                                           graph=graph)
            torch.cuda.synchronize()
            runs[graph] = (sur.master.cpu().numpy(), sur.m.cpu().numpy(), sur.v.cpu().numpy(), losses,
                           sur.step_count, int(sur.steps_dev.item()) if graph else None)
        e, c = runs[False], runs[True]
        assert e[4] == c[4] == 3 * 4 and c[5] == 12
        for i in range(3):
            assert np.array_equal(e[i].view(np.uint32), c[i].view(np.uint32)), (group, i)
        assert e[3] == c[3]


def test_training_step_speed():
    """A 4,096-row step inside a captured epoch (the training loop's
    configuration) takes well under 100 us; the figure is printed."""
    from paper_1701_08547_amd import correction

    n, batch = 1 << 18, 4096
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    ft = torch.randn((n, 24), generator=g, device="cuda")
    tt = torch.randn(n, generator=g, device="cuda") * 0.1
    correction.train(ft, tt, np.zeros(24, np.float32), np.ones(24, np.float32), epochs=1, batch=batch)
    torch.cuda.synchronize()
    import time

    t0 = time.perf_counter()
    correction.train(ft, tt, np.zeros(24, np.float32), np.ones(24, np.float32), epochs=3, batch=batch)
    torch.cuda.synchronize()
    per_step = (time.perf_counter() - t0) / (3 * n // batch)
    say("training: %.1f us per %d-row step (3 epochs, wall clock incl. capture and shuffles)" % (per_step * 1e6, batch))
    assert per_step < 1e-4
