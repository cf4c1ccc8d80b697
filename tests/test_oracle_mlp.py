"""Pins of the learned correction's binary64 oracle: backward pass against
central finite differences, GELU and bfloat16 rounding against their
definitions, features against the hand-worked case, Adam and the ranking
metrics against textbook values and scipy."""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp


def test_bf16_rounding_known_values():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5, 3.1415927, 0.0, 65504.0], np.float32)
    got = mlp.bf16(vals)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa -> 1.0;
    # 1 + 3 * 2^-8 is a tie between 1 + 2^-7 and 1 + 2^-6: even -> 1 + 2^-6
    want = [1.0, 1.0, 1.0 + 2 ** -6, 1.0, -2.5, 3.140625, 0.0, 65536.0]
    assert got.tolist() == want


def test_gelu_definition():
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    a = np.linspace(-6, 6, 121)
    num = (mlp.gelu(a + 1e-6) - mlp.gelu(a - 1e-6)) / 2e-6
    assert np.max(np.abs(num - mlp.gelu_grad(a))) < 1e-8
    # Phi(1) = 0.841344746...
    assert abs(mlp.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15


def test_backward_matches_finite_differences():
    g = np.random.default_rng(0)
    p = mlp.init_params(seed=3, hidden=8)
    p = {k: v.astype(np.float64) for k, v in p.items()}
    p["W1"][:, 24:] = 0.0
    x = g.standard_normal((16, 32))
    x[:, 24:] = 0.0
    r = g.standard_normal(16)
    loss, grads, _ = mlp.loss_and_grads(p, x, r, quantise=False)
    eps = 1e-6
    for name in ("W1", "b1", "W2", "b2", "w3", "b3"):
        flat = p[name].reshape(-1)
        num = np.zeros_like(flat)
        for i in range(flat.size):
            old = flat[i]
            flat[i] = old + eps
            lp, _, _ = mlp.loss_and_grads(p, x, r, quantise=False)
            flat[i] = old - eps
            lm, _, _ = mlp.loss_and_grads(p, x, r, quantise=False)
            flat[i] = old
            num[i] = (lp - lm) / (2 * eps)
        ana = np.asarray(grads[name]).reshape(-1)
        scale = max(1e-12, np.max(np.abs(num)))
        assert np.max(np.abs(num - ana)) / scale <= 1e-6, name


def test_features_of_the_hand_worked_case():
    a = oracle.arch_cdna4()
    v = dict(n_fp=200, n_int=150, n_ld=40, n_st=10, n_br=12, n_bar=2, n_reg=0, lds=0, div=0.25)
    f = oracle.features(a, v, [256], [4], [128], [512])[0]
    names = dict(zip(mlp.FEATURES, f))
    assert names["ln1p_n_fp"] == np.float32(math.log(201))
    assert names["log2T_10"] == np.float32(0.8)
    assert names["U_minus1_7"] == np.float32(3 / 7)
    assert names["WB_16"] == np.float32(0.25)
    assert names["GR_32"] == np.float32(4 / 32)  # 4 waves per SIMD x 4 SIMDs / 4 waves per block
    assert names["W_32"] == np.float32(16 / 32)
    assert names["ln_score"] == np.float32(math.log(23.203125))
    assert names["inv_F"] == np.float32(0.5)
    assert names["log2_G_ncu_3"] == np.float32(1 / 3)
    assert names["intensity_gt_4"] == 0.0 and names["ln1p_intensity"] == np.float32(math.log(5.0))


def test_adam_first_step_is_sign_of_gradient_times_lr():
    p = {"w": np.array([1.0, -2.0, 0.5], np.float32)}
    g = {"w": np.array([0.3, -4.0, 1e-3])}
    out = mlp.adam_step(p, g, {}, lr=1e-3)
    # bias-corrected first step: m_hat = g, v_hat = g^2 -> update lr * g / (|g| + eps)
    want = p["w"] - 1e-3 * g["w"] / (np.abs(g["w"]) + 1e-8)
    assert np.allclose(out["w"], want.astype(np.float32), rtol=0, atol=1e-7)


def _adam_run(p, grads, lr=1e-3):
    st = {}
    seq = []
    for g in grads:
        p = mlp.adam_step(p, {"w": g}, st, lr=lr)
        seq.append(p["w"].astype(np.float64))
    return seq, st


def test_adam_three_steps_closed_form():
    """Three steps in closed form (Adam's definition with bias correction at
    every step t).  A constant gradient g moves each weight by lr g / (|g| +
    eps) at every step (m_hat = g, v_hat = g^2 for all t); a frozen t = 1
    correction would give (1 - b1^2)/(1 - b1) / sqrt((1 - b2^2)/(1 - b2)) =
    1.344 times that at t = 2.  The alternating sequence g, -g, g gives m_hat
    = g, -(1 - b1)/(1 + b1) g, (1 - b1 + b1^2)/(1 + b1 + b1^2) g with v_hat =
    g^2 throughout; swapping b1 and b2 turns the second factor 1/19 into
    1/1999."""
    lr, b1, eps = 1e-3, 0.9, 1e-8
    w0 = np.array([1.0, -2.0, 0.5, 0.0], np.float32)
    g = np.array([0.3, -4.0, 1e-3, 2.5])
    step = lr * g / (np.abs(g) + eps)
    seq, st = _adam_run({"w": w0}, [g, g, g], lr=lr)
    for t in range(3):
        assert np.allclose(seq[t], w0 - (t + 1) * step, rtol=0, atol=2e-7), t
    assert st["t"] == 3
    assert np.allclose(st["m_w"], (1 - b1 ** 3) * g, rtol=1e-12, atol=0)
    assert np.allclose(st["v_w"], (1 - 0.999 ** 3) * g * g, rtol=1e-12, atol=0)
    factors = [1.0, -(1 - b1) / (1 + b1), (1 - b1 + b1 * b1) / (1 + b1 + b1 * b1)]
    assert abs(factors[1] + 1 / 19) < 1e-15 and abs(factors[2] - 91 / 271) < 1e-15
    seq, st = _adam_run({"w": w0}, [g, -g, g], lr=lr)
    want = w0.astype(np.float64)
    for t in range(3):
        want = want - lr * factors[t] * g / (np.abs(g) + eps)
        assert np.allclose(seq[t], want, rtol=0, atol=3e-7), t


def test_adam_planted_mistakes_fail_the_closed_form():
    """The closed form above tells Adam from its two plausible mistakes:
    beta1/beta2 swapped, and the bias correction frozen at t = 1."""
    lr, eps = 1e-3, 1e-8
    g = np.array([0.3, -4.0, 2.5])

    def wrong(seq_g, b1, b2, frozen):
        m = v = np.zeros(3)
        w = np.zeros(3)
        for t, gt in enumerate(seq_g, start=1):
            m = b1 * m + (1 - b1) * gt
            v = b2 * v + (1 - b2) * gt * gt
            tc = 1 if frozen else t
            w = w - lr * (m / (1 - b1 ** tc)) / (np.sqrt(v / (1 - b2 ** tc)) + eps)
        return w

    right = wrong([g, -g], 0.9, 0.999, False)
    assert np.allclose(right, -lr * (1 - 1 / 19) * g / (np.abs(g) + eps), rtol=0, atol=1e-12)
    assert np.abs(wrong([g, -g], 0.999, 0.9, False) - right).min() > 4e-5
    assert np.abs(wrong([g, g], 0.9, 0.999, True) - wrong([g, g], 0.9, 0.999, False)).min() > 3e-4
    seq, _ = _adam_run({"w": np.zeros(3, np.float32)}, [g, -g])
    assert np.allclose(seq[-1], right, rtol=0, atol=2e-7)


def test_ranking_metrics():
    scipy_stats = pytest.importorskip("scipy.stats")
    g = np.random.default_rng(1)
    for _ in range(20):
        a = g.integers(0, 10, 50).astype(float)
        b = a + g.standard_normal(50)
        assert abs(mlp.spearman(a, b) - scipy_stats.spearmanr(a, b).correlation) < 1e-12
    t = np.array([3.0, 1.0, 2.0])
    assert mlp.top1_regret(np.array([0.5, 0.1, 0.2]), t) == 0.0
    assert mlp.top1_regret(np.array([0.1, 0.5, 0.2]), t) == 2.0
    assert mlp.top1_regret(np.array([0.1, 0.5, 0.1]), t) == 2.0  # tie -> lower index


def test_quantised_forward_uses_bf16_weights_and_activations():
    p = mlp.init_params(seed=1)
    g = np.random.default_rng(2)
    x = mlp.bf16(g.standard_normal((4, 32)))
    fw = mlp.forward(p, x)
    assert np.array_equal(fw["h1"], mlp.bf16(fw["h1"]))
    assert np.array_equal(fw["W2"], mlp.bf16(p["W2"]))
    assert fw["delta"].shape == (4,)


def test_pairwise_loss_hand_cases():
    # one ordered pair at equal keys: softplus(0) = ln 2, gradient +-sigma(0)
    loss, g = mlp.pairwise_loss(np.array([0.0, 0.0]), np.array([1.0, 2.0]), 2)
    assert abs(loss - np.log(2.0)) < 1e-15 and g.tolist() == [0.5, -0.5]
    # equal measured times: no pair, no loss
    loss, g = mlp.pairwise_loss(np.array([0.3, -1.0]), np.array([1.0, 1.0]), 2)
    assert loss == 0.0 and g.tolist() == [0.0, 0.0]
    # keys in the measured order with a wide margin cost almost nothing; the
    # reverse order costs about the margin per pair
    y = np.arange(4.0)
    good, _ = mlp.pairwise_loss(np.array([0.0, 40.0, 80.0, 120.0]), y, 4)
    bad, _ = mlp.pairwise_loss(np.array([120.0, 80.0, 40.0, 0.0]), y, 4)
    assert good < 1e-15 and abs(bad - 400.0 / 6.0) < 1e-12   # mean of 40, 80, 120, 40, 80, 40
    # two groups: the mean over groups of each group's pair mean
    loss, _ = mlp.pairwise_loss(np.array([0.0, 0.0, 5.0, 0.0]), np.array([1.0, 2.0, 1.0, 2.0]), 2)
    assert abs(loss - 0.5 * (np.log(2.0) + np.log1p(np.exp(5.0)))) < 1e-12


def test_pairwise_loss_invariance_and_gradient():
    g = np.random.default_rng(4)
    z = g.standard_normal(24)
    y = g.integers(0, 6, 24).astype(np.float64)       # ties within groups
    loss, grad = mlp.pairwise_loss(z, y, 8)
    shifted = z.copy()
    shifted[8:16] += 3.0                              # a constant within one group changes nothing
    assert abs(mlp.pairwise_loss(shifted, y, 8)[0] - loss) < 1e-12
    eps = 1e-6
    for i in range(z.size):
        zp, zm = z.copy(), z.copy()
        zp[i] += eps
        zm[i] -= eps
        num = (mlp.pairwise_loss(zp, y, 8)[0] - mlp.pairwise_loss(zm, y, 8)[0]) / (2 * eps)
        assert abs(num - grad[i]) <= 1e-8 + 1e-6 * abs(grad[i]), i
    assert abs(grad[:8].sum()) < 1e-12                # each pair moves its two keys in opposite directions


def test_ranking_backward_matches_finite_differences():
    g = np.random.default_rng(1)
    p = mlp.init_params(seed=5, hidden=8)
    p = {k: v.astype(np.float64) for k, v in p.items()}
    p["W1"][:, 24:] = 0.0
    x = g.standard_normal((16, 32))
    x[:, 24:] = 0.0
    ln_s = g.standard_normal(16)
    y = g.standard_normal(16)
    loss, grads, _ = mlp.ranking_loss_and_grads(p, x, ln_s, y, 8, quantise=False)
    eps = 1e-6
    for name in ("W1", "b2", "w3", "b3"):
        flat = p[name].reshape(-1)
        for i in range(0, flat.size, max(1, flat.size // 24)):
            old = flat[i]
            flat[i] = old + eps
            lp = mlp.ranking_loss_and_grads(p, x, ln_s, y, 8, quantise=False)[0]
            flat[i] = old - eps
            lm = mlp.ranking_loss_and_grads(p, x, ln_s, y, 8, quantise=False)[0]
            flat[i] = old
            num = (lp - lm) / (2 * eps)
            ana = np.asarray(grads[name]).reshape(-1)[i]
            assert abs(num - ana) <= 1e-9 + 1e-6 * abs(ana), (name, i, num, ana)
