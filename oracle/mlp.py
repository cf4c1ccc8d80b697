"""Binary64 oracle of the learned correction -- TEST INFRASTRUCTURE ONLY.

The paper motivates learning from static features (Sec. V on STATuner's
learned classifier; Sec. VII, "machine learning for code classification" and
models informed by prior benchmarking) but specifies no network.  The
correction here is a small perceptron that predicts, from the static model's
own features of one (variant, configuration), a residual Delta of the
log-runtime that the plain score misses; the corrected ranking key is
ln(score) + Delta.

Definitions (shared with the GPU only through these written rules):
  * features: 24 values per evaluation (``FEATURES`` below), computed in
    binary64 from the oracle's occupancy and score, rounded to binary32;
  * normalisation x = (f - mean) * inv_std in binary32, then rounded to
    bfloat16 (round to nearest even), zero-padded to 32 inputs;
  * h1 = bf16(GELU(W1 x + b1)), h2 = bf16(GELU(W2 h1 + b2)), Delta = w3 . h2 + b3
    with W1 128x32, W2 128x128, w3 128 (bfloat16 values), b1, b2 (128) and b3
    float; GELU(a) = a/2 (1 + erf(a / sqrt 2));
  * loss = mean over the batch of (Delta - r)^2, or the pairwise ranking loss
    (``pairwise_loss``): within each group of consecutive rows (one kernel
    instance), every ordered pair (i, j) with measured y_i < y_j costs
    softplus(z_i - z_j), z = ln score + Delta; mean over each group's pairs,
    averaged over the groups;
  * Adam(lr, beta1, beta2, eps) on float master weights.

The backward pass treats the bf16 rounding of h1 and h2 as the identity (the
stored activations are what the next layer used).
"""
from __future__ import annotations

import math

import numpy as np

N_FEAT = 24
K_PAD = 32
HIDDEN = 128

FEATURES = (
    "ln1p_n_fp", "ln1p_n_int", "ln1p_n_ld", "ln1p_n_st", "ln1p_n_br", "n_bar_4", "ln1p_n_reg", "lds_64k", "div",
    "log2T_10", "U_minus1_7", "R_512", "log2_G_ncu_3", "WB_16", "GW_32", "GR_32", "GS_32", "B_32", "W_32",
    "ln1p_intensity", "ln_Eprime", "inv_F", "ln_score", "intensity_gt_4",
)


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even); returns float64 values."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    rounded = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32)
    nan = np.isnan(f)
    out = np.where(nan, np.float32(np.nan), out)
    return out.astype(np.float64)


_erf = np.vectorize(math.erf, otypes=[np.float64])


def gelu(a):
    return 0.5 * a * (1.0 + _erf(a / math.sqrt(2.0)))


def gelu_grad(a):
    return 0.5 * (1.0 + _erf(a / math.sqrt(2.0))) + a * np.exp(-0.5 * a * a) / math.sqrt(2.0 * math.pi)


def features_from_terms(v: dict, T, U, R, G, n_cu, terms: dict) -> np.ndarray:
    """The 24 features (binary32) of configurations of one variant, given the
    oracle's per-configuration terms (W_B, G_W, G_R, G_S, B, W, E', F,
    score; arrays).  G may be None (no grid dimension)."""
    T = np.asarray(T, np.float64)
    U = np.asarray(U, np.float64)
    R = np.asarray(R, np.float64)
    n = T.shape[0]
    f = np.zeros((n, N_FEAT), np.float64)
    f[:, 0] = math.log1p(v["n_fp"])
    f[:, 1] = math.log1p(v["n_int"])
    f[:, 2] = math.log1p(v["n_ld"])
    f[:, 3] = math.log1p(v["n_st"])
    f[:, 4] = math.log1p(v["n_br"])
    f[:, 5] = v["n_bar"] / 4.0
    f[:, 6] = math.log1p(v.get("n_reg", 0))
    f[:, 7] = v["lds"] / 65536.0
    f[:, 8] = float(np.float32(v["div"]))
    f[:, 9] = np.log2(T) / 10.0
    f[:, 10] = (U - 1.0) / 7.0
    f[:, 11] = R / 512.0
    f[:, 12] = 0.0 if G is None else np.log2(np.asarray(G, np.float64) / n_cu) / 3.0
    f[:, 13] = terms["W_B"] / 16.0
    f[:, 14] = np.minimum(terms["G_W"], 32) / 32.0
    f[:, 15] = np.minimum(terms["G_R"], 32) / 32.0
    f[:, 16] = np.minimum(terms["G_S"], 32) / 32.0
    f[:, 17] = terms["B"] / 32.0
    f[:, 18] = terms["W"] / 32.0
    inten = v["n_fp"] / max(1.0, float(v["n_ld"] + v["n_st"]))
    f[:, 19] = math.log1p(inten)
    with np.errstate(divide="ignore", invalid="ignore"):  # illegal rows: F = 0, score = inf
        f[:, 20] = np.log(terms["Eprime"])
        f[:, 21] = 1.0 / terms["F"]
        f[:, 22] = np.log(terms["score"])
    f[:, 23] = 1.0 if inten > 4.0 else 0.0
    return f.astype(np.float32)


def normalise(f32: np.ndarray, mean: np.ndarray, inv_std: np.ndarray) -> np.ndarray:
    """Binary32 (f - mean) * inv_std, bf16-rounded, zero-padded to 32."""
    x = (f32.astype(np.float32) - mean.astype(np.float32)) * inv_std.astype(np.float32)
    out = np.zeros((f32.shape[0], K_PAD), np.float64)
    out[:, :N_FEAT] = bf16(x)
    return out


def init_params(seed: int = 0, hidden: int = HIDDEN, n_in: int = K_PAD, n_feat: int = N_FEAT) -> dict:
    """U(+-1/sqrt(fan_in)) weights (padding columns of W1 zero), zero biases;
    float master copies."""
    g = np.random.default_rng(seed)
    W1 = g.uniform(-1, 1, (hidden, n_in)) / math.sqrt(n_feat)
    W1[:, n_feat:] = 0.0
    W2 = g.uniform(-1, 1, (hidden, hidden)) / math.sqrt(hidden)
    w3 = g.uniform(-1, 1, hidden) / math.sqrt(hidden)
    return {"W1": W1.astype(np.float32), "b1": np.zeros(hidden, np.float32), "W2": W2.astype(np.float32),
            "b2": np.zeros(hidden, np.float32), "w3": w3.astype(np.float32), "b3": np.zeros(1, np.float32)}


def forward(p: dict, x: np.ndarray, quantise: bool = True) -> dict:
    """Binary64 forward pass on bf16-rounded weights (quantise=True) or on
    the exact float weights (quantise=False, for finite differences)."""
    q = bf16 if quantise else (lambda a: np.asarray(a, np.float64))
    W1, W2, w3 = q(p["W1"]), q(p["W2"]), q(p["w3"])
    b1, b2, b3 = (np.asarray(p[k], np.float64) for k in ("b1", "b2", "b3"))
    a1 = x @ W1.T + b1
    h1 = q(gelu(a1))
    a2 = h1 @ W2.T + b2
    h2 = q(gelu(a2))
    delta = h2 @ w3 + b3[0]
    return {"x": x, "a1": a1, "h1": h1, "a2": a2, "h2": h2, "delta": delta, "W1": W1, "W2": W2, "w3": w3}


def loss_and_grads(p: dict, x: np.ndarray, r: np.ndarray, quantise: bool = True):
    """MSE loss and its gradients with respect to every parameter."""
    fw = forward(p, x, quantise)
    B = x.shape[0]
    d = fw["delta"] - np.asarray(r, np.float64)
    loss = float(np.mean(d * d))
    return loss, backward(fw, x, 2.0 * d / B), fw


def softplus(x):
    x = np.asarray(x, np.float64)
    return np.maximum(x, 0.0) + np.log1p(np.exp(-np.abs(x)))


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-np.asarray(x, np.float64)))


def pairwise_loss(z: np.ndarray, y: np.ndarray, group: int):
    """Pairwise ranking loss over groups of `group` consecutive rows and its
    gradient with respect to z, in binary64, pair by pair."""
    z = np.asarray(z, np.float64)
    y = np.asarray(y, np.float64)
    n = z.size
    n_groups = n // group
    loss, g = 0.0, np.zeros(n)
    for b in range(n_groups):
        lo = b * group
        pairs = [(i, j) for i in range(lo, lo + group) for j in range(lo, lo + group) if y[i] < y[j]]
        if not pairs:
            continue
        w = 1.0 / (n_groups * len(pairs))
        for i, j in pairs:
            loss += w * softplus(z[i] - z[j])
            s = sigmoid(z[i] - z[j])
            g[i] += w * s
            g[j] -= w * s
    return float(loss), g


def ranking_loss_and_grads(p: dict, x: np.ndarray, ln_score: np.ndarray, y: np.ndarray, group: int,
                           quantise: bool = True):
    """Pairwise ranking loss of z = ln_score + Delta and its gradients with
    respect to every parameter."""
    fw = forward(p, x, quantise)
    loss, g_delta = pairwise_loss(np.asarray(ln_score, np.float64) + fw["delta"], y, group)
    return loss, backward(fw, x, g_delta), fw


def backward(fw: dict, x: np.ndarray, g_delta: np.ndarray) -> dict:
    """Gradients of every parameter from dL/dDelta per row."""
    g = {}
    g["w3"] = fw["h2"].T @ g_delta
    g["b3"] = np.array([g_delta.sum()])
    g_h2 = np.outer(g_delta, fw["w3"])
    g_a2 = g_h2 * gelu_grad(fw["a2"])
    g["W2"] = g_a2.T @ fw["h1"]
    g["b2"] = g_a2.sum(0)
    g_h1 = g_a2 @ fw["W2"]
    g_a1 = g_h1 * gelu_grad(fw["a1"])
    g["W1"] = g_a1.T @ x
    g["b1"] = g_a1.sum(0)
    return g


def adam_step(p: dict, g: dict, state: dict, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8) -> dict:
    """One Adam update of the float master weights (binary64 arithmetic)."""
    t = state.get("t", 0) + 1
    out = {}
    for k in p:
        m = state.get("m_" + k, np.zeros_like(p[k], dtype=np.float64))
        v = state.get("v_" + k, np.zeros_like(p[k], dtype=np.float64))
        m = b1 * m + (1 - b1) * g[k]
        v = b2 * v + (1 - b2) * g[k] * g[k]
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        out[k] = (p[k].astype(np.float64) - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32)
        state["m_" + k], state["v_" + k] = m, v
    state["t"] = t
    return out


# ------------------------------------------------------------------ evaluation of a ranking


def top1_regret(key: np.ndarray, t: np.ndarray) -> float:
    """t(argmin key) / min t - 1; ties of the key go to the lower index."""
    i = int(np.argmin(key))
    return float(t[i] / np.min(t) - 1.0)


def spearman(a: np.ndarray, b: np.ndarray) -> float:
    """Spearman rank correlation with average ranks for ties."""

    def ranks(x):
        order = np.argsort(x, kind="mergesort")
        r = np.empty(len(x), np.float64)
        xs = x[order]
        i = 0
        while i < len(x):
            j = i
            while j + 1 < len(x) and xs[j + 1] == xs[i]:
                j += 1
            r[order[i:j + 1]] = (i + j) / 2.0
            i = j + 1
        return r

    ra, rb = ranks(np.asarray(a, np.float64)), ranks(np.asarray(b, np.float64))
    ra -= ra.mean()
    rb -= rb.mean()
    den = math.sqrt(float((ra * ra).sum() * (rb * rb).sum()))
    return float((ra * rb).sum() / den) if den > 0 else 0.0
