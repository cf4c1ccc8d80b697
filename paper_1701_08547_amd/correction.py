"""Training and evaluation of the learned correction on measured runtimes.

The static model ranks an instance's configurations by ln(score); the
correction adds Delta(features) so that the corrected key
z = ln(score) + Delta tracks the measured log-runtime.  Per instance the
target of a row is its log-runtime residual after removing the per-instance
medians: r = (ln t - median ln t) - (ln s - median ln s), so that the
network learns only what the static model gets wrong in the ranking.

Everything numeric runs through the library: features (sa_features),
training steps (sa_surrogate_train_step) and the corrected keys of the
evaluation (sa_surrogate_fwd).

Evaluation per held-out instance (10 % of the instances of each family):
top-1 regret t(argmin key) / min t - 1 (ties to the lower index) and the
Spearman rank correlation of key and runtime, for the plain and the
corrected key; means with bootstrap confidence intervals.  Also the paper's
own reduction of the space (T* and the intensity rule, sa_suggest): the
fraction of configurations it removes and the regret of choosing within
what it keeps.

CLI (GPU): python -m paper_1701_08547_amd.correction --data runtime.npz \\
              --epochs 40 --out correction.npz --report correction.json
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import api, runtime_dataset
from .runtime_dataset import COUNT_FIELDS, FAMILIES, N_CFG, load


def device_rows(rows: dict, device="cuda"):
    """The dataset's rows as a device batch with one segment per row."""
    import torch

    n = rows["ms"].size
    var = {}
    for f in COUNT_FIELDS:
        var[f] = torch.from_numpy(np.ascontiguousarray(rows[f], dtype=np.int32)).to(device)
    var["lds_bytes"] = torch.from_numpy(np.ascontiguousarray(rows["lds"], dtype=np.int32)).to(device)
    var["div"] = torch.from_numpy(np.ascontiguousarray(rows["div"], dtype=np.float32)).to(device)
    cfg = {"seg": torch.arange(n + 1, dtype=torch.int64, device=device)}
    for f in ("block", "unroll", "regs", "grid"):
        cfg[f] = torch.from_numpy(np.ascontiguousarray(rows[f], dtype=np.int32)).to(device)
    return var, cfg


def residual_targets(ln_t: np.ndarray, ln_s: np.ndarray) -> np.ndarray:
    """[n_inst, 128] -> per-row residual of ln t after the plain model."""
    return ((ln_t - np.median(ln_t, axis=1, keepdims=True)) - (ln_s - np.median(ln_s, axis=1, keepdims=True)))


def holdout_split(families: np.ndarray, frac: float = 0.1, seed: int = 0):
    """Instance indices (train, held_out), `frac` of each family held out."""
    g = np.random.default_rng(np.random.SeedSequence([170108547, 3, 200 + seed]))
    train, held = [], []
    for f in np.unique(families):
        idx = np.flatnonzero(families == f)
        g.shuffle(idx)
        k = max(1, int(round(frac * idx.size)))
        held += idx[:k].tolist()
        train += idx[k:].tolist()
    return np.sort(np.array(train, np.int64)), np.sort(np.array(held, np.int64))


def ranks(x: np.ndarray) -> np.ndarray:
    """Average ranks (ties share the mean of their positions)."""
    order = np.argsort(x, kind="mergesort")
    xs = x[order]
    r = np.empty(x.size, np.float64)
    i = 0
    while i < x.size:
        j = i
        while j + 1 < x.size and xs[j + 1] == xs[i]:
            j += 1
        r[order[i:j + 1]] = 0.5 * (i + j)
        i = j + 1
    return r


def spearman(a: np.ndarray, b: np.ndarray) -> float:
    ra, rb = ranks(np.asarray(a, np.float64)), ranks(np.asarray(b, np.float64))
    ra -= ra.mean()
    rb -= rb.mean()
    den = np.sqrt((ra * ra).sum() * (rb * rb).sum())
    return float((ra * rb).sum() / den) if den > 0 else 0.0


def regret(key: np.ndarray, t: np.ndarray) -> float:
    return float(t[int(np.argmin(key))] / t.min() - 1.0)


SEARCH_K = (1, 2, 4, 8, 16)


def search_regret(key: np.ndarray, t: np.ndarray, k: int):
    """Model-guided empirical search (the use Sec. III-C makes of the model:
    it narrows the space the autotuner then times): time the k configurations
    the key ranks first (ties to the lower index) and keep the fastest.
    Returns its regret and the share of a full sweep's timing spent."""
    order = np.argsort(key, kind="stable")[:k]
    return float(t[order].min() / t.min() - 1.0), float(t[order].sum() / t.sum())


def anneal_search_regret(key: np.ndarray, t: np.ndarray, k: int, g: np.random.Generator, shape=(16, 8),
                         temp0: float = 0.3, cooling: float = 0.85, max_steps: int = 400):
    """Simulated annealing over the configuration grid (block-size index x
    unroll index, neighbours one step along either axis), started at the
    key's best configuration and stopped once k distinct configurations have
    been timed (each timing read from t).  Moves are accepted by the
    Metropolis rule on log time with a geometric cooling schedule.  Returns
    the regret of the fastest configuration timed and its timing share."""
    nT, nU = shape
    timed = {}

    def time_of(c):
        if c not in timed:
            timed[c] = t[c]
        return timed[c]

    cur = int(np.argmin(key))
    f_cur = np.log(time_of(cur))
    temp = temp0
    for _ in range(max_steps):
        if len(timed) >= k:
            break
        iT, iU = divmod(cur, nU)
        moves = [(iT + d, iU) for d in (-1, 1) if 0 <= iT + d < nT] + [(iT, iU + d) for d in (-1, 1) if 0 <= iU + d < nU]
        nT2, nU2 = moves[int(g.integers(len(moves)))]
        nxt = nT2 * nU + nU2
        f_nxt = np.log(time_of(nxt))
        if f_nxt <= f_cur or g.random() < np.exp(-(f_nxt - f_cur) / temp):
            cur, f_cur = nxt, f_nxt
        temp *= cooling
    best = min(timed.values())
    return float(best / t.min() - 1.0), float(sum(timed.values()) / t.sum())


def random_search_regret(t: np.ndarray, k: int, draws: int, g: np.random.Generator):
    """The same budget spent on k configurations drawn at random (without
    replacement): mean regret and mean time share over `draws` draws."""
    n = t.size
    picks = np.argsort(g.random((draws, n)), axis=1)[:, :k]
    sel = t[picks]
    return float((sel.min(axis=1) / t.min() - 1.0).mean()), float((sel.sum(axis=1) / t.sum()).mean())


def bootstrap_ci(x: np.ndarray, reps: int = 2000, seed: int = 0):
    g = np.random.default_rng(seed)
    m = np.array([g.choice(x, x.size).mean() for _ in range(reps)])
    return float(np.quantile(m, 0.025)), float(np.quantile(m, 0.975))


def init_params(seed: int) -> dict:
    """U(+-1/sqrt(fan_in)) weights (padding columns of W1 zero), zero biases."""
    g = np.random.default_rng(np.random.SeedSequence([170108547, 3, 300 + seed]))
    W1 = (g.uniform(-1, 1, (128, 32)) / np.sqrt(24)).astype(np.float32)
    W1[:, 24:] = 0
    W2 = (g.uniform(-1, 1, (128, 128)) / np.sqrt(128)).astype(np.float32)
    w3 = (g.uniform(-1, 1, 128) / np.sqrt(128)).astype(np.float32)
    z = np.zeros(128, np.float32)
    return {"W1": W1, "b1": z.copy(), "W2": W2, "b2": z.copy(), "w3": w3, "b3": np.zeros(1, np.float32)}


def train(feat, target, mean, inv_std, epochs: int = 40, batch: int = 4096, lr: float = 1e-3, seed: int = 0,
          device="cuda", log=None, group: int = 0, graph: bool = True):
    """Adam over shuffled mini-batches (device tensors feat [n, 24] and
    target [n]); returns the Surrogate and the per-epoch mean loss.
    group = 0: MSE(Delta, r) with rows shuffled; group > 0: the pairwise
    ranking loss with target the log runtime, whole groups of `group`
    consecutive rows (one instance each) shuffled as units.  Each epoch
    gathers its shuffled rows once into fixed buffers; with `graph` the
    epoch's steps are captured once in a HIP graph (Adam's step number kept
    on the device) and replayed every epoch."""
    import torch

    sur = api.Surrogate(init_params(seed), mean, inv_std, device)
    n = int(feat.shape[0])
    gen = torch.Generator(device=device)
    gen.manual_seed(170108547 + seed)
    losses = []
    if group > 0:
        batch = max(group, batch // group * group)
    starts = list(range(0, n - batch + 1 if n >= batch else 1, batch))
    feat_p, target_p = torch.empty_like(feat), torch.empty_like(target)
    tot = torch.zeros((), dtype=torch.float32, device=device)
    sur.reserve(min(batch, n))

    def steps():
        for b0 in starts:
            tot.add_(sur.train_step(feat_p[b0:b0 + batch], target_p[b0:b0 + batch], lr=lr, group=group,
                                    device_counter=graph))

    g = None
    for ep in range(epochs):
        if group > 0:
            g_perm = torch.randperm(n // group, generator=gen, device=device)
            perm = (g_perm[:, None] * group + torch.arange(group, device=device)[None, :]).reshape(-1)
        else:
            perm = torch.randperm(n, generator=gen, device=device)
        # one gather per epoch into the fixed buffers; each batch is a slice of them
        torch.index_select(feat, 0, perm, out=feat_p)
        torch.index_select(target, 0, perm, out=target_p)
        tot.zero_()
        if not graph:
            steps()
        else:
            if g is None:
                sur.steps_dev.fill_(sur.step_count)
                side = torch.cuda.Stream(device=device)
                side.wait_stream(torch.cuda.current_stream(device))
                torch.cuda.synchronize(device)
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, stream=side):
                    steps()
                torch.cuda.current_stream(device).wait_stream(side)
            g.replay()
            sur.step_count += len(starts)
        losses.append(float(tot.item()) / max(1, len(starts)))
        if log:
            log("epoch %d loss %.5f" % (ep + 1, losses[-1]))
    return sur, losses


def corrected_keys(feat, sur):
    """z = ln score + Delta of every row: the unfused composition of the
    features and the forward pass (bit-identical to the fused corrected
    pass, which pays one workgroup pass per segment on one-row segments)."""
    return feat[:, 22] + sur.forward(feat)


def evaluate(ms: np.ndarray, ln_s: np.ndarray, z: np.ndarray, held: np.ndarray, families: np.ndarray,
             pruned: np.ndarray | None = None) -> dict:
    """Regret and Spearman of the plain and corrected keys per held-out
    instance ([n_inst, 128] arrays), overall and per family.  With `pruned`
    (bool [n_inst, 128], the configurations the paper's reduction keeps): the
    fraction of the space it removes and the regret of choosing within it
    (the best kept configuration, and the plain / corrected argmin over it)."""
    rep = {}

    def within(key, t, m):
        if not m.any():
            return np.nan
        k = np.where(m, key, np.inf)
        return float(t[int(np.argmin(k))] / t.min() - 1.0)

    def block(ids):
        rp = np.array([regret(ln_s[i], ms[i]) for i in ids])
        rc = np.array([regret(z[i], ms[i]) for i in ids])
        sp = np.array([spearman(ln_s[i], ms[i]) for i in ids])
        sc = np.array([spearman(z[i], ms[i]) for i in ids])
        out = {"instances": int(len(ids)),
               "regret_plain": float(rp.mean()), "regret_plain_ci": bootstrap_ci(rp),
               "regret_corrected": float(rc.mean()), "regret_corrected_ci": bootstrap_ci(rc),
               "regret_diff_ci": bootstrap_ci(rp - rc),
               "spearman_plain": float(sp.mean()), "spearman_corrected": float(sc.mean())}
        search = {}
        g = np.random.default_rng(np.random.SeedSequence([170108547, 3, 400]))
        for k in SEARCH_K:
            p = np.array([search_regret(ln_s[i], ms[i], k) for i in ids])
            c = np.array([search_regret(z[i], ms[i], k) for i in ids])
            rnd = np.array([random_search_regret(ms[i], k, 32, g) for i in ids])
            sa_c = np.array([anneal_search_regret(z[i], ms[i], k, g) for i in ids])
            sa_p = np.array([anneal_search_regret(ln_s[i], ms[i], k, g) for i in ids])
            search[str(k)] = {"regret_plain": float(p[:, 0].mean()), "regret_corrected": float(c[:, 0].mean()),
                              "regret_random": float(rnd[:, 0].mean()),
                              "regret_anneal_plain": float(sa_p[:, 0].mean()),
                              "regret_anneal_corrected": float(sa_c[:, 0].mean()),
                              "time_share_plain": float(p[:, 1].mean()),
                              "time_share_corrected": float(c[:, 1].mean()),
                              "time_share_random": float(rnd[:, 1].mean())}
        out["search"] = search
        if pruned is not None:
            out["pruned_fraction"] = float(1.0 - pruned[ids].mean())
            out["regret_pruned_best"] = float(np.nanmean([within(ms[i], ms[i], pruned[i]) for i in ids]))
            out["regret_pruned_plain"] = float(np.nanmean([within(ln_s[i], ms[i], pruned[i]) for i in ids]))
            out["regret_pruned_corrected"] = float(np.nanmean([within(z[i], ms[i], pruned[i]) for i in ids]))
        return out

    rep["all"] = block(held)
    for f, name in enumerate(FAMILIES):
        ids = held[families[held] == f]
        if ids.size:
            rep[name] = block(ids)
    return rep


# features computed from the static model's terms (occupancy bounds, W_B, B*,
# W*, E', F and ln score): zeroed by the ablation without the model
MODEL_FEATURES = (13, 14, 15, 16, 17, 18, 20, 21, 22)


def run(data: dict, epochs: int = 40, batch: int = 4096, lr: float = 1e-3, seed: int = 0, device="cuda", log=None,
        loss: str = "mse", held_frac: float = 0.1, split=None, key: str = "residual", drop=()):
    """Train on the training instances, evaluate on the held-out ones
    (`held_frac` of each family, or the explicit (train, held) instance
    split).  Returns the Surrogate and the report; the report's "keys" entry
    holds the held-out instances and their plain and corrected keys.

    Ablations: key="direct" trains the network on the centred log runtime
    itself and ranks by Delta alone (no ln score term in the key); `drop`
    lists feature indices the network does not see (their normalisation
    scale set to zero, so the input is zero on every row)."""
    import torch

    n_inst = int(data["instance"].max()) + 1
    arch = api.arch_default(torch.device(device).index or 0)
    var, cfg = device_rows(data, device)
    feat = api.features(arch, var, cfg)
    ln_s = feat[:, 22].cpu().numpy().astype(np.float64).reshape(n_inst, N_CFG)
    ms = data["ms"].astype(np.float64).reshape(n_inst, N_CFG)
    legal = np.isfinite(ln_s)
    if not legal.all():
        raise ValueError("%d configurations are illegal under the model" % int((~legal).sum()))
    if key == "residual":
        r = residual_targets(np.log(ms), ln_s)
    elif key == "direct":
        if loss != "mse":
            raise ValueError("the direct key is trained on the squared error only")
        r = np.log(ms) - np.median(np.log(ms), axis=1, keepdims=True)
    else:
        raise ValueError("key must be 'residual' or 'direct'")
    families = data["family"].reshape(n_inst, N_CFG)[:, 0]
    tr, held = holdout_split(families, held_frac, seed) if split is None else (np.asarray(split[0]),
                                                                                 np.asarray(split[1]))
    rows_tr = (tr[:, None] * N_CFG + np.arange(N_CFG)[None, :]).reshape(-1)
    f_np = feat.cpu().numpy()
    mean = f_np[rows_tr].mean(0).astype(np.float32)
    sd = f_np[rows_tr].std(0)
    inv = np.where(sd > 1e-12, 1.0 / np.maximum(sd, 1e-12), 1.0).astype(np.float32)
    for j in drop:
        mean[j], inv[j] = 0.0, 0.0
    idx = torch.from_numpy(rows_tr).to(device)
    f_tr = feat.index_select(0, idx).contiguous()
    if loss == "pairwise":
        # whole instances (128 consecutive rows each), targets the log runtimes
        r_tr = torch.from_numpy(np.log(ms).reshape(-1)[rows_tr].astype(np.float32)).to(device)
        group = N_CFG
    elif loss == "mse":
        r_tr = torch.from_numpy(r.reshape(-1)[rows_tr].astype(np.float32)).to(device)
        group = 0
    else:
        raise ValueError("loss must be 'mse' or 'pairwise'")
    t0 = time.time()
    sur, losses = train(f_tr, r_tr, mean, inv, epochs, batch, lr, seed, device, log, group=group)
    torch.cuda.synchronize()
    train_s = time.time() - t0
    zt = corrected_keys(feat, sur) if key == "residual" else sur.forward(feat)
    z = zt.cpu().numpy().astype(np.float64).reshape(n_inst, N_CFG)
    kept = api.suggest(arch, var).cpu().numpy().view(np.uint64)
    ws = int(arch["wave_size"])
    T = data["block"].astype(np.int64)
    j = np.clip(T // ws - 1, 0, 63).astype(np.uint64)
    pruned = ((T % ws == 0) & (((kept >> j) & np.uint64(1)) == 1)).reshape(n_inst, N_CFG)
    rep = evaluate(ms, ln_s, z, held, families, pruned)
    rep["keys"] = {"held": held, "plain": ln_s[held], "corrected": z[held]}
    rep["train"] = {"loss": loss, "key": key, "dropped_features": [int(j) for j in drop], "rows": int(rows_tr.size), "epochs": epochs, "batch": batch, "lr": lr, "seconds": train_s,
                    "loss_first": losses[0], "loss_last": losses[-1],
                    "target_var": float(np.var(r.reshape(-1)[rows_tr]))}
    return sur, rep


def leave_one_family_out(data: dict, **kw) -> dict:
    """Regret and Spearman on each family when the correction is trained on
    the other two only (no instance of the family seen in training)."""
    n_inst = int(data["instance"].max()) + 1
    families = data["family"].reshape(n_inst, N_CFG)[:, 0]
    out = {}
    for f, name in enumerate(FAMILIES):
        held = np.flatnonzero(families == f)
        tr = np.flatnonzero(families != f)
        if held.size == 0 or tr.size == 0:
            continue
        _, rep = run(data, split=(tr, held), **kw)
        a = rep["all"]
        out[name] = {k: a[k] for k in ("instances", "regret_plain", "regret_corrected", "regret_corrected_ci",
                                       "spearman_plain", "spearman_corrected")}
    return out


def live_search(data: dict, keys: dict, k: int = 8, device="cuda", seed: int = 0) -> dict:
    """Model-guided empirical search as the paper intends it (Sec. III-C,
    Sec. IV-C): for each held-out instance, time the full sweep of its 128
    configurations, then time only the k configurations each key ranks
    first, and keep the fastest of those.  Regret is measured against the
    full sweep's fastest (the survivor's time taken from the same sweep);
    the time saved is the measured wall clock of the survivors' timing
    against the sweep's, beside the pruning estimate 1 - k / 128 (t r of
    Sec. IV-C, every configuration costing the same)."""
    import torch

    n_inst = int(data["instance"].max()) + 1
    fam = data["family"].reshape(n_inst, N_CFG)[:, 0]
    size = data["n"].reshape(n_inst, N_CFG)[:, 0]
    held = np.asarray(keys["held"])
    inst = [(FAMILIES[int(fam[i])], int(size[i])) for i in held]
    timer = runtime_dataset.Timer(inst, torch.cuda.get_device_properties(device).multi_processor_count, device,
                                  seed=seed)
    T, U = runtime_dataset.config_grid()
    wall_full = 0.0
    wall = {"plain": 0.0, "corrected": 0.0}
    reg = {"plain": [], "corrected": []}
    for j, (f, n) in enumerate(inst):
        ms_full, w_full = timer.time(f, n, T, U)
        wall_full += w_full
        for name in ("plain", "corrected"):
            order = np.argsort(np.asarray(keys[name][j]), kind="stable")[:k]
            ms_k, w_k = timer.time(f, n, T[order], U[order])
            wall[name] += w_k
            best = int(order[int(np.argmin(ms_k))])
            reg[name].append(float(ms_full[best] / ms_full.min() - 1.0))
    out = {"instances": len(inst), "k": k, "sweep_seconds": wall_full, "pruned_fraction": 1.0 - k / N_CFG}
    for name in ("plain", "corrected"):
        r = np.array(reg[name])
        out[name] = {"regret": float(r.mean()), "regret_ci": bootstrap_ci(r), "search_seconds": wall[name],
                     "time_saved": 1.0 - wall[name] / wall_full}
    return out


def time_synthetic(n: int, epochs: int, batch: int, lr: float, seed: int) -> int:
    """Training throughput alone: n random rows (standard normal features,
    targets of standard deviation 0.3), one untimed epoch, then `epochs`
    timed ones."""
    import time

    import torch

    g = torch.Generator(device="cuda").manual_seed(170108547 + seed)
    feat = torch.randn(n, api.N_FEAT, generator=g, device="cuda")
    target = torch.randn(n, generator=g, device="cuda") * 0.3
    mean, inv = np.zeros(api.N_FEAT, np.float32), np.ones(api.N_FEAT, np.float32)
    train(feat, target, mean, inv, epochs=1, batch=batch, lr=lr, seed=seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, losses = train(feat, target, mean, inv, epochs=epochs, batch=batch, lr=lr, seed=seed)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(json.dumps({"rows": n, "epochs": epochs, "batch": batch, "seconds": dt, "ms_per_epoch": dt * 1e3 / epochs,
                      "loss_last": losses[-1]}), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser()
    src = ap.add_mutually_exclusive_group(required=True)
    src.add_argument("--data", help="npz of dataset rows")
    src.add_argument("--parts", nargs="+", help="timing parts of one sampling, assembled here")
    src.add_argument("--synthetic-rows", type=int, help="time training alone on this many random rows (no report)")
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--loss", choices=("mse", "pairwise"), default="mse")
    ap.add_argument("--out", default=None, help="npz of the trained network state")
    ap.add_argument("--report", default=None)
    a = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)
    if a.synthetic_rows:
        return time_synthetic(a.synthetic_rows, a.epochs, a.batch, a.lr, a.seed)
    data = load(a.data) if a.data else runtime_dataset.assemble(a.parts)
    sur, rep = run(data, a.epochs, a.batch, a.lr, a.seed, log=log, loss=a.loss)
    rep.pop("keys")
    if a.out:
        np.savez(a.out, **{k: np.asarray(v) for k, v in sur.state_dict().items()})
    txt = json.dumps(rep, indent=1)
    if a.report:
        with open(a.report, "w") as f:
            f.write(txt + "\n")
    print(txt, flush=True)


if __name__ == "__main__":
    sys.exit(main())
