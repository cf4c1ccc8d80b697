"""Host logic of the correction pipeline: ranking metrics against the
oracle's definitions and scipy, residual targets, the held-out split."""
import numpy as np
import pytest

from oracle import mlp as omlp
from paper_1701_08547_amd import correction


def test_metrics_match_oracle_and_scipy():
    stats = pytest.importorskip("scipy.stats")
    g = np.random.default_rng(5)
    for _ in range(30):
        a = g.integers(0, 12, 128).astype(float)
        t = np.exp(g.standard_normal(128))
        assert correction.spearman(a, t) == pytest.approx(stats.spearmanr(a, t).correlation, abs=1e-12)
        assert correction.spearman(a, t) == pytest.approx(omlp.spearman(a, t), abs=1e-12)
        assert correction.regret(a, t) == omlp.top1_regret(a, t)
    assert correction.regret(np.array([2.0, 1.0, 1.0]), np.array([3.0, 2.0, 1.0])) == 1.0  # tie -> lower index


def test_residual_targets_remove_instance_medians():
    ln_t = np.array([[1.0, 2.0, 3.0], [0.0, 0.0, 6.0]])
    ln_s = np.array([[5.0, 5.0, 5.0], [1.0, 2.0, 3.0]])
    r = correction.residual_targets(ln_t, ln_s)
    assert np.allclose(r, [[-1.0, 0.0, 1.0], [1.0, 0.0, 5.0]])
    # a plain key that already ranks perfectly up to scale leaves a zero residual
    assert np.allclose(correction.residual_targets(ln_s * 1.0, ln_s), 0.0)


def test_holdout_split_is_stratified_and_disjoint():
    fam = np.repeat(np.arange(3), [50, 30, 20])
    tr, ho = correction.holdout_split(fam, 0.1, 0)
    assert np.intersect1d(tr, ho).size == 0 and tr.size + ho.size == 100
    assert [int((fam[ho] == f).sum()) for f in range(3)] == [5, 3, 2]
    tr2, ho2 = correction.holdout_split(fam, 0.1, 0)
    assert np.array_equal(ho, ho2)


def test_init_params_layout():
    p = correction.init_params(0)
    assert p["W1"].shape == (128, 32) and np.all(p["W1"][:, 24:] == 0)
    assert np.abs(p["W2"]).max() <= 1 / np.sqrt(128)


def test_search_regret_hand_case():
    t = np.array([4.0, 1.0, 2.0, 8.0])
    key = np.array([0.1, 0.3, 0.2, 0.2])           # ranks: 0, then 2 and 3 tied (lower index first), then 1
    assert correction.search_regret(key, t, 1) == (3.0, 4.0 / 15.0)
    assert correction.search_regret(key, t, 2) == (1.0, 6.0 / 15.0)
    assert correction.search_regret(key, t, 3) == (1.0, 14.0 / 15.0)
    assert correction.search_regret(key, t, 4) == (0.0, 1.0)
    # k = 1 is the plain top-1 regret
    g = np.random.default_rng(3)
    for _ in range(20):
        k2, t2 = g.random(128), g.random(128) + 0.1
        assert correction.search_regret(k2, t2, 1)[0] == correction.regret(k2, t2)


def test_random_search_regret():
    g = np.random.default_rng(0)
    t = np.array([1.0, 2.0, 3.0, 4.0])
    r, share = correction.random_search_regret(t, 4, 16, g)
    assert r == 0.0 and abs(share - 1.0) < 1e-12          # every configuration timed
    r1, s1 = correction.random_search_regret(t, 1, 20000, g)
    assert abs(r1 - (0 + 1 + 2 + 3) / 4) < 0.05          # mean regret of one random pick
    assert abs(s1 - 0.25) < 0.01


def test_anneal_search_regret():
    g = np.random.default_rng(1)
    # a bowl over the 16 x 8 grid with its minimum at (9, 5)
    iT, iU = np.meshgrid(np.arange(16), np.arange(8), indexing="ij")
    t = (1.0 + 0.05 * ((iT - 9) ** 2 + (iU - 5) ** 2)).reshape(-1)
    key_at_min = np.zeros(128)
    key_at_min[9 * 8 + 5] = -1.0
    r, share = correction.anneal_search_regret(key_at_min, t, 1, g)
    assert r == 0.0 and abs(share - t.min() / t.sum()) < 1e-15     # started at the optimum, one timing
    key_far = np.zeros(128)
    key_far[0] = -1.0
    r_few = np.mean([correction.anneal_search_regret(key_far, t, 2, g)[0] for _ in range(50)])
    r_many = np.mean([correction.anneal_search_regret(key_far, t, 40, g)[0] for _ in range(50)])
    assert r_many < r_few                                           # more timings, closer to the bowl's bottom
    _, share = correction.anneal_search_regret(key_far, t, 16, g)
    assert share <= 16 * t.max() / t.sum() + 1e-12                 # never more than k distinct timings
