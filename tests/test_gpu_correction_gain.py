"""The gain test of the learned correction: on instances it was not
trained on, ranking by the corrected key z = ln(score) + Delta picks faster
configurations than ranking by the plain static score.  The dataset is
measured here (40 instances per family, the paper's timing protocol), the
network trained through the library, 10 % of each family held out."""
import sys

import numpy as np
import pytest

from paper_1701_08547_amd import correction, runtime_dataset as rd

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)


@pytest.fixture(scope="module")
def data():
    print("[gpu-gain] measuring 150 instances", flush=True)
    sys.stdout.flush()
    return rd.build(50, seed=1)


@pytest.mark.parametrize("loss", ["mse", "pairwise"])
def test_corrected_ranking_beats_plain_on_held_out_instances(data, loss):
    """A quarter of each family held out (36 instances); the mean regret
    difference plain - corrected has a bootstrap interval above zero."""
    print("[gpu-gain] training", loss, flush=True)
    sur, rep = correction.run(data, epochs=150, seed=1, loss=loss, held_frac=0.25)
    a = rep["all"]
    print("[gpu-gain]", loss, {k: a[k] for k in ("instances", "regret_plain", "regret_corrected", "regret_diff_ci",
                                                 "spearman_plain", "spearman_corrected")}, flush=True)
    assert a["instances"] >= 30
    assert rep["train"]["loss_last"] < 0.5 * rep["train"]["loss_first"]
    assert a["regret_corrected"] < a["regret_plain"]
    assert a["regret_diff_ci"][0] > 0
    assert a["spearman_corrected"] > a["spearman_plain"]
    assert np.isfinite(a["regret_corrected"])


def test_live_search_times_only_the_survivors(data):
    """Model-guided search (Sec. III-C, IV-C): timing only the 8 survivors of
    the corrected key costs a fraction of the full sweep's wall clock and
    finds a configuration within the regret the offline analysis predicts."""
    sur, rep = correction.run(data, epochs=150, seed=1, held_frac=0.25)
    keys = rep["keys"]
    keys = {"held": keys["held"][::3], "plain": keys["plain"][::3], "corrected": keys["corrected"][::3]}
    out = correction.live_search(data, keys, k=8)
    print("[gpu-gain] live search", out, flush=True)
    assert out["instances"] == len(keys["held"])
    assert out["corrected"]["time_saved"] > 0.5
    assert out["corrected"]["regret"] < out["plain"]["regret"]
