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


def test_corrected_ranking_beats_plain_on_held_out_instances():
    print("[gpu-gain] measuring 120 instances", flush=True)
    sys.stdout.flush()
    data = rd.build(40, seed=1)
    print("[gpu-gain] training", flush=True)
    sur, rep = correction.run(data, epochs=150, seed=1)
    a = rep["all"]
    print("[gpu-gain]", {k: a[k] for k in ("regret_plain", "regret_corrected", "spearman_plain",
                                           "spearman_corrected")}, flush=True)
    assert rep["train"]["loss_last"] < 0.5 * rep["train"]["loss_first"]
    assert a["regret_corrected"] < a["regret_plain"]
    assert a["spearman_corrected"] > a["spearman_plain"]
    assert np.isfinite(a["regret_corrected"])
