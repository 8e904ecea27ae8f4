"""The breakup study's driver (jet_study.run) on a four-domain copy of the
Weber sweep: the batch advances, every sample reduces the domains, takes the
intact lengths and labels the drops, and the result holds one entry per
domain with intact lengths inside the domains."""
import sys

import numpy as np
import pytest

from paper_2505_12205_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_jet_study_small_sweep():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a GPU")
    from paper_2505_12205_amd import jet_study
    lines = []
    print("[jet_study test] n=4, steps 128..256 every 64", flush=True)
    sys.stdout.flush()
    res = jet_study.run(steps=256, start=128, every=64, n=4, log=lines.append)
    assert res["steps"] == [128, 256]
    assert len(lines) == 1 + 3          # one advance line, three samples
    assert np.allclose(res["weber"], W.sweep_weber(4))
    assert res["finite"] == [True] * 4
    lengths = W.sweep_lengths(12205, 4)
    lb = np.asarray(res["lb_over_Dj"]) * res["D_j"]
    assert np.all(np.isfinite(lb)) and np.all(lb > 0) and np.all(lb <= lengths)
    assert all(c >= 0 for c in res["drops_per_sample"])
    de = np.asarray(res["de_over_Dj"])
    for k in range(4):
        if res["drop_observations"][k]:
            assert np.isfinite(de[k]) and de[k] > 0
        else:
            assert np.isnan(de[k])
