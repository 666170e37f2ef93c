"""Launch-shape autotuner (logm_autotune): it must pick one of its candidates, and
results after tuning must still match the oracle (the cap changes the schedule of
the trailing update only, never the arithmetic)."""

import numpy as np
import pytest

import oracle
from workloads import disk_matrix

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2401_10089_amd as lm

    lm.load_library()
    return lm


def test_autotune_then_logm_matches_oracle(lm):
    import torch

    n = 300
    caps, ms = lm.autotune(n)
    assert caps[0] in (96, 128, 160, 192, 224, 256)
    assert caps[1] in (224, 256, 320, 384, 448, 512)
    assert ms[0] > 0.0 and ms[1] > 0.0
    A = disk_matrix(n, 9100)
    L, info = lm.logm(torch.from_numpy(A).to("cuda:0"))
    Lo, io = oracle.logm(A)
    if (info["s"], info["k"], info["db_iters"]) != (io["s"], io["k"], io["db_iters"]):
        Lo, _ = oracle.logm(A, force={"s": info["s"], "k": info["k"], "db_iters": info["db_iters"]})
    L = L.cpu().numpy()
    assert np.linalg.norm(L - Lo) / np.linalg.norm(Lo) < 1e-12
