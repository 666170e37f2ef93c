"""The allocation-free entry point (logm_forward_noalloc): its fixed device scratch
must give the results of logm_forward with a caller workspace, call after call on
the same array (a smaller matrix after a larger one), and the oracle's."""

import numpy as np
import pytest

import oracle
from workloads import disk_matrix, rotscale_matrix

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def lm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2401_10089_amd as lm

    lm.load_library()
    return lm


def relf(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_noalloc_matches_forward_twice(lm):
    import torch

    cases = [rotscale_matrix(256, 9301)[0], disk_matrix(40, 9302)]   # the second one smaller
    for A in cases:
        dA = torch.from_numpy(A).cuda()
        L1, i1 = lm.logm(dA)
        L2, i2 = lm.logm_noalloc(dA)
        torch.cuda.synchronize()
        L1, L2 = L1.cpu().numpy(), L2.cpu().numpy()
        assert (i2["s"], i2["k"], i2["db_iters"]) == (i1["s"], i1["k"], i1["db_iters"])
        assert i2["flops"] == i1["flops"]
        assert relf(L2, L1) < TOL
        Lo, io = oracle.logm(A, force={"s": i2["s"], "k": i2["k"], "db_iters": i2["db_iters"]})
        assert relf(L2, Lo) < TOL


def test_noalloc_rejects_large_and_complex(lm):
    import torch

    with pytest.raises(lm.LogmError) as e:
        lm.logm_noalloc(torch.eye(lm.NOALLOC_MAX_N + 1, dtype=torch.float64, device="cuda"))
    assert e.value.status == "LOGM_EINVAL"
    with pytest.raises(TypeError):
        lm.logm_noalloc(torch.eye(4, dtype=torch.complex128, device="cuda"))
