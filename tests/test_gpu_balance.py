"""Balancing on the GPU (steps 1 and 14 of Algorithm 1): the power-of-two similarity
must be bit-identical to the oracle's (same decisions, exact scalings), and logm
with balancing must match the oracle's balanced logm and the closed form."""

from __future__ import annotations

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


def scaled_spd(n, seed, spread=20):
    rng = np.random.default_rng(seed)
    R = rng.standard_normal((n, n))
    M = R @ R.T / n + 0.5 * np.eye(n)
    D = 2.0 ** rng.integers(-spread, spread + 1, size=n)
    return (D[:, None] * M) / D[None, :], M, D


def relf(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("n", [12, 64, 300])
def test_balance_bit_identical_to_oracle(lm, n):
    import torch

    A, _, _ = scaled_spd(n, 6000 + n)
    B, d, sweeps = lm.balance(torch.from_numpy(A).to("cuda:0"))
    Bo, do, so = oracle.balance(A)
    assert sweeps == so
    assert np.array_equal(d.cpu().numpy(), do)
    assert np.array_equal(B.cpu().numpy(), Bo)


@pytest.mark.parametrize("n", [40, 150])
def test_balanced_logm_vs_oracle_and_closed_form(lm, n):
    import torch

    A, M, D = scaled_spd(n, 6100 + n)
    L, info = lm.logm(torch.from_numpy(A).to("cuda:0"), balance=True)
    L = L.cpu().numpy()
    Lo, io = oracle.logm(A, balanced=True)
    if (info["s"], info["k"], info["db_iters"]) != (io["s"], io["k"], io["db_iters"]):
        Bo, do, _ = oracle.balance(A)
        Lb, _ = oracle.logm(Bo, force={"s": info["s"], "k": info["k"], "db_iters": info["db_iters"]})
        Lo = Lb * do[:, None] / do[None, :]
    assert relf(L, Lo) < 1e-12
    w, V = np.linalg.eigh(M)
    exact = D[:, None] * ((V * np.log(w)) @ V.T) / D[None, :]
    assert relf(L, exact) < 1e-12
    L0, i0 = lm.logm(torch.from_numpy(A).to("cuda:0"))
    assert info["s"] < i0["s"]          # balancing removed square roots


def test_balance_on_balanced_input_changes_nothing(lm):
    import torch

    A = disk_matrix(70, 6200)
    At = torch.from_numpy(A).to("cuda:0")
    L1, i1 = lm.logm(At, balance=True)
    L0, i0 = lm.logm(At)
    assert relf(L1.cpu().numpy(), L0.cpu().numpy()) < 1e-13
