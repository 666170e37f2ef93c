"""Complex logm on the GPU (LOGM_C128): the library runs Algorithm 1 on the real
representation P of A; the result must match the oracle on P (same decisions,
element by element), the closed form, and the oracle's complex Algorithm 1."""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from workloads import complex_matrix, real_representation

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2401_10089_amd as lm

    lm.load_library()
    return lm


def relf(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("n", [1, 8, 50, 130])
def test_complex_logm_vs_oracle_on_real_representation(lm, n):
    import torch

    A, Lx = complex_matrix(n, 8100 + n)
    L, info = lm.logm(torch.from_numpy(A).to("cuda:0"))
    assert L.dtype == torch.complex128
    L = L.cpu().numpy()
    P = real_representation(A)
    LP, io = oracle.logm(P)
    if (info["s"], info["k"], info["db_iters"]) != (io["s"], io["k"], io["db_iters"]):
        LP, _ = oracle.logm(P, force={"s": info["s"], "k": info["k"], "db_iters": info["db_iters"]})
    Lo = LP[:n, :n] + 1j * LP[n:, :n]
    assert relf(L, Lo) < 1e-12
    assert relf(L, Lx) < 1e-11
    Lc, _ = oracle.logm(A)
    assert relf(L, Lc) < 1e-11


def test_complex_logm_strided_input(lm):
    import torch

    n = 40
    A, Lx = complex_matrix(n, 8200)
    big = torch.zeros((n, n + 7), dtype=torch.complex128, device="cuda:0")
    big[:, :n] = torch.from_numpy(A).to("cuda:0")
    L, _ = lm.logm(big[:, :n])
    assert relf(L.cpu().numpy(), Lx) < 1e-11


def test_complex_backward_vs_oracle_and_block_form(lm):
    """gradA = L_log(A^H, G) for complex A: the real reverse mode on the
    representation against the oracle's on the same 2n matrices, and against the
    block form log([[A^H, G], [0, A^H]]) of the oracle's complex Algorithm 1."""
    import torch

    n = 24
    A, _ = complex_matrix(n, 8300)
    rng = np.random.default_rng(8301)
    G = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    dev = torch.device("cuda:0")
    gA, info = lm.logm_backward(torch.from_numpy(A).to(dev), torch.from_numpy(G).to(dev))
    gA = gA.cpu().numpy()
    gP, _ = oracle.logm_backward(real_representation(A), real_representation(G),
                                 force={"s": info["s"], "k": info["k"], "db_iters": info["db_iters"]})
    assert relf(gA, gP[:n, :n] + 1j * gP[n:, :n]) < 1e-12
    ref = oracle.frechet_block(A.conj().T, G)
    assert relf(gA, ref) < 1e-11


def test_complex_autograd(lm):
    import torch

    n = 12
    A, _ = complex_matrix(n, 8400)
    dev = torch.device("cuda:0")
    At = torch.from_numpy(A).to(dev).requires_grad_(True)
    G = torch.from_numpy(np.random.default_rng(8401).standard_normal((n, n)) + 0j).to(dev)
    L = lm.logm_autograd(At)
    L.backward(G)
    gA, _ = lm.logm_backward(torch.from_numpy(A).to(dev), G)
    assert torch.equal(At.grad, gA)


def test_complex_taped_pair(lm):
    """The taped pair on complex input: the forward equals logm_forward, the backward
    equals the self-contained logm_backward bit for bit, and one tape serves several
    G (each checked against the block form of the oracle's complex Algorithm 1)."""
    import torch

    n = 20
    A, _ = complex_matrix(n, 8600)
    dev = torch.device("cuda:0")
    Ad = torch.from_numpy(A).to(dev)
    tape = lm.Tape(n, dev, complex=True)
    L, info = lm.logm_forward_taped(Ad, tape)
    L_plain, _ = lm.logm(Ad)   # orders reused across roots too: equal to rounding
    assert L.dtype == torch.complex128
    assert relf(L.cpu().numpy(), L_plain.cpu().numpy()) < 1e-12
    rng = np.random.default_rng(8601)
    for _ in range(2):
        G = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        Gd = torch.from_numpy(G).to(dev)
        gA, _ = lm.logm_backward_taped(Gd, tape)
        gS, _ = lm.logm_backward(Ad, Gd)
        assert torch.equal(gA, gS)
        ref = oracle.frechet_block(A.conj().T, G)
        assert relf(gA.cpu().numpy(), ref) < 1e-11
    with pytest.raises(ValueError):
        lm.logm_backward_taped(torch.zeros((n, n), dtype=torch.float64, device=dev), tape)
