"""Reverse mode on the GPU (logm_backward): gradient of <G, log A> with respect to A.

Compared element by element with the oracle's reverse mode run on the GPU's
decisions (same discrete map, so only rounding differs), with the block Frechet
form log([[A^T, G], [0, A^T]]) from the oracle, and with central finite
differences of the GPU forward; the autograd wrapper must return the same
gradient."""

from __future__ import annotations

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
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_backward(lm, A, G, **kw):
    import torch

    dev = torch.device("cuda:0")
    gA, info = lm.logm_backward(torch.from_numpy(A).to(dev), torch.from_numpy(G).to(dev), **kw)
    torch.cuda.synchronize()
    return gA.cpu().numpy(), info


def forced(info):
    return {"s": info["s"], "k": info["k"], "db_iters": info["db_iters"]}


@pytest.mark.parametrize("n,make", [(8, "disk"), (64, "disk"), (64, "rotscale"), (100, "rotscale"),
                                    (300, "rotscale")])
def test_backward_vs_oracle(lm, n, make):
    A = disk_matrix(n, 4100 + n) if make == "disk" else rotscale_matrix(n, 4200 + n, 1e-2, 1e2)[0]
    G = np.random.default_rng(4300 + n).standard_normal((n, n))
    gA, info = gpu_backward(lm, A, G)
    go, _ = oracle.logm_backward(A, G, force=forced(info))
    assert relf(gA, go) < TOL, (n, info["s"], info["k"])


@pytest.mark.parametrize("k_max", [1, 2, 3])
def test_backward_each_scheme_vs_oracle(lm, k_max):
    n = 40
    A = rotscale_matrix(n, 4400 + k_max, 1e-1, 1e1)[0]
    G = np.random.default_rng(4500 + k_max).standard_normal((n, n))
    gA, info = gpu_backward(lm, A, G, k_max=k_max)
    assert info["k"] <= k_max
    go, _ = oracle.logm_backward(A, G, k_max=k_max, force=forced(info))
    assert relf(gA, go) < TOL


def test_backward_s0_path(lm):
    n = 33
    R = np.random.default_rng(7).standard_normal((n, n))
    A = np.eye(n) + 0.05 * R / np.linalg.norm(R, 1)
    G = np.random.default_rng(8).standard_normal((n, n))
    gA, info = gpu_backward(lm, A, G)
    assert info["s"] == 0
    go, _ = oracle.logm_backward(A, G, force=forced(info))
    assert relf(gA, go) < TOL


def test_backward_vs_block_frechet_and_fd(lm):
    import torch

    n = 64
    A = rotscale_matrix(n, 4001, 1e-2, 1e2)[0]
    rng = np.random.default_rng(4002)
    G = rng.standard_normal((n, n))
    gA, _ = gpu_backward(lm, A, G)
    assert relf(gA, oracle.frechet_block(A.T, G)) < 1e-11
    dev = torch.device("cuda:0")
    h = 1e-6
    for _ in range(2):
        E = rng.standard_normal((n, n))
        Lp, _ = lm.logm(torch.from_numpy(A + h * E).to(dev))
        Lm, _ = lm.logm(torch.from_numpy(A - h * E).to(dev))
        fd = float(np.sum(G * (Lp.cpu().numpy() - Lm.cpu().numpy()))) / (2 * h)
        assert abs(fd - float(np.sum(gA * E))) <= 1e-6 * abs(fd)


def test_autograd_matches_backward(lm):
    import torch

    n = 48
    A = disk_matrix(n, 4600)
    G = np.random.default_rng(4601).standard_normal((n, n))
    dev = torch.device("cuda:0")
    At = torch.from_numpy(A).to(dev).requires_grad_(True)
    L = lm.logm_autograd(At)
    L.backward(torch.from_numpy(G).to(dev))
    gA, _ = gpu_backward(lm, A, G)
    assert np.array_equal(At.grad.cpu().numpy(), gA)
    # the taped forward reuses row orders only within a root (the reverse sweep may
    # replay a root): the plain forward with or without reuse agrees to rounding
    L1, _ = lm.logm(torch.from_numpy(A).to(dev), pivot_search=True)
    assert relf(L.detach().cpu().numpy(), L1.cpu().numpy()) < 1e-12
    L2, _ = lm.logm(torch.from_numpy(A).to(dev))
    assert relf(L.detach().cpu().numpy(), L2.cpu().numpy()) < 1e-12


def test_backward_nonfinite_G(lm):
    n = 16
    A = disk_matrix(n, 4700)
    G = np.ones((n, n))
    G[2, 3] = np.inf
    with pytest.raises(lm.LogmError) as e:
        gpu_backward(lm, A, G)
    assert e.value.code == 4


def test_taped_pair_matches_self_contained_backward(lm):
    """logm_forward_taped + logm_backward_taped give the gradient of the self-contained
    logm_backward bit for bit (and L equal to logm_forward to rounding), also with a
    ring too short for the whole tape (roots replayed) and for several G after one
    forward."""
    import torch

    n = 96
    A = rotscale_matrix(n, 4800, 1e-2, 1e2)[0]
    rng = np.random.default_rng(4801)
    Gs = [rng.standard_normal((n, n)) for _ in range(2)]
    dev = torch.device("cuda:0")
    At = torch.from_numpy(A).to(dev)
    L_ref, _ = lm.logm(At)
    L_first = None
    for tape_mats in (None, 0):
        tape = lm.Tape(n, dev, tape_mats=tape_mats)
        L, info = lm.logm_forward_taped(At, tape)
        # the taped forward reuses orders within roots only: the plain forward to
        # rounding, and every taped forward bit for bit
        assert relf(L.cpu().numpy(), L_ref.cpu().numpy()) < 1e-12
        if L_first is None:
            L_first = L.clone()
        assert torch.equal(L, L_first)
        for G in Gs + Gs[:1]:          # a G repeated after another: the tape stays valid
            gA, ib = lm.logm_backward_taped(torch.from_numpy(G).to(dev), tape)
            ref, _ = lm.logm_backward(At, torch.from_numpy(G).to(dev))
            assert torch.equal(gA, ref)
            assert (ib["s"], ib["k"]) == (info["s"], info["k"])


def test_taped_backward_needs_its_forward(lm):
    import torch

    dev = torch.device("cuda:0")
    tape = lm.Tape(32, dev)
    tape.ws.zero_()
    with pytest.raises(lm.LogmError) as e:
        lm.logm_backward_taped(torch.ones((32, 32), dtype=torch.float64, device=dev), tape)
    assert e.value.code == 1
