"""Complex input: the oracle's complex Algorithm 1 against the closed form, and the
real representation P = [[Re A, -Im A], [Im A, Re A]] whose logarithm (real
Algorithm 1 at size 2n) must be the representation of log A."""

import numpy as np
import pytest

import oracle
from workloads import complex_matrix, real_representation


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("n,seed", [(6, 1), (20, 2)])
def test_complex_logm_closed_form(n, seed):
    A, Lx = complex_matrix(n, 8000 + seed)
    L, _ = oracle.logm(A)
    assert rel(L, Lx) < 1e-12


@pytest.mark.parametrize("n,seed", [(6, 3), (20, 4)])
def test_real_representation_logm_is_representation_of_logm(n, seed):
    A, Lx = complex_matrix(n, 8000 + seed)
    LP, _ = oracle.logm(real_representation(A))
    assert rel(LP, real_representation(Lx)) < 1e-12
    # the block structure is kept to rounding
    assert np.abs(LP[:n, :n] - LP[n:, n:]).max() < 1e-12 * np.abs(LP).max()
    assert np.abs(LP[:n, n:] + LP[n:, :n]).max() < 1e-12 * np.abs(LP).max()


def test_real_representation_gradient_is_complex_adjoint():
    """The real reverse mode at P = rep(A) with rep(G) is rep(L_log(A^H, G)): checked
    against the block form of the complex Frechet derivative."""
    n = 7
    A, _ = complex_matrix(n, 8500)
    rng = np.random.default_rng(8501)
    G = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    gP, _ = oracle.logm_backward(real_representation(A), real_representation(G))
    ref = oracle.frechet_block(A.conj().T, G)
    assert rel(gP[:n, :n] + 1j * gP[n:, :n], ref) < 1e-12
    assert rel(gP, real_representation(ref)) < 1e-12
