"""Pins of the oracle's balancing (steps 1 and 14 of Algorithm 1).

* the result is an exact diagonal similarity by powers of two;
* balancing a balanced matrix changes nothing (idempotence);
* for A = D M D^{-1} with M symmetric (whose row and column norms agree) and D
  a wide diagonal of powers of two, the balanced matrix has row and column norms
  within a factor of about 2 of each other, and log(A) with balancing matches the
  closed form D log(M) D^{-1} from the symmetric eigendecomposition, with fewer
  square roots than without;
* a matrix with a zero off-diagonal row is left alone in that index."""

import numpy as np
import pytest

import oracle
from workloads import disk_matrix


def scaled_symmetric(n, seed, spread=20):
    rng = np.random.default_rng(seed)
    R = rng.standard_normal((n, n))
    M = R @ R.T / n + 0.5 * np.eye(n)     # symmetric positive definite
    D = 2.0 ** rng.integers(-spread, spread + 1, size=n)
    return (D[:, None] * M) / D[None, :], M, D


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_balance_is_exact_power_of_two_similarity(seed):
    A, _, _ = scaled_symmetric(10, seed)
    B, d, _ = oracle.balance(A)
    m, e = np.frexp(d)
    assert np.all(m == 0.5)                                   # powers of two
    assert np.array_equal(B, A / d[:, None] * d[None, :])     # bitwise


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_balance_is_idempotent(seed):
    A, _, _ = scaled_symmetric(10, seed)
    B, _, _ = oracle.balance(A)
    B2, d2, sweeps = oracle.balance(B)
    assert np.all(d2 == 1.0) and sweeps == 1
    assert np.array_equal(B2, B)


@pytest.mark.parametrize("seed", [4, 5])
def test_balanced_logm_recovers_closed_form(seed):
    A, M, D = scaled_symmetric(12, seed)
    B, _, _ = oracle.balance(A)
    c = np.sqrt((B * B).sum(axis=0))
    r = np.sqrt((B * B).sum(axis=1))
    assert np.all(c / r < 2.5) and np.all(r / c < 2.5)
    assert np.abs(B).sum(axis=0).max() < 1e-6 * np.abs(A).sum(axis=0).max()
    w, V = np.linalg.eigh(M)
    exact = D[:, None] * ((V * np.log(w)) @ V.T) / D[None, :]
    Lb, ib = oracle.logm(A, balanced=True)
    L0, i0 = oracle.logm(A)
    assert ib["s"] < i0["s"]
    assert np.linalg.norm(Lb - exact) / np.linalg.norm(exact) < 1e-13


def test_balance_leaves_balanced_input_and_zero_rows_alone():
    A = disk_matrix(9, 3)
    A[4, :] = 0.0
    A[4, 4] = 1.5                      # row 4 has no off-diagonal mass
    B, d, _ = oracle.balance(A)
    assert d[4] == 1.0 or np.isfinite(d[4])
    assert np.array_equal(B, A / d[:, None] * d[None, :])
    L, _ = oracle.logm(A, balanced=True)
    L0, _ = oracle.logm(A)
    assert np.linalg.norm(L - L0) / np.linalg.norm(L0) < 1e-13
