"""Pins of the oracle's balancing (steps 1 and 14 of Algorithm 1).

* the result is an exact diagonal similarity by powers of two;
* balancing a balanced matrix changes nothing (idempotence);
* for A = D M D^{-1} with M symmetric (whose row and column norms agree) and D
  a wide diagonal of powers of two, the balanced matrix has row and column norms
  within a factor of about 2 of each other, and log(A) with balancing matches the
  closed form D log(M) D^{-1} from the symmetric eigendecomposition, with fewer
  square roots than without;
* a matrix with a zero off-diagonal row is left alone in that index;
* the permutation step isolates the triangular parts of a reducible matrix: upper
  triangular input is left as it is, lower triangular input is reversed into upper
  triangular form, and a hidden block-triangular matrix (a dense block between two
  triangular ones, rows and columns shuffled) comes back block triangular with the
  dense block as the active range, with log A unchanged by balancing."""

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
    B, d, _, perm = oracle.balance(A)
    assert perm == list(range(10))                            # nothing to isolate
    m, e = np.frexp(d)
    assert np.all(m == 0.5)                                   # powers of two
    assert np.array_equal(B, A / d[:, None] * d[None, :])     # bitwise


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_balance_is_idempotent(seed):
    A, _, _ = scaled_symmetric(10, seed)
    B, _, _, _ = oracle.balance(A)
    B2, d2, sweeps, perm = oracle.balance(B)
    assert np.all(d2 == 1.0) and sweeps == 1 and perm == list(range(10))
    assert np.array_equal(B2, B)


@pytest.mark.parametrize("seed", [4, 5])
def test_balanced_logm_recovers_closed_form(seed):
    A, M, D = scaled_symmetric(12, seed)
    B, _, _, _ = oracle.balance(A)
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
    B, d, _, perm = oracle.balance(A)
    assert perm[-1] == 4                                      # isolated at the bottom
    assert np.array_equal(B, A[np.ix_(perm, perm)] / d[:, None] * d[None, :])
    L, _ = oracle.logm(A, balanced=True)
    L0, _ = oracle.logm(A)
    assert np.linalg.norm(L - L0) / np.linalg.norm(L0) < 1e-13



def test_permutation_step_triangular():
    rng = np.random.default_rng(21)
    U = np.triu(rng.standard_normal((7, 7))) + 3.0 * np.eye(7)
    B, d, _, perm = oracle.balance(U)
    assert perm == list(range(7)) and np.array_equal(B, U) and np.all(d == 1.0)
    Lw = U.T.copy()
    B, d, _, perm = oracle.balance(Lw)
    assert perm == list(range(6, -1, -1))                     # reversed: upper triangular
    assert not np.tril(B, -1).any()
    assert np.array_equal(B, Lw[np.ix_(perm, perm)])


def hidden_block_triangular(seed):
    """P0 [[T1, X, Y], [0, M, Z], [0, 0, T2]] P0^T: T1 (3 x 3) and T2 (4 x 4) upper
    triangular, M (10 x 10) dense with wide power-of-two row/column scaling."""
    rng = np.random.default_rng(seed)
    n1, nm, n2 = 3, 10, 4
    n = n1 + nm + n2
    T = np.zeros((n, n))
    T[:n1, :n1] = np.triu(rng.uniform(1, 2, (n1, n1)))
    D = 2.0 ** rng.integers(-12, 13, size=nm)
    M = rng.standard_normal((nm, nm)) / nm + 1.5 * np.eye(nm)
    T[n1:n1 + nm, n1:n1 + nm] = D[:, None] * M / D[None, :]
    T[n1 + nm:, n1 + nm:] = np.triu(rng.uniform(1, 2, (n2, n2)))
    T[:n1, n1:] = rng.standard_normal((n1, n - n1))
    T[n1:n1 + nm, n1 + nm:] = rng.standard_normal((nm, n2))
    p0 = rng.permutation(n)
    A = np.empty_like(T)
    A[np.ix_(p0, p0)] = T
    return A, set(int(v) for v in p0[n1:n1 + nm]), n1, nm


@pytest.mark.parametrize("seed", [31, 32, 33])
def test_permutation_step_isolates_block_triangular(seed):
    A, dense, n1, nm = hidden_block_triangular(seed)
    n = A.shape[0]
    B, d, _, perm = oracle.balance(A)
    assert sorted(perm) == list(range(n))
    assert np.array_equal(B, A[np.ix_(perm, perm)] / d[:, None] * d[None, :])
    # the active range [n1, n1 + nm) holds exactly the dense block's indices, both
    # triangular parts are upper triangular, and nothing sits below the blocks
    assert set(perm[n1:n1 + nm]) == dense
    assert not np.tril(B[:, :n1], -1).any()
    assert not B[n1 + nm:, :n1 + nm].any() and not np.tril(B[n1 + nm:, n1 + nm:], -1).any()
    assert np.all(d[:n1] == 1.0) and np.all(d[n1 + nm:] == 1.0)
    # log A is unchanged by balancing up to the rounding of the unbalanced run, whose
    # residual exp(L) - A is the larger one on these badly scaled blocks
    import scipy.linalg as sl
    L, ib = oracle.logm(A, balanced=True)
    L0, i0 = oracle.logm(A)
    assert np.linalg.norm(L - L0) / np.linalg.norm(L0) < 1e-11
    assert np.linalg.norm(sl.expm(L) - A) / np.linalg.norm(A) < 1e-14
