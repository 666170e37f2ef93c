"""Pins for the oracle's building blocks: 1-norm, 1-norm estimator, Denman-Beavers
square root (eq. ScalDB) and the polynomial evaluation (eq. five_mult_degopt)."""

import math

import numpy as np
import pytest
import scipy.linalg as sl

import oracle


def test_norm1_is_max_column_sum():
    rng = np.random.default_rng(1)
    for n in (1, 3, 17):
        M = rng.standard_normal((n, n))
        assert oracle.norm1(M) == pytest.approx(np.linalg.norm(M, 1), rel=1e-15)
    M = np.array([[1.0, -5.0], [2.0, 1.0]])
    assert oracle.norm1(M) == 6.0          # column 2, not row 1 (which would be the inf-norm)


@pytest.mark.parametrize("q,r", [(1, 0), (3, 0), (7, 0), (7, 1), (2, 1)])
def test_normest_exact_on_nonnegative(q, r):
    """For entrywise nonnegative matrices the estimator returns the exact norm."""
    rng = np.random.default_rng(10 * q + r)
    n = 9
    B = rng.uniform(0, 1, (n, n)) * 0.3
    B[:, 4] *= 5        # make one column dominant
    B2 = B @ B
    est, nmv = oracle.normest_power(B2, B, q, r)
    M = np.linalg.matrix_power(B2, q) @ np.linalg.matrix_power(B, r)
    assert est == pytest.approx(np.linalg.norm(M, 1), rel=1e-13)
    assert nmv % (q + r) == 0


def test_normest_lower_bound_and_close():
    rng = np.random.default_rng(3)
    worst = 1.0
    for trial in range(40):
        n = int(rng.integers(2, 12))
        B = rng.standard_normal((n, n)) / n
        B2 = B @ B
        for q, r in ((1, 0), (2, 1), (4, 0)):
            est, _ = oracle.normest_power(B2, B, q, r)
            exact = np.linalg.norm(np.linalg.matrix_power(B2, q) @ np.linalg.matrix_power(B, r), 1)
            assert est <= exact * (1 + 1e-12)
            worst = min(worst, est / exact)
    assert worst > 0.3            # Hager-Higham is rarely off by more than ~3x


def test_normest_diagonal_and_scalar():
    d = np.array([0.3, -0.9, 0.1, 0.5])
    D = np.diag(d)
    est, _ = oracle.normest_power(D @ D, D, 1, 1)
    assert est == pytest.approx(0.9 ** 3)
    est1, nmv = oracle.normest_power(np.array([[0.25]]), np.array([[-0.5]]), 3, 1)
    assert est1 == pytest.approx(0.5 ** 7) and nmv == 4


def test_normest_catches_transposed_apply():
    """A nonnegative matrix whose largest row sum and largest column sum differ."""
    B = np.array([[0.0, 0.0, 0.0], [0.9, 0.1, 0.1], [0.0, 0.0, 0.0]]) + 0.01
    est, _ = oracle.normest_power(B @ B, B, 1, 1)
    exact = np.linalg.norm(B @ B @ B, 1)
    assert est == pytest.approx(exact, rel=1e-13)
    assert exact != pytest.approx(np.linalg.norm(B @ B @ B, np.inf))


def test_db_sqrt_scalar_closed_form():
    """n = 1: the scaled first step lands on sqrt(a) (mu = a^{-1/2})."""
    for a in (4.0, 0.01, 123.0):
        X, it, hist, ninv = oracle.db_sqrt(np.array([[a]]))
        assert X[0, 0] == pytest.approx(math.sqrt(a), rel=4e-16)
        assert it <= 3
        assert ninv == 2 * it - 1


def test_db_sqrt_spd_matches_eigen():
    rng = np.random.default_rng(5)
    G = rng.standard_normal((20, 20))
    A = G @ G.T / 20 + 0.1 * np.eye(20)
    X, it, hist, _ = oracle.db_sqrt(A)
    w, V = np.linalg.eigh(A)
    ref = (V * np.sqrt(w)) @ V.T
    assert np.linalg.norm(X - ref) / np.linalg.norm(ref) < 1e-13
    assert np.linalg.norm(X - X.T) / np.linalg.norm(X) < 1e-13


def test_db_sqrt_nonnormal_residual_and_principal():
    from workloads import rotscale_matrix
    A, _ = rotscale_matrix(40, 99, 1e-2, 1e2)
    X, it, hist, _ = oracle.db_sqrt(A)
    assert np.linalg.norm(X @ X - A) / np.linalg.norm(A) < 1e-12
    ev = np.linalg.eigvals(X)
    assert np.all(ev.real > 0)             # principal root: spectrum in the right half plane
    ref = sl.sqrtm(A)
    assert np.linalg.norm(X - ref) / np.linalg.norm(ref) < 1e-11


def test_db_sqrt_2x2_rotation():
    r, th = 3.0, 2.5
    A = r * np.array([[math.cos(th), math.sin(th)], [-math.sin(th), math.cos(th)]])
    X, *_ = oracle.db_sqrt(A)
    ref = math.sqrt(r) * np.array([[math.cos(th / 2), math.sin(th / 2)],
                                   [-math.sin(th / 2), math.cos(th / 2)]])
    assert np.max(np.abs(X - ref)) < 1e-15 * 10


def test_db_sqrt_forced_iterations():
    rng = np.random.default_rng(8)
    A = np.eye(6) + 0.3 * rng.standard_normal((6, 6))
    X, it, hist, _ = oracle.db_sqrt(A)
    Xf, itf, histf, _ = oracle.db_sqrt(A, force_iters=it)
    assert itf == it and np.array_equal(X, Xf)


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_eval_scheme_scalar_matches_log(k):
    """-S(-b) ~ log(1+b) within the scheme's truncation at |b| well inside Theta_k."""
    th = oracle.TABLE2[k][1]
    for b in (0.5 * th, -0.5 * th):
        x = np.array([[-b]])
        z = oracle.eval_scheme(k, x, x @ x)
        assert -z[0, 0] == pytest.approx(math.log1p(b), rel=2e-15, abs=1e-300)


def test_eval_scheme_diagonal_commutes():
    d = np.array([0.1, -0.2, 0.05])
    x = np.diag(d)
    z = oracle.eval_scheme(5, x, x @ x)
    ref = -np.log1p(-d)                    # S approximates -log(1-x), eq. Taylor_log
    assert np.allclose(np.diag(z), ref, rtol=1e-15, atol=1e-17)
    assert np.count_nonzero(z - np.diag(np.diag(z))) == 0
