"""End-to-end pins for the oracle's logm (Algorithm 1): closed forms, invariants,
brute force at 50 digits, hand-derived decisions and error paths."""

import math

import mpmath
import numpy as np
import pytest
import scipy.linalg as sl

import oracle
from conftest import decision_cases
from workloads import disk_matrix, rotscale_matrix


def relf(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def test_identity_gives_zero():
    L, info = oracle.logm(np.eye(5))
    assert np.count_nonzero(L) == 0
    assert info["s"] == 0


@pytest.mark.parametrize("c", [2.5, 0.3, 1e-3, 1e3])
def test_scalar_multiple_of_identity(c):
    L, info = oracle.logm(c * np.eye(4))
    assert relf(L, math.log(c) * np.eye(4)) < 1e-15 * 4


def test_diagonal_wide_spectrum():
    d = np.array([1e-3, 0.5, 1.0, 2.0, 7.0, 1e3])
    L, info = oracle.logm(np.diag(d))
    assert np.allclose(np.diag(L), np.log(d), rtol=0, atol=1e-14 * np.abs(np.log(d)).max())
    assert np.count_nonzero(L - np.diag(np.diag(L))) == 0
    assert info["s"] >= 4     # 1e3^(1/2^s) - 1 <= Theta_8 = 0.5739 needs s >= 4


@pytest.mark.parametrize("r,th", [(1.0, 0.3), (5.0, 2.0), (0.01, -2.8), (300.0, 0.9 * math.pi)])
def test_rotation_scaling_block(r, th):
    a, b = r * math.cos(th), r * math.sin(th)
    L, _ = oracle.logm(np.array([[a, b], [-b, a]]))
    ref = np.array([[math.log(r), th], [-th, math.log(r)]])
    assert relf(L, ref) < 5e-15


@pytest.mark.parametrize("a,b,c", [(2.0, 1.0, 0.5), (0.1, 3.0, 40.0), (1.3, -2.0, 1.2)])
def test_upper_triangular_2x2(a, b, c):
    L, _ = oracle.logm(np.array([[a, b], [0.0, c]]))
    off = b * (math.log(a) - math.log(c)) / (a - c)
    ref = np.array([[math.log(a), off], [0.0, math.log(c)]])
    assert relf(L, ref) < 5e-15
    assert L[1, 0] == 0.0


@pytest.mark.parametrize("lam", [1.15, 0.2, 9.0])
def test_jordan_block(lam):
    L, _ = oracle.logm(np.array([[lam, 1.0], [0.0, lam]]))
    ref = np.array([[math.log(lam), 1.0 / lam], [0.0, math.log(lam)]])
    assert relf(L, ref) < 5e-15


def test_complex_diagonal():
    d = np.array([1 + 1j, -2 + 0.1j, 0.5j, 3.0 - 4.0j])
    L, _ = oracle.logm(np.diag(d))
    assert np.allclose(np.diag(L), np.log(d), rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("n,seed,lo,hi", [(16, 11, 1e-3, 1e3), (64, 12, 1e-2, 1e2), (65, 13, 1e-3, 1e3)])
def test_rotscale_exact_log(n, seed, lo, hi):
    A, Lx = rotscale_matrix(n, seed, lo, hi)
    L, info = oracle.logm(A)
    assert relf(L, Lx) < 1e-12
    assert info["k"] >= 5


def test_disk_matrix_vs_scipy_and_expm():
    A = disk_matrix(64, 1001)
    L, info = oracle.logm(A)
    assert relf(L, sl.logm(A)) < 1e-13
    assert relf(sl.expm(L), A) < 1e-14
    assert info["s"] <= 3


@pytest.mark.parametrize("n,seed", [(3, 1), (5, 2), (8, 3)])
def test_brute_force_mpmath(n, seed):
    """log A at 50 digits (mpmath) on small nonnormal matrices."""
    rng = np.random.default_rng(seed)
    A = np.eye(n) * 2 + rng.standard_normal((n, n))
    # keep the spectrum away from the negative real axis
    while np.any((np.abs(np.linalg.eigvals(A).imag) < 0.05) & (np.linalg.eigvals(A).real < 0.05)):
        A += np.eye(n)
    L, _ = oracle.logm(A)
    mpmath.mp.dps = 50
    Lmp = mpmath.logm(mpmath.matrix(A.tolist()))
    ref = np.array([[float(mpmath.re(Lmp[i, j])) for j in range(n)] for i in range(n)])
    assert relf(L, ref) < 5e-14


def test_invariants():
    A, _ = rotscale_matrix(24, 21, 1e-2, 1e2)
    L, _ = oracle.logm(A)
    Li, _ = oracle.logm(np.linalg.inv(A))
    assert relf(Li, -L) < 1e-12                                  # log(A^-1) = -log A
    Lt, _ = oracle.logm(A.T.copy())
    assert relf(Lt, L.T) < 1e-13                                 # log(A^T) = log(A)^T
    assert np.linalg.norm(A @ L - L @ A) / (np.linalg.norm(A) * np.linalg.norm(L)) < 1e-13
    Q, _ = np.linalg.qr(np.random.default_rng(4).standard_normal((24, 24)))
    Lq, _ = oracle.logm(Q.T @ A @ Q)
    assert relf(Lq, Q.T @ L @ Q) < 1e-12                         # similarity covariance
    assert relf(sl.expm(L), A) < 1e-12


def test_spd_gives_symmetric():
    rng = np.random.default_rng(6)
    X = rng.standard_normal((64, 30))
    A = X.T @ X / 64 + 1e-3 * np.eye(30)
    L, _ = oracle.logm(A)
    w, V = np.linalg.eigh(A)
    assert relf(L, (V * np.log(w)) @ V.T) < 1e-12
    assert np.linalg.norm(L - L.T) / np.linalg.norm(L) < 1e-13


def test_log_of_square_halves():
    A = disk_matrix(20, 77, 0.5)             # spectrum in Re > 0.5: log(A^2) = 2 log A
    L, _ = oracle.logm(A)
    L2, _ = oracle.logm(A @ A)
    assert relf(L2, 2 * L) < 1e-13


def _parse_matrix(txt, n):
    vals = [float(v) for v in txt.split(",")]
    return np.array(vals).reshape(n, n)


def test_hand_derived_decisions(golden):
    """(s, k, number of estimates) from the paper's inequalities, derived by hand.
    Together the cases reach every statement of the finish test and of the degree
    selection except first_pass's fallback, which Algorithm 1 cannot reach (the
    finish test leaves every value it is given at or below Theta of the top scheme)."""
    cases = decision_cases(golden)
    assert len(cases) >= 15
    for name, (A, expected, kw) in cases.items():
        if isinstance(expected, str):
            with pytest.raises(oracle.OracleError) as e:
                oracle.logm(A, **kw)
            assert e.value.code == expected, name
            continue
        L, info = oracle.logm(A, **kw)
        assert (info["s"], info["k"], info["n_est"]) == expected, name
        if A.shape[0] == 1:
            assert L[0, 0] == pytest.approx(math.log(A[0, 0]), rel=4e-15)


def test_hand_derived_decisions_are_accurate(golden):
    """Each decision is also a valid one: the logarithm it yields matches the
    50-digit logm of the same matrix."""
    for name, (A, expected, kw) in decision_cases(golden).items():
        if isinstance(expected, str):
            continue
        L, _ = oracle.logm(A, **kw)
        with mpmath.workdps(50):
            Le = np.array(mpmath.logm(mpmath.matrix(A.tolist())).tolist(), dtype=float)
        assert np.linalg.norm(L - Le) <= 1e-14 * max(np.linalg.norm(Le), 1.0), name


def test_select_degree_fallback_above_top_theta():
    """first_pass's fallback: a value above every Theta maps to the top scheme (only a
    direct call reaches it)."""
    est = lambda q, r: pytest.fail("no estimate expected")  # noqa: E731
    # e_top above Theta_5: min_in falls back to 5, max_in is 5, so k = 5 at once
    assert oracle.select_degree(10.0, 1.0, 0.5 ** 14, None, est, (1, 2, 3, 4, 5)) == 5


def test_forced_replay_reproduces():
    A, _ = rotscale_matrix(32, 5, 1e-3, 1e3)
    L, info = oracle.logm(A)
    Lf, infof = oracle.logm(A, force={"s": info["s"], "k": info["k"], "db_iters": info["db_iters"]})
    assert np.array_equal(L, Lf)
    assert infof["n_inv"] == info["n_inv"]


def test_forced_other_k_is_still_accurate():
    """Every shipped k is a valid approximation once ||B|| is small enough."""
    A = disk_matrix(16, 3, 0.001)
    L5, info = oracle.logm(A)
    for k in (3, 5):
        Lk, _ = oracle.logm(A, force={"s": 0, "k": k, "db_iters": []})
        assert relf(Lk, L5) < 1e-14


def test_flop_count_formula():
    A = disk_matrix(10, 1, 0.6)
    _, info = oracle.logm(A)
    n = 10
    assert info["flops"] == 2 * n ** 3 * (info["n_inv"] + info["n_gemm"]) + 2 * n ** 2 * info["n_matvec"]
    assert info["n_inv"] == sum(2 * it - 1 for it in info["db_iters"])
    assert info["n_gemm"] == info["k"]


def test_error_paths():
    with pytest.raises(oracle.OracleError) as e:
        oracle.logm(np.array([[1.0, np.nan], [0.0, 1.0]]))
    assert e.value.code == "ENONFINITE"
    with pytest.raises(oracle.OracleError) as e:
        oracle.logm(np.zeros((3, 3)))
    assert e.value.code == "ESINGULAR"
    with pytest.raises(oracle.OracleError):
        oracle.logm(np.diag([-1.0, 2.0]))      # eigenvalue on the negative real axis
    with pytest.raises(ValueError):
        oracle.logm(np.ones((2, 3)))
