"""Pivoting under stress.  The inversions pick pivot rows by tournament pivoting
with a threshold (a pivot within 1 + 2^-17 of its column's largest candidate at each
tournament level) or, in the square-root iteration, reuse the previous inversion's
row order when every multiplier stays within 2.  These tests take inputs where the
choice matters: a condition number of 1e10, rows scaled over twelve orders of
magnitude, the Wilkinson matrix (element growth 2^(n-1) under partial pivoting), and
logarithms whose eigenvalues lie close to the negative real axis, so that the
Denman-Beavers iterates are nearly singular in the first iterations."""

import numpy as np
import pytest

import oracle
from workloads import rotscale_matrix

torch = pytest.importorskip("torch")
lm = pytest.importorskip("paper_2401_10089_amd")

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lm.load_library()
    yield
    torch.cuda.synchronize()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relf(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def left_residual(A, X):
    """Normwise left residual of an inverse, ||X A - I||_1 / (||A||_1 ||X||_1).  Gauss-
    Jordan elimination applies row operations to A, so this one is of order n u
    whatever the condition number; the right residual A X - I of the blocked form
    (rank-256 updates through the processed panel) grows like kappa u, as a NumPy
    model of the same blocking shows (1e-9 at kappa = 1e11, n = 300), while the
    forward error stays that of LAPACK's inverse."""
    n = A.shape[0]
    return np.linalg.norm(X @ A - np.eye(n), 1) / (np.linalg.norm(A, 1) * np.linalg.norm(X, 1))


@pytest.mark.parametrize("n", [300, 1024])
def test_inverse_condition_1e10(n):
    rng = np.random.default_rng(5100 + n)
    Q1, _ = np.linalg.qr(rng.standard_normal((n, n)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Q1 * np.logspace(0, -10, n)) @ Q2
    Xg, ld = lm.inverse(dev(A))
    Xg = host(Xg)
    Xn = np.linalg.inv(A)
    assert left_residual(A, Xg) < 10 * n * U
    kappa = np.linalg.cond(A, 1)
    # both are within kappa u of the exact inverse; measured distance ~1e-7
    assert relf(Xg, Xn) < n * kappa * U
    assert ld == pytest.approx(np.linalg.slogdet(A)[1], rel=1e-10)


def test_inverse_rows_scaled_over_twelve_decades():
    n = 520
    rng = np.random.default_rng(5200)
    A = 10.0 ** rng.uniform(-6, 6, size=(n, 1)) * (rng.standard_normal((n, n)) + 2 * np.eye(n))
    Xg, _ = lm.inverse(dev(A))
    Xg = host(Xg)
    Xn = np.linalg.inv(A)
    assert left_residual(A, Xg) < 10 * n * U
    # row scaling is a left diagonal similarity of the problem: the error relative to
    # the unscaled inverse stays at the unscaled matrix's conditioning
    d = np.abs(A).max(axis=1)
    kappa_scaled = np.linalg.cond(A / d[:, None], 1)
    assert relf(Xg * d[None, :], Xn * d[None, :]) < 20 * n * kappa_scaled * U


@pytest.mark.parametrize("n", [24, 40])
def test_inverse_wilkinson_growth(n):
    """W: 1 on the diagonal and in the last column, -1 below the diagonal; partial
    pivoting keeps the diagonal and the last column doubles at every step (growth
    2^(n-1)).  The exact inverse comes from rational Gauss-Jordan elimination on the
    host."""
    from fractions import Fraction

    W = np.tril(-np.ones((n, n)), -1) + np.eye(n)
    W[:, -1] = 1.0
    M = [[Fraction(int(W[i, j])) for j in range(n)] + [Fraction(int(i == j)) for j in range(n)]
         for i in range(n)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        piv = M[c][c]
        M[c] = [v / piv for v in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [a - f * b for a, b in zip(M[r], M[c])]
    X_exact = np.array([[float(v) for v in row[n:]] for row in M])
    Xg, ld = lm.inverse(dev(W))
    Xg = host(Xg)
    Xn = np.linalg.inv(W)
    err_g, err_n = relf(Xg, X_exact), relf(Xn, X_exact)
    print(f"n={n}: error {err_g:.2e} (LAPACK {err_n:.2e})")
    # W is well conditioned (kappa ~ n); LAPACK happens to be exact on it.  The
    # tournament breaks the magnitude ties differently, so its elimination is not
    # exact, but its error must be that of a stable inversion, far below the growth
    # bound of partial pivoting
    kappa = np.linalg.cond(W, 1)
    assert err_g <= max(10 * err_n, 100 * n * kappa * U)
    assert err_g < 2.0 ** (n - 1) * n * U
    assert ld == pytest.approx(np.log(2.0) * (n - 1), rel=1e-12)


@pytest.mark.parametrize("n,seed,theta_max", [(256, 72, 0.99), (300, 73, 0.999)])
@pytest.mark.parametrize("pivot_search", [False, True])
def test_logm_eigenvalues_near_negative_axis(n, seed, theta_max, pivot_search):
    """Eigenvalue pairs up to 0.1% of pi from the negative real axis: the first
    Denman-Beavers iterates are nearly singular.  With and without the reuse of row
    orders, against the oracle (same decisions, or a replay of the device's) and the
    exact logarithm."""
    A, Lx = rotscale_matrix(n, seed, theta_max=theta_max)
    L, info = lm.logm(dev(A), pivot_search=pivot_search)
    Lg = host(L)
    Lo, io = oracle.logm(A)
    if (info["s"], info["k"], info["db_iters"]) != (io["s"], io["k"], io["db_iters"]):
        assert (info["s"], info["k"]) == (io["s"], io["k"])
        Lo, _ = oracle.logm(A, force={"s": info["s"], "k": info["k"], "db_iters": info["db_iters"]})
    assert relf(Lg, Lo) < 1e-12
    assert relf(Lg, Lx) < 1e-11
    if not pivot_search and n > 256:   # orders are reused above one outer block
        assert info["n_inv_reordered"] > 0
