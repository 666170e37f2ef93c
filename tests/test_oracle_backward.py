"""Pins of the oracle's reverse mode (gradient of <G, log A> with respect to A).

* closed form: for diagonal A, L_log(A, G)_ij = G_ij f[a_i, a_j] with the divided
  difference f[x, y] = (log x - log y) / (x - y), f[x, x] = 1 / x;
* block form: L_log(A^T, G) is the upper-right block of log([[A^T, G], [0, A^T]]);
* central finite differences of <G, log A> along random directions.
Each scheme (k = 1, 2, 3, 5) and both s = 0 and s > 0 are exercised, so a dropped
term, a missing transpose or a wrong coefficient in any adjoint fails a test."""

import numpy as np
import pytest

import oracle
from workloads import disk_matrix, rotscale_matrix


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def divided_difference_log(d):
    n = len(d)
    F = np.empty((n, n))
    for i in range(n):
        for j in range(n):
            F[i, j] = 1.0 / d[i] if d[i] == d[j] else (np.log(d[i]) - np.log(d[j])) / (d[i] - d[j])
    return F


@pytest.mark.parametrize("d", [[0.3, 1.5, 2.0, 7.0, 0.01], [1.01, 0.99, 1.0, 1.02], [1e-2, 1e2, 3.0]])
def test_backward_diagonal_closed_form(d):
    d = np.array(d)
    G = np.random.default_rng(11).standard_normal((len(d), len(d)))
    gA, _ = oracle.logm_backward(np.diag(d), G)
    assert rel(gA, G * divided_difference_log(d)) < 1e-13


@pytest.mark.parametrize("k_max", [1, 2, 3, 5])
@pytest.mark.parametrize("make", ["disk", "rotscale"])
def test_backward_matches_block_frechet(k_max, make):
    n = 10
    A = disk_matrix(n, 21) if make == "disk" else rotscale_matrix(n, 22, 1e-2, 1e2)[0]
    G = np.random.default_rng(23).standard_normal((n, n))
    gA, info = oracle.logm_backward(A, G, k_max=k_max)
    assert info["k"] <= k_max
    ref = oracle.frechet_block(A.T, G)
    assert rel(gA, ref) < 1e-12, (info["s"], info["k"])


def test_backward_s0_path_matches_block_frechet():
    n = 8
    R = np.random.default_rng(5).standard_normal((n, n))
    A = np.eye(n) + 0.05 * R / np.linalg.norm(R, 1)     # ||A - I||_1 below Theta_5: s = 0
    G = np.random.default_rng(6).standard_normal((n, n))
    gA, info = oracle.logm_backward(A, G)
    assert info["s"] == 0
    assert rel(gA, oracle.frechet_block(A.T, G)) < 1e-13


@pytest.mark.parametrize("seed", [1, 2])
def test_backward_central_differences(seed):
    n = 12
    A = rotscale_matrix(n, 4000 + seed, 1e-2, 1e2)[0]
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    gA, _ = oracle.logm_backward(A, G)
    h = 1e-6
    for _ in range(3):
        E = rng.standard_normal((n, n))
        fd = (np.sum(G * oracle.logm(A + h * E)[0]) - np.sum(G * oracle.logm(A - h * E)[0])) / (2 * h)
        assert abs(fd - np.sum(gA * E)) <= 1e-6 * abs(fd)


def test_backward_is_linear_in_G_and_replays_forced_decisions():
    n = 9
    A = disk_matrix(n, 31)
    rng = np.random.default_rng(32)
    G1, G2 = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    g1, info = oracle.logm_backward(A, G1)
    g2, _ = oracle.logm_backward(A, G2)
    g12, _ = oracle.logm_backward(A, 2.0 * G1 - G2)
    assert rel(g12, 2.0 * g1 - g2) < 1e-13
    forced = {"s": info["s"], "k": info["k"], "db_iters": info["db_iters"]}
    gf, _ = oracle.logm_backward(A, G1, force=forced)
    assert np.array_equal(gf, g1)
