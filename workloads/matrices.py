"""Synthetic matrices for the logarithm workloads (numpy PCG64 streams).

The paper's own test sets (Section 7) are not available; these constructions
stand in for them with the shapes and spectra the benchmark workloads name:

* ``disk_matrix``: A = I + rho * R / ||R||_2, R iid N(0,1), so every eigenvalue
  lies in the disk of radius rho about 1 (few square roots needed).
* ``rotscale_matrix``: A = V D V^{-1} with V = I + 0.1 N(0,1)/sqrt(n) and D block
  diagonal with 2x2 rotation-scaling blocks [[a, b], [-b, a]] (eigenvalues
  r e^{+-i theta}, log r uniform in [log r_lo, log r_hi], theta uniform in
  (-0.9 pi, 0.9 pi)); the exact principal logarithm V log(D) V^{-1} is known
  by construction (log of a block is [[log r, theta], [-theta, log r]]).
* ``spd_batch``: SPD covariance-like matrices X^T X / 64 + 1e-3 I of uneven
  sizes (batched workload).
"""

from __future__ import annotations

import numpy as np

# Seeds of the named workloads.
CONFIG_SEEDS = {
    "disk64": 1001,
    "rotscale1024": 2001,
    "rotscale4096": 2002,
    "spd_batch": 3001,
    "rotscale64_batch": 4001,
    "rotscale8192": 5001,
}


def disk_matrix(n: int, seed: int, rho: float = 0.8) -> np.ndarray:
    """A = I + rho R/||R||_2 with R iid standard normal."""
    rng = np.random.default_rng(seed)
    R = rng.standard_normal((n, n))
    return np.eye(n) + rho * R / np.linalg.norm(R, 2)


def rotscale_matrix(n: int, seed: int, r_lo: float = 1e-3, r_hi: float = 1e3,
                    with_log: bool = True, theta_max: float = 0.9):
    """Real A = V D V^{-1} with conjugate-pair spectrum; returns (A, log A exact).

    theta ~ U(-theta_max pi, theta_max pi) (0.9 in the benchmark workloads; values
    near 1 put eigenvalues close to the negative real axis).  For odd n the last
    eigenvalue is real and positive (log-uniform like r).
    """
    rng = np.random.default_rng(seed)
    V = np.eye(n) + 0.1 * rng.standard_normal((n, n)) / np.sqrt(n)
    npair = n // 2
    r = np.exp(rng.uniform(np.log(r_lo), np.log(r_hi), size=npair + (n % 2)))
    theta = rng.uniform(-theta_max * np.pi, theta_max * np.pi, size=npair)
    a = r[:npair] * np.cos(theta)
    b = r[:npair] * np.sin(theta)
    D = np.zeros((n, n))
    LD = np.zeros((n, n))
    idx = 2 * np.arange(npair)
    D[idx, idx] = a
    D[idx + 1, idx + 1] = a
    D[idx, idx + 1] = b
    D[idx + 1, idx] = -b
    LD[idx, idx] = np.log(r[:npair])
    LD[idx + 1, idx + 1] = np.log(r[:npair])
    LD[idx, idx + 1] = theta
    LD[idx + 1, idx] = -theta
    if n % 2:
        D[n - 1, n - 1] = r[npair]
        LD[n - 1, n - 1] = np.log(r[npair])
    Vinv = np.linalg.inv(V)
    A = (V @ D) @ Vinv
    if not with_log:
        return A, None
    return A, (V @ LD) @ Vinv


def spd_batch(count: int, seed: int, n_lo: int = 8, n_hi: int = 128):
    """List of SPD matrices X_i^T X_i / 64 + 1e-3 I, X_i 64 x n_i, n_i uniform."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(n_lo, n_hi + 1, size=count)
    out = []
    for n in sizes:
        Xm = rng.standard_normal((64, int(n)))
        out.append(Xm.T @ Xm / 64.0 + 1e-3 * np.eye(int(n)))
    return out


def named_workload(name: str):
    """(A, exact log or None) for a named single-matrix workload."""
    seed = CONFIG_SEEDS[name]
    if name == "disk64":
        return disk_matrix(64, seed), None
    if name == "rotscale1024":
        return rotscale_matrix(1024, seed)
    if name == "rotscale4096":
        return rotscale_matrix(4096, seed)
    if name == "rotscale8192":
        return rotscale_matrix(8192, seed, 1e-2, 1e2)
    raise KeyError(name)


def complex_matrix(n: int, seed: int, r_lo: float = 1e-2, r_hi: float = 1e2):
    """Complex A = V diag(lambda) V^{-1} with V = I + 0.1 (N + iN)/sqrt(2n) and
    lambda = r e^{i theta}, log r uniform in [log r_lo, log r_hi], theta uniform in
    (-0.9 pi, 0.9 pi); returns (A, log A exact) with log A = V diag(log lambda) V^{-1}."""
    rng = np.random.default_rng(seed)
    V = np.eye(n) + 0.1 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
    logr = rng.uniform(np.log(r_lo), np.log(r_hi), size=n)
    theta = rng.uniform(-0.9 * np.pi, 0.9 * np.pi, size=n)
    loglam = logr + 1j * theta
    Vi = np.linalg.inv(V)
    A = (V * np.exp(loglam)) @ Vi
    L = (V * loglam) @ Vi
    return A, L


def real_representation(A: np.ndarray) -> np.ndarray:
    """[[Re A, -Im A], [Im A, Re A]]: the 2n x 2n real matrix of the complex A."""
    return np.block([[A.real, -A.imag], [A.imag, A.real]])
