"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds input generators only: designs X, responses y and batches
of correlation parameters theta.  It contains none of the likelihood's
arithmetic, and both the GPU path and the CPU oracle consume what it makes.

The paper's own data (maximin Latin-hypercube designs, Goldstein-Price and
Hartman-6 responses, Sec. 4) are not available; these generators stand in for
them with the same shapes: d from 2 to 12, n up to several thousand points in
the unit cube, smooth responses with a little noise.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    X: np.ndarray       # n x d, row-major, float64
    y: np.ndarray       # n, float64
    theta: np.ndarray   # B x d, float64
    p: float
    delta: float
    seed: int
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.X.shape[0]

    @property
    def d(self) -> int:
        return self.X.shape[1]

    @property
    def B(self) -> int:
        return self.theta.shape[0]


def uniform_design(n: int, d: int, rng: np.random.Generator) -> np.ndarray:
    return rng.random((n, d))


def lhs_design(n: int, d: int, rng: np.random.Generator) -> np.ndarray:
    """Latin-hypercube-like design: one point per stratum of width 1/n in
    every coordinate, x_ik = (pi_k(i) + u_ik) / n with random permutations."""
    X = np.empty((n, d))
    for k in range(d):
        X[:, k] = (rng.permutation(n) + rng.random(n)) / n
    return X


def sine_response(X: np.ndarray, rng: np.random.Generator, noise: float = 0.01) -> np.ndarray:
    """y_i = sum_k w_k sin(pi x_ik) + noise * eps_i, w_k ~ U(0.5, 2)."""
    n, d = X.shape
    w = rng.uniform(0.5, 2.0, d)
    return np.sin(np.pi * X) @ w + noise * rng.standard_normal(n)


def log_uniform_theta(B: int, d: int, lo: float, hi: float, rng: np.random.Generator) -> np.ndarray:
    return np.exp(rng.uniform(np.log(lo), np.log(hi), (B, d)))


def small_2d(seed: int = 1, n: int = 200, B: int = 64) -> Workload:
    """n=200, d=2, X ~ U[0,1]^2, y = sin(2 pi x1) + cos(2 pi x2) + 0.01 eps,
    p=2, nugget 1e-8, theta log-uniform on [0.1, 10]^2."""
    rng = np.random.default_rng(seed)
    X = uniform_design(n, 2, rng)
    y = np.sin(2 * np.pi * X[:, 0]) + np.cos(2 * np.pi * X[:, 1]) + 0.01 * rng.standard_normal(n)
    th = log_uniform_theta(B, 2, 0.1, 10.0, rng)
    return Workload("fp64_n200_d2", X, y, th, 2.0, 1e-8, seed)


def lhs_workload(name: str, n: int, d: int, B: int, p: float, delta: float, seed: int,
                 lo: float = 0.05, hi: float = 20.0) -> Workload:
    rng = np.random.default_rng(seed)
    X = lhs_design(n, d, rng)
    y = sine_response(X, rng)
    th = log_uniform_theta(B, d, lo, hi, rng)
    return Workload(name, X, y, th, p, delta, seed)


def fp64_at_scale(seed: int = 2, n: int = 4096, B: int = 128) -> Workload:
    """n=4096, d=8, LHS-like, p=1.95, nugget 1e-6, 128 theta in [0.05, 20]^8."""
    return lhs_workload("fp64_n4096_d8", n, 8, B, 1.95, 1e-6, seed)


def mixed_at_scale(seed: int = 3, n: int = 8192, B: int = 32) -> Workload:
    """n=8192, d=10, same generator, p=2, nugget 1e-6, 32 theta."""
    return lhs_workload("mixed_n8192_d10", n, 10, B, 2.0, 1e-6, seed)


def gradient_workload(seed: int = 5, n: int = 4096, B: int = 16) -> Workload:
    """n=4096, d=6, p=2, nugget 1e-6, 16 theta (finite-difference check)."""
    return lhs_workload("grad_n4096_d6", n, 6, B, 2.0, 1e-6, seed)


@dataclass
class PredictionWorkload:
    X: np.ndarray
    y: np.ndarray
    theta: np.ndarray
    p: float
    delta: float
    Xs: np.ndarray        # test points
    ys: np.ndarray        # noiseless response at the test points


def prediction_workload(seed: int = 8, n: int = 4096, d: int = 8, B: int = 8, N: int = 1000,
                        p: float = 1.95, delta: float = 1e-6) -> PredictionWorkload:
    """Training data as the n=4096, d=8 workload (LHS-like design, sine
    response with noise 0.01), an N-point LHS-like test set with the same
    response function without noise, and B theta in [0.05, 20]^d."""
    rng = np.random.default_rng(seed)
    X = lhs_design(n, d, rng)
    w = rng.uniform(0.5, 2.0, d)
    y = np.sin(np.pi * X) @ w + 0.01 * rng.standard_normal(n)
    Xs = lhs_design(N, d, rng)
    ys = np.sin(np.pi * Xs) @ w
    th = log_uniform_theta(B, d, 0.05, 20.0, rng)
    return PredictionWorkload(X, y, th, p, delta, Xs, ys)


def ga_workload(n: int, d: int, seed: int, N: int = 1000, p: float = 1.95,
                delta: float = 0.0) -> PredictionWorkload:
    """A fit at the shapes of the paper's examples (d = 2 or 6, n up to
    4064, p = 1.95, no nugget, a deterministic response): LHS-like design,
    sine response without noise, an N-point LHS-like test set with its
    response.  theta is left empty (the GA chooses it)."""
    rng = np.random.default_rng(seed)
    X = lhs_design(n, d, rng)
    w = rng.uniform(0.5, 2.0, d)
    y = np.sin(np.pi * X) @ w
    Xs = lhs_design(N, d, rng)
    ys = np.sin(np.pi * Xs) @ w
    return PredictionWorkload(X, y, np.empty((0, d)), p, delta, Xs, ys)


@dataclass
class ServingDataset:
    X: np.ndarray
    y: np.ndarray
    p: float
    delta: float


def serving_datasets(seed: int = 4, count: int = 64, n_lo: int = 256, n_hi: int = 6144,
                     d_lo: int = 2, d_hi: int = 12, delta: float = 1e-6):
    """64 resident datasets: n uniform over multiples of 64 in [256, 6144],
    d uniform in 2..12, p drawn from {1.5, 1.95, 2}."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.arange(n_lo, n_hi + 1, 64), size=count)
    ds = rng.integers(d_lo, d_hi + 1, size=count)
    ps = rng.choice(np.array([1.5, 1.95, 2.0]), size=count)
    out = []
    for n, d, p in zip(ns, ds, ps):
        X = lhs_design(int(n), int(d), rng)
        y = sine_response(X, rng)
        out.append(ServingDataset(X, y, float(p), delta))
    return out


def serving_requests(datasets, count: int, rate: float, seed: int = 6,
                     lo: float = 0.05, hi: float = 20.0):
    """(arrival_time, dataset_index, theta) with Poisson arrivals at `rate`/s
    and theta log-uniform on [lo, hi]^d of the chosen dataset."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps)
    reqs = []
    for q in range(count):
        k = int(rng.integers(0, len(datasets)))
        th = log_uniform_theta(1, datasets[k].X.shape[1], lo, hi, rng)[0]
        reqs.append((float(t[q]), k, th))
    return reqs
