"""Shared helpers for the GPU parity tests (tolerance rule and comparisons)."""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

import oracle

FP64_TOL = 1e-10   # stated tolerance of the FP64 path
SLACK = 10.0       # multiple of the FP64 rounding spread of independent codes


def scales(y):
    """Relative-error floors per output: 1 for log|R| and nll, sd(y) for mu,
    0 for sigma2 (always > 0 when info == 0)."""
    return {"logdet": 1.0, "nll": 1.0, "mu": float(np.std(y)) or 1.0, "sigma2": 0.0}


def lapack_fp64(X, y, theta, p, delta, family="powexp"):
    """A second, independent FP64 evaluation of eq. (3)-(4): LAPACK's blocked
    Cholesky (SciPy) on the oracle's R, triangular solves, two-pass Q.  Used
    only to measure how far two correct FP64 orderings drift apart."""
    n = X.shape[0]
    out = {k: np.full(theta.shape[0], np.nan) for k in ("logdet", "mu", "sigma2", "nll")}
    for t in range(theta.shape[0]):
        th = theta[t]
        if not np.all(np.isfinite(th)) or np.any(th < 0):
            continue
        R = oracle.corr(X, th, p, delta, family=family)
        try:
            L = np.tril(sla.cho_factor(R, lower=True)[0])
        except np.linalg.LinAlgError:
            continue
        a = sla.solve_triangular(L, np.ones(n), lower=True)
        b = sla.solve_triangular(L, y, lower=True)
        mu = a @ b / (a @ a)
        Q = np.sum((b - mu * a) ** 2)
        ld = 2 * np.sum(np.log(np.diag(L)))
        out["logdet"][t], out["mu"][t], out["sigma2"][t] = ld, mu, Q / n
        out["nll"][t] = ld + n * np.log(Q / n)
    return out


def tolerances(r64, r80, y, lap=None, floor=FP64_TOL):
    """Per-theta tolerance for each output:
        max(floor, SLACK * max(rel(oracle_f64, oracle_f80), rel(lapack_f64, oracle_f80))).
    An FP64 result cannot be expected closer to the exact value than two
    independent correct FP64 codes come for that theta's conditioning."""
    sc = scales(y)
    tol = {}
    for k in ("logdet", "mu", "sigma2", "nll"):
        err64 = oracle.rel(getattr(r64, k), getattr(r80, k), sc[k])
        if lap is not None:
            e2 = oracle.rel(lap[k], getattr(r80, k), sc[k])
            err64 = np.fmax(err64, np.where(np.isfinite(e2), e2, 0.0))
        tol[k] = np.maximum(floor, SLACK * err64)
    tol["floor"] = floor
    return tol


def compare(gpu: dict, r80, tol: dict, y, label=""):
    """Assert every output of every theta is within its tolerance of the
    80-bit oracle; returns the worst relative error per output."""
    sc = scales(y)
    worst = {}
    info = gpu["info"]
    assert np.array_equal(info, r80.info), f"{label}: info {info} vs {r80.info}"
    ok = info == 0
    for k in ("logdet", "mu", "sigma2", "nll"):
        e = oracle.rel(gpu[k][ok], getattr(r80, k)[ok], sc[k])
        bad = np.nonzero(e > tol[k][ok])[0]
        assert bad.size == 0, (f"{label}: {k} off for thetas {np.nonzero(ok)[0][bad]}: "
                               f"err {e[bad]} tol {tol[k][ok][bad]}")
        worst[k] = float(e.max()) if e.size else 0.0
    # how many thetas needed a bar above the floor (ill-conditioned R)
    floor = tol.get("floor", 0.0)
    relaxed = {k: int(np.sum(tol[k][ok] > floor)) for k in ("logdet", "mu", "sigma2", "nll")}
    print(f"{label}: thetas with a bar above the floor per output: {relaxed}", flush=True)
    return worst


def to_host(res: dict) -> dict:
    return {k: v.cpu().numpy() for k, v in res.items()}


def lapack_predict(X, y, theta, p, delta, Xs, family="powexp"):
    """A second, independent FP64 predictor for one theta (LAPACK Cholesky
    of the oracle's R, cho_solve, the cross-correlations from the oracle's
    correlation of the stacked points): mean and mse at the rows of Xs.  Used
    only to measure the FP64 rounding spread of the predictions."""
    n = X.shape[0]
    R = oracle.corr(X, theta, p, delta, family=family)
    cf = sla.cho_factor(R, lower=True)
    one = np.ones(n)
    Ri1 = sla.cho_solve(cf, one)
    mu = (Ri1 @ y) / (one @ Ri1)
    res = y - mu
    a = sla.cho_solve(cf, res)
    sigma2 = res @ a / n
    # cross-correlations without the nugget: the off-diagonal block of R of
    # the stacked points [X; Xs]
    full = oracle.corr(np.vstack([X, Xs]), theta, p, 0.0, family=family)
    r = full[:n, n:]
    u = sla.cho_solve(cf, r)
    mean = mu + r.T @ a
    mse = sigma2 * (1.0 - np.sum(r * u, axis=0) + (1.0 - one @ u) ** 2 / (one @ Ri1))
    return mean, mse


def pred_tolerance(m64, v64, m80, v80, mlap, vlap, sd_y, sigma2, floor=FP64_TOL):
    """Per-point tolerances of mean (scale sd(y)) and mse (scale sigma2):
    max(floor, SLACK * the larger distance of the two FP64 codes from the
    80-bit values)."""
    em = np.fmax(np.abs(m64 - m80), np.abs(mlap - m80)) / np.maximum(np.abs(m80), sd_y)
    ev = np.fmax(np.abs(v64 - v80), np.abs(vlap - v80)) / np.maximum(np.abs(v80), sigma2)
    return np.maximum(floor, SLACK * em), np.maximum(floor, SLACK * ev)


def _dlog_corr(diff, th, p, family):
    """-d ln(correlation factor) / d theta_k for one dimension (test-side
    restatement used only for the LAPACK gradient below)."""
    if family == "powexp":
        return np.where(diff == 0, 0.0, np.abs(diff) ** p)
    h = th * diff
    if family == "matern32":
        c = np.sqrt(3.0)
        return diff * c * c * h / (1 + c * h)
    c = np.sqrt(5.0)
    return diff * c * c * h * (1 + c * h) / (3 * (1 + c * h + c * c * h * h / 3))


def lapack_grad(X, y, theta, p, delta, family="powexp"):
    """A second, independent FP64 gradient of nll (adjoint formula with R^-1
    from LAPACK's Cholesky and dense NumPy sums), to measure the FP64
    rounding spread of the gradient.  theta: B x d."""
    n, d = X.shape
    out = np.full(theta.shape, np.nan)
    one = np.ones(n)
    for t in range(theta.shape[0]):
        R = oracle.corr(X, theta[t], p, delta, family=family)
        cf = sla.cho_factor(R, lower=True)
        Ri = sla.cho_solve(cf, np.eye(n))
        mu = (one @ sla.cho_solve(cf, y)) / (one @ sla.cho_solve(cf, one))
        alpha = sla.cho_solve(cf, y - mu)
        Q = (y - mu) @ alpha
        Wm = (n / Q) * np.outer(alpha, alpha) - Ri
        Roff = R - np.diag(np.diag(R))
        for k in range(d):
            diff = np.abs(X[:, k, None] - X[None, :, k])
            out[t, k] = np.sum(Roff * _dlog_corr(diff, theta[t, k], p, family) * Wm)
    return out


def grad_tolerance(g64, g80, glap, floor=1e-9, slack=20.0):
    """Per-component bar for a gradient: max(floor, slack x the larger
    distance of two FP64 codes from the 80-bit oracle), relative to
    max(|g80|, 1)."""
    scale = np.maximum(np.abs(g80), 1.0)
    spread = np.fmax(np.abs(g64 - g80), np.abs(glap - g80)) / scale
    return np.maximum(floor, slack * spread), scale
