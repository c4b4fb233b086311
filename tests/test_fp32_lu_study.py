"""How far a single-precision LU evaluation of -2logL (the paper's GPU route:
R built in FP32, an FP32 LU factorisation, FP32 solves, Sec. 3-4) lands from
the exact value, next to an FP64 evaluation, at the shapes of the paper's
two examples (p = 1.95, no nugget).  The paper attributes the differences
between its CPU and GPU tables partly to this precision (Sec. 4-5); the
FP64 and matched mixed paths of this library avoid it.

FP32 LU: LAPACK's sgetrf/sgetrs through SciPy on an R computed in float32;
reference: the 80-bit oracle."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from paper_1203_1269_amd import inputs


def nll_fp32_lu(X, y, theta, p, delta):
    n = X.shape[0]
    X32 = X.astype(np.float32)
    diff = np.abs(X32[:, None, :] - X32[None, :, :])
    s = np.sum(theta.astype(np.float32) * diff ** np.float32(p), axis=2, dtype=np.float32)
    R = np.exp(-s).astype(np.float32)
    R[np.diag_indices(n)] += np.float32(delta)
    lu, piv = sla.lu_factor(R, check_finite=False)
    assert lu.dtype == np.float32
    logdet = np.sum(np.log(np.abs(np.diag(lu))), dtype=np.float32)
    one = np.ones(n, np.float32)
    y32 = y.astype(np.float32)
    mu = (one @ sla.lu_solve((lu, piv), y32)) / (one @ sla.lu_solve((lu, piv), one))
    r = y32 - mu
    Q = r @ sla.lu_solve((lu, piv), r)
    return float(logdet + n * np.log(Q / n))


@pytest.mark.parametrize("n,d", [(128, 2), (512, 2), (256, 6), (1024, 6)])
def test_fp32_lu_discrepancy(n, d):
    w = inputs.ga_workload(n, d, seed=5)
    th = inputs.log_uniform_theta(6, d, 0.5, 20, np.random.default_rng(1))
    r80 = oracle.nll_batch(w.X, w.y, th, 1.95, 0.0, extended=True)
    r64 = oracle.nll_batch(w.X, w.y, th, 1.95, 0.0)
    assert np.all(r80.info == 0)
    e32 = np.array([abs(nll_fp32_lu(w.X, w.y, th[t], 1.95, 0.0) - r80.nll[t]) for t in range(6)])
    e64 = np.abs(r64.nll - r80.nll)
    print(f"n={n} d={d}: |-2logL error| FP32 LU median {np.median(e32):.3g} max {e32.max():.3g}; "
          f"FP64 max {e64.max():.3g}")
    # single precision loses at least three more digits than double here
    assert np.median(e32) > 1e3 * max(e64.max(), 1e-13)
    assert np.all(e64 <= 1e-9 * np.abs(r80.nll))
