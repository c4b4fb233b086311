"""The stated limits of the C ABI at their maximum: d = GP_DMAX (32, the
widest kernel instantiation) through every entry point that builds
correlations, and a batch of GP_BATCH_MAX thetas (the largest grid the
kernels are launched with) on a small n.  n = GP_NMAX (8192) is covered by
the n=8192 launches of test_gpu_mixed.py."""
import numpy as np
import pytest

import oracle
from paper_1203_1269_amd import inputs
from parity_util import (compare, grad_tolerance, lapack_fp64, lapack_grad, lapack_predict,
                         pred_tolerance, to_host, tolerances)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1203_1269_amd import binding
    binding.lib()
    return binding


@pytest.mark.parametrize("family,p", [("powexp", 1.95), ("matern52", 2.0)])
def test_d_max_all_entry_points(gp, family, p):
    d = gp.header_constant("GP_DMAX")
    assert d == 32
    rng = np.random.default_rng(6100)
    n = 333
    X = inputs.lhs_design(n, d, rng)
    y = inputs.sine_response(X, rng)
    th = inputs.log_uniform_theta(3, d, 0.01, 0.5, rng)
    print(f"[parity] d=32 {family} n={n}", flush=True)
    ds = gp.Dataset(X, y, p, 1e-6, corr=family)
    r64 = oracle.nll_batch(X, y, th, p, 1e-6, family=family)
    r80 = oracle.nll_batch(X, y, th, p, 1e-6, extended=True, family=family)
    tol = tolerances(r64, r80, y, lapack_fp64(X, y, th, p, 1e-6, family=family))
    assert np.all(r80.info == 0)
    compare(to_host(gp.nll_batch(ds, th)), r80, tol, y, "d=32 fp64")
    compare(to_host(gp.nll_batch(ds, th, prec="mixed")), r80,
            {k: np.maximum(v, 1e-8) for k, v in tol.items()}, y, "d=32 mixed")
    res, g = gp.nll_grad(ds, th)
    compare(to_host(res), r80, tol, y, "d=32 grad values")
    _, g64 = oracle.grad_batch(X, y, th, p, 1e-6, family=family)
    _, g80 = oracle.grad_batch(X, y, th, p, 1e-6, extended=True, family=family)
    gtol, scale = grad_tolerance(g64, g80, lapack_grad(X, y, th, p, 1e-6, family=family))
    err = np.abs(g.cpu().numpy() - g80) / scale
    print("d=32 gradient max rel err", err.max(), "bar", gtol.min(), flush=True)
    assert np.all(err <= gtol), (err.max(), gtol[err > gtol])
    Xs = inputs.lhs_design(20, d, rng)
    fit, mean, mse = gp.predict(ds, th[:1], Xs)
    m80, v80, f80 = oracle.predict(X, y, th[0], p, 1e-6, Xs, extended=True, family=family)
    m64, v64, _ = oracle.predict(X, y, th[0], p, 1e-6, Xs, family=family)
    ml, vl = lapack_predict(X, y, th[0], p, 1e-6, Xs, family=family)
    tm, tv = pred_tolerance(m64, v64, m80, v80, ml, vl, float(np.std(y)), float(f80.sigma2[0]))
    em = np.abs(mean[0].cpu().numpy() - m80) / np.maximum(np.abs(m80), np.std(y))
    ev = np.abs(mse[0].cpu().numpy() - v80) / np.maximum(np.abs(v80), f80.sigma2[0])
    assert np.all(em <= tm) and np.all(ev <= tv)


def test_batch_max(gp):
    """GP_BATCH_MAX thetas in one call (n = 70, two 64-blocks with padding):
    sampled thetas against the oracle, and the first theta bitwise as alone."""
    bmax = gp.header_constant("GP_BATCH_MAX")
    rng = np.random.default_rng(6200)
    n, d = 70, 3
    X = inputs.lhs_design(n, d, rng)
    y = inputs.sine_response(X, rng)
    th = inputs.log_uniform_theta(bmax, d, 0.05, 20, rng)
    print(f"[parity] batch {bmax} n={n}", flush=True)
    ds = gp.Dataset(X, y, 2.0, 1e-6)
    got = to_host(gp.nll_batch(ds, th))
    torch.cuda.empty_cache()
    assert got["nll"].shape == (bmax,)
    idx = np.array([0, 1, 12345, 40000, bmax - 2, bmax - 1])
    r64 = oracle.nll_batch(X, y, th[idx], 2.0, 1e-6)
    r80 = oracle.nll_batch(X, y, th[idx], 2.0, 1e-6, extended=True)
    tol = tolerances(r64, r80, y, lapack_fp64(X, y, th[idx], 2.0, 1e-6))
    compare({k: v[idx] for k, v in got.items()}, r80, tol, y, "batch max")
    one = to_host(gp.nll_batch(ds, th[bmax - 1:]))
    assert one["nll"][0] == got["nll"][bmax - 1]
    with pytest.raises(gp.GPError):
        gp.nll_batch(ds, np.ones((bmax + 1, d)))
