"""The Matern correlation families (smoothness 3/2 and 5/2, the alternative
to eq. 2 that Sec. 2 names) through every entry point that builds
correlations: gp_corr_build, gp_nll_batch (FP64 and the matched mixed
mode), gp_nll_grad and gp_predict, against the oracle's Matern families.

Bars as for the power exponential: entries of R to 1e-13 relative; the
likelihood outputs within max(1e-10, 10 x the FP64 rounding spread) of the
80-bit oracle (1e-8 floor for the mixed mode); gradients within max(1e-9,
20 x the oracle's FP64 spread); predictions as in test_gpu_predict."""
import numpy as np
import pytest

import oracle
from paper_1203_1269_amd import inputs
from parity_util import (compare, lapack_fp64, lapack_predict, pred_tolerance, to_host,
                         tolerances)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
FAMILIES = ["matern32", "matern52"]


@pytest.fixture(scope="module")
def gp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1203_1269_amd import binding
    binding.lib()
    return binding


def _case(n, d, B, seed, lo=0.05, hi=20.0):
    rng = np.random.default_rng(seed)
    X = inputs.lhs_design(n, d, rng)
    y = inputs.sine_response(X, rng)
    th = inputs.log_uniform_theta(B, d, lo, hi, rng)
    return X, y, th, rng


@pytest.mark.parametrize("family", FAMILIES)
@pytest.mark.parametrize("n,d", [(130, 3), (700, 9)])
def test_matern_corr_build_entrywise(gp, family, n, d):
    X, _, th, _ = _case(n, d, 3, 400 + n)
    print(f"[parity] matern corr_build {family} n={n} d={d}", flush=True)
    ds = gp.Dataset(X, np.zeros(n), 2.0, 1e-6, corr=family)
    R, info = gp.corr_build(ds, th)
    R = R.cpu().numpy()
    assert np.all(info.cpu().numpy() == 0)
    low = np.tril(np.ones((n, n), dtype=bool))
    for b in range(3):
        G = R[b].T
        ref = oracle.corr(X, th[b], 2.0, 1e-6, extended=True, family=family)
        err = np.abs(G[:n, :n] - ref)[low]
        assert np.all(err <= 1e-13 * np.abs(ref[low]) + 1e-300), err.max()


@pytest.mark.parametrize("family", FAMILIES)
@pytest.mark.parametrize("n,d,delta,B", [
    (300, 2, 1e-6, 4),      # one outer panel
    (1500, 8, 1e-6, 3),     # three panels with the lookahead
    (1000, 12, 1e-8, 3),    # d > 8, small nugget
])
def test_matern_nll_fp64_against_oracle(gp, family, n, d, delta, B):
    X, y, th, _ = _case(n, d, B, 410 + n)
    print(f"[parity] matern nll {family} n={n} d={d} delta={delta}", flush=True)
    ds = gp.Dataset(X, y, 2.0, delta, corr=family)
    got = to_host(gp.nll_batch(ds, th))
    r64 = oracle.nll_batch(X, y, th, 2.0, delta, family=family)
    r80 = oracle.nll_batch(X, y, th, 2.0, delta, extended=True, family=family)
    tol = tolerances(r64, r80, y, lapack_fp64(X, y, th, 2.0, delta, family=family))
    worst = compare(got, r80, tol, y, f"matern {family} n={n}")
    print("worst rel err vs 80-bit oracle:", worst, flush=True)


@pytest.mark.parametrize("family", FAMILIES)
def test_matern_mixed_matched(gp, family):
    n, d, B = 2048, 6, 4
    X, y, th, _ = _case(n, d, B, 420)
    print(f"[parity] matern mixed {family} n={n}", flush=True)
    ds = gp.Dataset(X, y, 2.0, 1e-6, corr=family)
    got = to_host(gp.nll_batch(ds, th, prec="mixed"))
    r64 = oracle.nll_batch(X, y, th, 2.0, 1e-6, family=family)
    r80 = oracle.nll_batch(X, y, th, 2.0, 1e-6, extended=True, family=family)
    tol = tolerances(r64, r80, y, lapack_fp64(X, y, th, 2.0, 1e-6, family=family), floor=1e-8)
    compare(got, r80, tol, y, f"matern mixed {family}")


@pytest.mark.parametrize("family", FAMILIES)
def test_matern_gradient_against_oracle(gp, family):
    n, d = 400, 4
    X, y, th, _ = _case(n, d, 3, 430, lo=0.2, hi=20)
    print(f"[parity] matern gradient {family} n={n}", flush=True)
    ds = gp.Dataset(X, y, 2.0, 1e-6, corr=family)
    res, g = gp.nll_grad(ds, th)
    res, g = to_host(res), g.cpu().numpy()
    r64 = oracle.nll_batch(X, y, th, 2.0, 1e-6, family=family)
    r80 = oracle.nll_batch(X, y, th, 2.0, 1e-6, extended=True, family=family)
    compare(res, r80, tolerances(r64, r80, y, lapack_fp64(X, y, th, 2.0, 1e-6, family=family)), y,
            "matern grad values")
    _, g64 = oracle.grad_batch(X, y, th, 2.0, 1e-6, family=family)
    _, g80 = oracle.grad_batch(X, y, th, 2.0, 1e-6, extended=True, family=family)
    scale = np.maximum(np.abs(g80), 1.0)
    err = np.abs(g - g80) / scale
    tol = np.maximum(1e-9, 20 * np.abs(g64 - g80) / scale)
    print("grad max rel err", err.max(), flush=True)
    assert np.all(err <= tol), (err, tol)


@pytest.mark.parametrize("family", FAMILIES)
def test_matern_predict_against_oracle(gp, family):
    n, d, N = 900, 5, 70
    X, y, th, rng = _case(n, d, 2, 440)
    Xs = inputs.lhs_design(N, d, rng)
    print(f"[parity] matern predict {family} n={n} N={N}", flush=True)
    ds = gp.Dataset(X, y, 2.0, 1e-6, corr=family)
    fit, mean, mse = gp.predict(ds, th, Xs)
    fit = to_host(fit)
    mean, mse = mean.cpu().numpy(), mse.cpu().numpy()
    assert np.all(fit["info"] == 0)
    sd = float(np.std(y))
    for t in range(2):
        m80, v80, f80 = oracle.predict(X, y, th[t], 2.0, 1e-6, Xs, extended=True, family=family)
        m64, v64, _ = oracle.predict(X, y, th[t], 2.0, 1e-6, Xs, family=family)
        ml, vl = lapack_predict(X, y, th[t], 2.0, 1e-6, Xs, family=family)
        s2 = float(f80.sigma2[0])
        tm, tv = pred_tolerance(m64, v64, m80, v80, ml, vl, sd, s2)
        em = np.abs(mean[t] - m80) / np.maximum(np.abs(m80), sd)
        ev = np.abs(mse[t] - v80) / np.maximum(np.abs(v80), s2)
        assert np.all(em <= tm) and np.all(ev <= tv), (t, em.max(), ev.max())


def test_families_differ_and_p_is_ignored_for_matern(gp):
    """The family field selects the correlation (same data, three different
    likelihoods); for a Matern family the power exponent plays no part."""
    X, y, th, _ = _case(200, 3, 2, 450)
    print("[parity] family selection n=200", flush=True)
    v = {}
    for fam in ("powexp", "matern32", "matern52"):
        v[fam] = to_host(gp.nll_batch(gp.Dataset(X, y, 1.95, 1e-6, corr=fam), th))["nll"]
    assert not np.allclose(v["powexp"], v["matern32"]) and not np.allclose(v["matern32"],
                                                                              v["matern52"])
    a = to_host(gp.nll_batch(gp.Dataset(X, y, 1.0, 1e-6, corr="matern52"), th))["nll"]
    assert np.array_equal(a, v["matern52"])
