"""Kriging prediction on the GPU (gp_predict: the [1 y] and cross-correlation
rows factored below R, then the predictor reduction) against the 80-bit
oracle, through the C ABI.

Bar: the fit (log|R|, mu, sigma2, -2logL, info) as gp_nll_batch's; mean and
mse at every test point within max(1e-10, 10 x the FP64 rounding spread of
two independent FP64 predictors for that point) of the 80-bit oracle, the
mean relative to max(|mean|, sd(y)), the mse relative to max(|mse|, sigma2).
Shapes span one to several outer panels (with the lookahead), ragged test
sets and N = 0; the full-size launch is checked at the stored sampled points.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1203_1269_amd import inputs
from parity_util import (FP64_TOL, compare, lapack_fp64, lapack_predict, pred_tolerance,
                         scales, to_host, tolerances)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def gp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1203_1269_amd import binding
    binding.lib()
    return binding


def _check_points(X, y, th, p, delta, Xs, mean, mse, label):
    """mean[t], mse[t] (host) against the oracle for every theta row."""
    worst = [0.0, 0.0]
    for t in range(th.shape[0]):
        m80, v80, f80 = oracle.predict(X, y, th[t], p, delta, Xs, extended=True)
        m64, v64, _ = oracle.predict(X, y, th[t], p, delta, Xs)
        ml, vl = lapack_predict(X, y, th[t], p, delta, Xs)
        s2 = float(f80.sigma2[0])
        tm, tv = pred_tolerance(m64, v64, m80, v80, ml, vl, float(np.std(y)), s2)
        em = np.abs(mean[t] - m80) / np.maximum(np.abs(m80), np.std(y))
        ev = np.abs(mse[t] - v80) / np.maximum(np.abs(v80), s2)
        bad = np.nonzero((em > tm) | (ev > tv))[0]
        assert bad.size == 0, (label, t, bad[:5], em[bad[:5]], tm[bad[:5]], ev[bad[:5]],
                               tv[bad[:5]])
        worst = [max(worst[0], float(em.max())), max(worst[1], float(ev.max()))]
    return worst


@pytest.mark.parametrize("n,d,p,delta,B,N", [
    (300, 2, 2.0, 1e-6, 3, 100),     # one outer panel, ragged test set
    (1000, 3, 1.5, 1e-8, 2, 77),     # two panels, small nugget
    (1500, 8, 1.95, 1e-6, 2, 130),   # three panels: the lookahead updates test rows
    (2048, 6, 1.0, 1e-6, 2, 64),     # p = 1, exactly one 64-row test block
])
def test_predict_against_oracle(gp, n, d, p, delta, B, N):
    rng = np.random.default_rng(9000 + n)
    X = inputs.lhs_design(n, d, rng)
    y = inputs.sine_response(X, rng)
    Xs = inputs.lhs_design(N, d, rng)
    th = inputs.log_uniform_theta(B, d, 0.05, 20, rng)
    print(f"[parity] predict n={n} d={d} p={p} delta={delta} B={B} N={N}", flush=True)
    ds = gp.Dataset(X, y, p, delta)
    fit, mean, mse = gp.predict(ds, th, Xs)
    fit = to_host(fit)
    mean, mse = mean.cpu().numpy(), mse.cpu().numpy()
    r64 = oracle.nll_batch(X, y, th, p, delta)
    r80 = oracle.nll_batch(X, y, th, p, delta, extended=True)
    tol = tolerances(r64, r80, y, lapack_fp64(X, y, th, p, delta))
    compare(fit, r80, tol, y, f"predict fit n={n}")
    worst = _check_points(X, y, th, p, delta, Xs, mean, mse, f"predict n={n}")
    print("predict worst rel err (mean, mse) vs 80-bit oracle:", worst, flush=True)


def test_predict_fit_matches_nll_batch(gp):
    """The factorisation with the extra rows leaves R's factor as without
    them: log|R| as gp_nll_batch's to 1e-14, the other outputs to the FP64
    bar.  N = 0 returns the fit alone."""
    rng = np.random.default_rng(9300)
    n, d = 1700, 5
    X = inputs.lhs_design(n, d, rng)
    y = inputs.sine_response(X, rng)
    th = inputs.log_uniform_theta(6, d, 0.05, 20, rng)
    print("[parity] predict fit vs nll_batch n=1700, N=0 and N=5", flush=True)
    ds = gp.Dataset(X, y, 1.95, 1e-6)
    ref = to_host(gp.nll_batch(ds, th))
    f0, m0, v0 = gp.predict(ds, th, np.zeros((0, d)))
    f5, m5, v5 = gp.predict(ds, th, inputs.lhs_design(5, d, rng))
    assert m0.shape == (6, 0) and m5.shape == (6, 5)
    sc = scales(y)
    for f in (to_host(f0), to_host(f5)):
        assert np.array_equal(f["info"], ref["info"])
        assert np.all(oracle.rel(f["logdet"], ref["logdet"], 1.0) <= 1e-14)
        for k in ("mu", "sigma2", "nll"):
            assert np.all(oracle.rel(f[k], ref[k], sc[k]) <= FP64_TOL), k


def test_predict_interpolates_without_nugget(gp):
    """delta = 0: at design points the predictor returns the observed y and
    a zero mse (to rounding); the rest of the test set follows the oracle."""
    rng = np.random.default_rng(9400)
    n, d = 500, 3
    X = inputs.lhs_design(n, d, rng)
    y = inputs.sine_response(X, rng)
    th = inputs.log_uniform_theta(2, d, 30, 100, rng)
    at = np.array([0, 17, 250, 499])
    Xs = np.vstack([X[at], inputs.lhs_design(60, d, rng)])
    print("[parity] predict interpolation n=500 delta=0", flush=True)
    ds = gp.Dataset(X, y, 2.0, 0.0)
    fit, mean, mse = gp.predict(ds, th, Xs)
    fit = to_host(fit)
    mean, mse = mean.cpu().numpy(), mse.cpu().numpy()
    assert np.all(fit["info"] == 0)
    for t in range(2):
        assert np.all(np.abs(mean[t, :4] - y[at]) <= 1e-8 * np.std(y))
        assert np.all(np.abs(mse[t, :4]) <= 1e-8 * fit["sigma2"][t])
    _check_points(X, y, th, 2.0, 0.0, Xs, mean, mse, "interpolation")


def test_predict_edge_thetas(gp):
    """An invalid theta (-3) and a numerically singular R (info > 0) give NaN
    predictions; the other thetas of the batch follow the oracle."""
    rng = np.random.default_rng(9500)
    n, d = 700, 3
    X = inputs.lhs_design(n, d, rng)
    y = inputs.sine_response(X, rng)
    th = np.vstack([inputs.log_uniform_theta(1, d, 30, 100, rng),
                    np.array([[1.0, -1.0, 1.0]]),
                    np.full((1, d), 1e-3),
                    inputs.log_uniform_theta(1, d, 30, 100, rng)])
    Xs = inputs.lhs_design(40, d, rng)
    print("[parity] predict edge thetas n=700 delta=0", flush=True)
    ds = gp.Dataset(X, y, 2.0, 0.0)
    fit, mean, mse = gp.predict(ds, th, Xs)
    fit = to_host(fit)
    mean, mse = mean.cpu().numpy(), mse.cpu().numpy()
    assert fit["info"][1] == -3 and fit["info"][2] > 0
    for t in (1, 2):
        assert np.all(np.isnan(mean[t])) and np.all(np.isnan(mse[t]))
    assert fit["info"][0] == 0 and fit["info"][3] == 0
    _check_points(X, y, th[[0, 3]], 2.0, 0.0, Xs, mean[[0, 3]], mse[[0, 3]], "edge")


def test_predict_rejects_bad_arguments(gp):
    rng = np.random.default_rng(9600)
    X = inputs.lhs_design(200, 2, rng)
    y = inputs.sine_response(X, rng)
    ds = gp.Dataset(X, y, 2.0, 1e-6)
    assert gp.predict_workspace_bytes(200, 2, 1, (1 << 20) + 1) == 0
    assert gp.predict_workspace_bytes(200, 2, 1, 10) > 0
    with pytest.raises(gp.GPError):
        gp.predict(ds, np.ones((1, 2)), np.zeros(((1 << 20) + 1, 2)))


def test_fullsize_predict_n4096_d8(gp):
    """The benchmarked prediction launch (n=4096, d=8, 8 thetas, 1000 test
    points) against the stored oracle values at the sampled thetas and test
    points."""
    path = os.path.join(HERE, "golden", "pred_n4096_d8_expected.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    exp = json.load(open(path))
    w = inputs.prediction_workload()
    print("[parity] fullsize predict n=4096 d=8 B=8 N=1000", flush=True)
    ds = gp.Dataset(w.X, w.y, w.p, w.delta)
    fit, mean, mse = gp.predict(ds, w.theta, w.Xs)
    fit = to_host(fit)
    mean, mse = mean.cpu().numpy(), mse.cpu().numpy()
    assert np.all(fit["info"] == 0)
    sd = float(np.std(w.y))
    for rec in exp["samples"]:
        t, pts = rec["index"], np.array(rec["points"])
        s2 = rec["sigma2_f80"]
        m80, v80 = np.array(rec["mean_f80"]), np.array(rec["mse_f80"])
        tm, tv = pred_tolerance(np.array(rec["mean_f64"]), np.array(rec["mse_f64"]), m80, v80,
                                np.array(rec["mean_lapack"]), np.array(rec["mse_lapack"]), sd, s2)
        em = np.abs(mean[t, pts] - m80) / np.maximum(np.abs(m80), sd)
        ev = np.abs(mse[t, pts] - v80) / np.maximum(np.abs(v80), s2)
        assert np.all(em <= tm), (t, em, tm)
        assert np.all(ev <= tv), (t, ev, tv)
