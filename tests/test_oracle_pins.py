"""Pins for the CPU oracle: closed forms, brute force and invariants.

Each test ties the oracle to something other than itself (high-precision
closed forms, eigenvalues, LAPACK, exact special cases, the paper's printed
tables) so that a dropped term, a wrong sign, a wrong index or a transposed
operand in the oracle fails at least one of them.
"""
import math

import mpmath
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from paper_1203_1269_amd import inputs

mpmath.mp.dps = 50


def mp_rho(xi, xj, theta, p):
    """exp(-sum_k theta_k |x_ik - x_jk|^p) at 50 digits (eq. 2, sum form)."""
    s = mpmath.mpf(0)
    for a, b, t in zip(xi, xj, theta):
        diff = abs(mpmath.mpf(a) - mpmath.mpf(b))
        s += mpmath.mpf(t) * (diff ** mpmath.mpf(p) if diff != 0 else 0)
    return mpmath.exp(-s)


def mp_R(X, theta, p, delta):
    n = X.shape[0]
    R = mpmath.matrix(n, n)
    for i in range(n):
        for j in range(n):
            R[i, j] = (1 + mpmath.mpf(delta)) if i == j else mp_rho(X[i], X[j], theta, p)
    return R


def mp_profile(X, y, theta, p, delta):
    """eq. (3)-(4) by 50-digit linear algebra: returns logdet, mu, sigma2, nll."""
    n = X.shape[0]
    R = mp_R(X, theta, p, delta)
    one = mpmath.matrix([1] * n)
    Y = mpmath.matrix([mpmath.mpf(v) for v in y])
    Ri1 = mpmath.lu_solve(R, one)
    RiY = mpmath.lu_solve(R, Y)
    mu = (one.T * RiY)[0] / (one.T * Ri1)[0]
    r = Y - one * mu
    Q = (r.T * mpmath.lu_solve(R, r))[0]
    logdet = mpmath.log(mpmath.det(R))
    s2 = Q / n
    return float(logdet), float(mu), float(s2), float(logdet + n * mpmath.log(s2))


def one(X, y, theta, p, delta, extended=False):
    r = oracle.nll_batch(X, y, np.atleast_2d(theta), p, delta, extended=extended)
    return r


# --------------------------------------------------------------------------
# Correlation matrix, eq. (2) plus nugget

def test_corr_entries_match_50_digit_sum_form():
    rng = np.random.default_rng(10)
    X = rng.random((6, 3))
    th = np.array([0.7, 3.0, 11.0])
    for p in (2.0, 1.95, 1.0, 0.5):
        R = oracle.corr(X, th, p, 1e-3)
        Rm = mp_R(X, th, p, 1e-3)
        for i in range(6):
            for j in range(6):
                assert abs(R[i, j] - float(Rm[i, j])) <= 4e-16 * max(1.0, abs(float(Rm[i, j])))


def test_corr_structure():
    rng = np.random.default_rng(11)
    X = rng.random((40, 4))
    th = np.array([0.3, 1.0, 5.0, 20.0])
    R = oracle.corr(X, th, 1.95, 1e-6)
    assert np.array_equal(R, R.T)
    assert np.all(np.diag(R) == 1 + 1e-6)
    off = R[~np.eye(40, dtype=bool)]
    assert np.all(off > 0) and np.all(off <= 1)


def test_corr_invariances():
    rng = np.random.default_rng(12)
    X = rng.random((30, 3))
    th = np.array([2.0, 0.5, 7.0])
    p = 1.5
    R = oracle.corr(X, th, p, 0.0)
    # translation and reflection of the inputs
    assert np.allclose(oracle.corr(X + 0.25, th, p, 0.0), R, rtol=1e-13, atol=0)
    assert np.allclose(oracle.corr(1.0 - X, th, p, 0.0), R, rtol=1e-13, atol=0)
    # point permutation permutes rows and columns
    perm = rng.permutation(30)
    assert np.allclose(oracle.corr(X[perm], th, p, 0.0), R[np.ix_(perm, perm)], rtol=0, atol=0)
    # theta-x rescaling: x_k -> s x_k, theta_k -> theta_k / s^p
    s = np.array([2.0, 0.5, 3.0])
    assert np.allclose(oracle.corr(X * s, th / s ** p, p, 0.0), R, rtol=1e-12, atol=0)
    # dimension order does not matter (product over k)
    q = np.array([2, 0, 1])
    assert np.allclose(oracle.corr(X[:, q], th[q], p, 0.0), R, rtol=1e-14, atol=0)


# --------------------------------------------------------------------------
# Closed forms at n = 2 and n = 3

@pytest.mark.parametrize("p", [2.0, 1.95, 1.0])
@pytest.mark.parametrize("delta", [0.0, 1e-6, 0.1])
def test_n2_closed_form(p, delta):
    rng = np.random.default_rng(20)
    X = rng.random((2, 3))
    y = np.array([0.3, -1.2])
    th = np.array([0.4, 1.5, 3.0])
    rho = float(mp_rho(X[0], X[1], th, p))
    e = 1 + delta
    r = one(X, y, th, p, delta)
    logdet = math.log(e * e - rho * rho)
    mu = (y[0] + y[1]) / 2
    s2 = (y[0] - y[1]) ** 2 / (4 * (e - rho))
    assert r.info[0] == 0
    assert abs(r.logdet[0] - logdet) <= 1e-13 * max(1, abs(logdet))
    assert abs(r.mu[0] - mu) <= 1e-14
    assert abs(r.sigma2[0] - s2) <= 1e-13 * s2
    assert abs(r.nll[0] - (logdet + 2 * math.log(s2))) <= 1e-12 * max(1, abs(r.nll[0]))
    # the literal eq. (4) value differs from nll by n ln n
    assert abs(r.nll_paper[0] - r.nll[0] - 2 * math.log(2)) <= 1e-12 * max(1, abs(r.nll[0]))


def test_n2_det_is_one_minus_r12_squared():
    X = np.array([[0.1, 0.2], [0.5, 0.9]])
    th = np.array([1.0, 2.0])
    rho = float(mp_rho(X[0], X[1], th, 2.0))
    r = one(X, np.array([1.0, 2.0]), th, 2.0, 0.0)
    assert abs(math.exp(r.logdet[0]) - (1 - rho * rho)) <= 1e-14


def test_n3_closed_form_det():
    rng = np.random.default_rng(21)
    for trial in range(5):
        X = rng.random((3, 2))
        th = np.exp(rng.uniform(-1, 2, 2))
        delta = [0.0, 1e-4, 0.5][trial % 3]
        e = 1 + delta
        a = float(mp_rho(X[0], X[1], th, 1.95))
        b = float(mp_rho(X[0], X[2], th, 1.95))
        c = float(mp_rho(X[1], X[2], th, 1.95))
        det = e ** 3 + 2 * a * b * c - e * (a * a + b * b + c * c)
        r = one(X, rng.standard_normal(3), th, 1.95, delta)
        assert abs(r.logdet[0] - math.log(det)) <= 1e-12 * max(1, abs(math.log(det)))


@pytest.mark.parametrize("n", [3, 5, 8])
def test_tiny_n_against_50_digit_linear_algebra(n):
    rng = np.random.default_rng(30 + n)
    X = rng.random((n, 2))
    y = rng.standard_normal(n)
    th = np.array([0.8, 2.5])
    ref = mp_profile(X, y, th, 1.95, 1e-3)
    r = one(X, y, th, 1.95, 1e-3)
    got = (r.logdet[0], r.mu[0], r.sigma2[0], r.nll[0])
    for g, e in zip(got, ref):
        assert abs(g - e) <= 1e-11 * max(1.0, abs(e))


@pytest.mark.parametrize("n", [4, 7, 12])
def test_logdet_equals_sum_log_eigenvalues(n):
    rng = np.random.default_rng(40 + n)
    X = rng.random((n, 3))
    th = np.exp(rng.uniform(-1, 2, 3))
    R = oracle.corr(X, th, 2.0, 1e-2)
    ev = np.linalg.eigvalsh(R)
    r = one(X, rng.standard_normal(n), th, 2.0, 1e-2)
    assert abs(r.logdet[0] - np.sum(np.log(ev))) <= 1e-11 * max(1, abs(r.logdet[0]))


# --------------------------------------------------------------------------
# Special cases with closed forms at any n

def kms(n, theta, h, perm=None, y=None):
    """d=1, p=1, delta=0, x_i = i h: R_ij = rho^|i-j| with rho = exp(-theta h)."""
    x = np.arange(n) * h
    rho = math.exp(-theta * h)
    logdet = (n - 1) * math.log(1 - rho * rho)
    mu = ((y[0] + y[-1]) + (1 - rho) * y[1:-1].sum()) / (n - (n - 2) * rho)
    r = y - mu
    Q = r[0] ** 2 + np.sum((r[1:] - rho * r[:-1]) ** 2) / (1 - rho * rho)
    return x, logdet, mu, Q


@pytest.mark.parametrize("n,theta", [(50, 8.0), (257, 30.0), (600, 100.0)])
def test_kms_closed_form_any_n(n, theta):
    rng = np.random.default_rng(50 + n)
    y = rng.standard_normal(n)
    h = 1.0 / 1024
    x, logdet, mu, Q = kms(n, theta, h, y=y)
    perm = rng.permutation(n)   # order of points does not matter
    r = one(x[perm, None], y[perm], [theta], 1.0, 0.0)
    assert r.info[0] == 0
    assert abs(r.logdet[0] - logdet) <= 1e-10 * abs(logdet)
    assert abs(r.mu[0] - mu) <= 1e-10 * max(1, abs(mu))
    assert abs(r.Q[0] - Q) <= 1e-10 * Q
    assert abs(r.sigma2[0] - Q / n) <= 1e-10 * Q / n


def test_kronecker_grid_logdet():
    """Separable product correlation on a full grid: R = R_A (x) R_B, so
    log|R| = n_B log|R_A| + n_A log|R_B|, each factor a KMS matrix."""
    nA, nB = 9, 13
    hA, hB = 1.0 / 16, 1.0 / 32
    thA, thB = 5.0, 7.0
    a = np.arange(nA) * hA
    b = np.arange(nB) * hB
    X = np.array([[ai, bj] for ai in a for bj in b])
    rhoA, rhoB = math.exp(-thA * hA), math.exp(-thB * hB)
    ldA = (nA - 1) * math.log(1 - rhoA ** 2)
    ldB = (nB - 1) * math.log(1 - rhoB ** 2)
    r = one(X, np.arange(nA * nB, dtype=float), [thA, thB], 1.0, 0.0)
    assert abs(r.logdet[0] - (nB * ldA + nA * ldB)) <= 1e-11 * abs(nB * ldA + nA * ldB)


def test_theta_to_infinity_limit():
    rng = np.random.default_rng(60)
    n = 80
    X = inputs.lhs_design(n, 2, rng)
    y = rng.standard_normal(n)
    delta = 1e-6
    r = one(X, y, [1e9, 1e9], 2.0, delta)
    assert r.logdet[0] == pytest.approx(n * math.log1p(delta), rel=1e-12)
    assert r.mu[0] == pytest.approx(y.mean(), rel=1e-12, abs=1e-14)
    assert r.sigma2[0] == pytest.approx(np.sum((y - y.mean()) ** 2) / (n * (1 + delta)), rel=1e-12)


def test_constant_y_gives_mu_equal_c():
    rng = np.random.default_rng(61)
    X = rng.random((60, 3))
    c = 3.25
    r = one(X, np.full(60, c), [1.0, 2.0, 3.0], 1.95, 1e-6)
    assert abs(r.mu[0] - c) <= 1e-10 * c
    assert r.sigma2[0] <= 1e-20 * c * c
    assert r.info[0] in (0, -1)


def test_hadamard_bound():
    w = inputs.small_2d(B=16)
    r = oracle.nll_batch(w.X, w.y, w.theta, w.p, w.delta)
    assert np.all(r.logdet <= w.n * math.log1p(w.delta) + 1e-9)


# --------------------------------------------------------------------------
# Independent FP64 implementation (LAPACK via SciPy) on random cases

@pytest.mark.parametrize("seed", range(4))
def test_against_lapack(seed):
    rng = np.random.default_rng(70 + seed)
    n, d = 120, 3
    X = inputs.lhs_design(n, d, rng)
    y = inputs.sine_response(X, rng)
    th = inputs.log_uniform_theta(3, d, 0.5, 20, rng)
    r = oracle.nll_batch(X, y, th, 1.95, 1e-4)
    for t in range(3):
        R = oracle.corr(X, th[t], 1.95, 1e-4)
        c = sla.cho_factor(R, lower=True)
        logdet = 2 * np.sum(np.log(np.diag(c[0])))
        Ri1 = sla.cho_solve(c, np.ones(n))
        Riy = sla.cho_solve(c, y)
        mu = Ri1 @ y / Ri1.sum()
        Q = (y - mu) @ sla.cho_solve(c, y - mu)
        assert abs(r.logdet[t] - logdet) <= 1e-10 * max(1, abs(logdet))
        assert abs(r.mu[t] - mu) <= 1e-10 * max(1, abs(mu))
        assert abs(r.Q[t] - Q) <= 1e-9 * Q
        assert abs(r.ab[t] - Riy.sum()) <= 1e-9 * max(1, abs(Riy.sum()))


# --------------------------------------------------------------------------
# Invariances of the profile likelihood

def test_profile_invariances():
    rng = np.random.default_rng(80)
    n, d = 90, 2
    X = inputs.lhs_design(n, d, rng)
    y = inputs.sine_response(X, rng)
    th = np.array([[3.0, 9.0]])
    base = oracle.nll_batch(X, y, th, 1.95, 1e-5)
    perm = rng.permutation(n)
    pr = oracle.nll_batch(X[perm], y[perm], th, 1.95, 1e-5)
    assert pr.nll[0] == pytest.approx(base.nll[0], rel=1e-11)
    # y shift: mu shifts, sigma2 unchanged
    sh = oracle.nll_batch(X, y + 5.0, th, 1.95, 1e-5)
    assert sh.mu[0] == pytest.approx(base.mu[0] + 5.0, rel=1e-11)
    assert sh.sigma2[0] == pytest.approx(base.sigma2[0], rel=1e-9)
    # y scale: sigma2 * a^2, nll + 2 n ln|a|
    a = -3.0
    sc = oracle.nll_batch(X, a * y, th, 1.95, 1e-5)
    assert sc.sigma2[0] == pytest.approx(a * a * base.sigma2[0], rel=1e-11)
    assert sc.nll[0] == pytest.approx(base.nll[0] + 2 * n * math.log(abs(a)), rel=1e-11)
    assert sc.mu[0] == pytest.approx(a * base.mu[0], rel=1e-11)


# --------------------------------------------------------------------------
# Failure semantics

def test_singular_matrix_sets_info():
    # theta = 0 and no nugget: R is all ones, the second pivot is exactly 0
    X = np.random.default_rng(90).random((10, 2))
    r = one(X, np.arange(10.0), [0.0, 0.0], 2.0, 0.0)
    assert r.info[0] == 2
    assert np.isnan(r.nll[0]) and np.isnan(r.logdet[0])
    # duplicate points, no nugget
    X2 = np.array([[0.3, 0.4], [0.3, 0.4]])
    r2 = one(X2, np.array([1.0, 2.0]), [1.0, 1.0], 2.0, 0.0)
    assert r2.info[0] == 2


def test_invalid_theta_sets_info():
    X = np.random.default_rng(91).random((10, 2))
    r = oracle.nll_batch(X, np.arange(10.0), np.array([[1.0, -1.0], [np.nan, 1.0], [1.0, 1.0]]), 2.0, 1e-6)
    assert list(r.info) == [-3, -3, 0]
    assert np.isnan(r.nll[0]) and np.isnan(r.nll[1]) and np.isfinite(r.nll[2])


# --------------------------------------------------------------------------
# Gradient against central finite differences of the 80-bit oracle

def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(100)
    n, d = 70, 3
    X = inputs.lhs_design(n, d, rng)
    y = inputs.sine_response(X, rng)
    th = inputs.log_uniform_theta(3, d, 0.5, 10, rng)
    p, delta = 2.0, 1e-6
    res, g = oracle.grad_batch(X, y, th, p, delta)
    res80, g80 = oracle.grad_batch(X, y, th, p, delta, extended=True)
    for t in range(3):
        for k in range(d):
            h = 1e-6 * th[t, k]
            tp = th[t].copy(); tp[k] += h
            tm = th[t].copy(); tm[k] -= h
            fp = oracle.nll_batch(X, y, tp[None], p, delta, extended=True).nll[0]
            fm = oracle.nll_batch(X, y, tm[None], p, delta, extended=True).nll[0]
            fd = (fp - fm) / (2 * h)
            assert abs(g[t, k] - fd) <= 1e-5 * max(1.0, abs(fd)), (t, k, g[t, k], fd)
            assert abs(g[t, k] - g80[t, k]) <= 1e-7 * max(1.0, abs(g80[t, k]))


def test_gradient_vanishes_at_large_theta():
    rng = np.random.default_rng(101)
    X = rng.random((30, 2))
    _, g = oracle.grad_batch(X, rng.standard_normal(30), np.array([[1e9, 1e9]]), 2.0, 1e-6)
    assert np.all(np.abs(g) < 1e-100)


# --------------------------------------------------------------------------
# The paper's printed tables: which constant eq. (4) carries

def test_paper_tables_fix_the_eq4_convention():
    """Under the literal eq. (4), log|R| = nll_paper - n ln(n sigma2) must be
    <= 0 for a correlation matrix without nugget (Hadamard).  The tables in
    Sec. 4 satisfy this for every CPU row, while the n ln(sigma2) convention
    would make several rows positive.  The oracle's nll_paper is therefore
    the tables' convention and nll = nll_paper - n ln n."""
    rows = []
    path = __file__.replace("test_oracle_pins.py", "golden/paper_tables.txt")
    for line in open(path):
        line = line.split("#")[0].strip()
        if line:
            tag, n, nll, mu, s2 = line.split()
            rows.append((tag, int(n), float(nll), float(mu), float(s2)))
    assert len(rows) == 20
    literal_ok, ns_positive = 0, 0
    for tag, n, nll, mu, s2 in rows:
        if tag.endswith("cpu"):
            assert nll - n * math.log(n * s2) <= 0.0, (tag, n)
            literal_ok += 1
            if nll - n * math.log(s2) > 0:
                ns_positive += 1
    assert literal_ok == 10 and ns_positive >= 5
    # and the oracle's two conventions differ by exactly n ln n
    w = inputs.small_2d(B=4)
    r = oracle.nll_batch(w.X, w.y, w.theta, w.p, w.delta)
    assert np.allclose(r.nll_paper - r.nll, w.n * math.log(w.n), rtol=1e-12)


# ---------------------------------------------------------------------------
# Predictions (Sec. 3: one R, one factorisation, back-solves per test point;
# Sec. 4: SSPE on a test set).  The predictor is the best linear unbiased one
# of the model of Sec. 2; its pins come from independent routes.

def _pred_case(seed=21, n=60, d=3, delta=1e-6):
    rng = np.random.default_rng(seed)
    X = inputs.lhs_design(n, d, rng)
    y = inputs.sine_response(X, rng)
    th = np.array([2.0, 1.0, 4.0])[:d]
    Xs = rng.uniform(size=(25, d))
    return X, y, th, delta, Xs


def test_prediction_interpolates_without_nugget():
    """delta = 0: the predictor passes through the data and its mean squared
    error vanishes there."""
    X, y, th, _, _ = _pred_case()
    mean, mse, fit = oracle.predict(X, y, th, 2.0, 0.0, X[:12])
    assert fit.info[0] == 0
    np.testing.assert_allclose(mean, y[:12], rtol=0, atol=1e-8 * np.std(y))
    assert np.all(np.abs(mse) <= 1e-9 * fit.sigma2[0])


def test_prediction_matches_ordinary_kriging_system():
    """Independent route: the weights of ordinary kriging from the bordered
    system [[R, 1], [1', 0]] [lam; m] = [r; 1] (dense solve on the oracle's
    R) give mean = lam' y and mse = sigma2 (1 - lam' r - m)."""
    X, y, th, delta, Xs = _pred_case()
    n = X.shape[0]
    R = oracle.corr(X, th, 2.0, delta)
    K = np.zeros((n + 1, n + 1))
    K[:n, :n] = R
    K[:n, n] = K[n, :n] = 1.0
    mean, mse, fit = oracle.predict(X, y, th, 2.0, delta, Xs)
    s2 = fit.sigma2[0]
    for j in range(Xs.shape[0]):
        r = np.exp(-np.sum(th * np.abs(Xs[j] - X) ** 2.0, axis=1))
        sol = np.linalg.solve(K, np.append(r, 1.0))
        lam, m = sol[:n], sol[n]
        assert abs(mean[j] - lam @ y) <= 1e-9 * np.std(y)
        assert abs(mse[j] - s2 * (1 - lam @ r - m)) <= 1e-9 * s2


def test_prediction_far_from_the_data():
    """r -> 0 far from every design point: mean -> mu, mse -> sigma2 (1 +
    1 / (1' R^-1 1)), with 1' R^-1 1 from a dense solve."""
    X, y, th, delta, _ = _pred_case()
    mean, mse, fit = oracle.predict(X, y, th, 2.0, delta, np.full((2, 3), 50.0))
    R = oracle.corr(X, th, 2.0, delta)
    oRo = np.sum(np.linalg.solve(R, np.ones(X.shape[0])))
    np.testing.assert_allclose(mean, fit.mu[0], rtol=1e-12)
    np.testing.assert_allclose(mse, fit.sigma2[0] * (1 + 1 / oRo), rtol=1e-9)


def test_prediction_invariances():
    """y -> a y + c moves the mean the same way and scales the mse by a^2; a
    permutation of the design points changes nothing."""
    X, y, th, delta, Xs = _pred_case()
    m0, v0, _ = oracle.predict(X, y, th, 2.0, delta, Xs)
    m1, v1, _ = oracle.predict(X, 3.0 * y - 2.0, th, 2.0, delta, Xs)
    np.testing.assert_allclose(m1, 3.0 * m0 - 2.0, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(v1, 9.0 * v0, rtol=1e-8, atol=1e-12)
    perm = np.random.default_rng(5).permutation(X.shape[0])
    m2, v2, _ = oracle.predict(X[perm], y[perm], th, 2.0, delta, Xs)
    np.testing.assert_allclose(m2, m0, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(v2, v0, rtol=1e-8, atol=1e-14)


def test_prediction_extended_agrees():
    X, y, th, delta, Xs = _pred_case()
    m64, v64, _ = oracle.predict(X, y, th, 1.95, delta, Xs)
    m80, v80, _ = oracle.predict(X, y, th, 1.95, delta, Xs, extended=True)
    np.testing.assert_allclose(m64, m80, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(v64, v80, rtol=1e-7, atol=1e-14)


# --------------------------------------------------------------------------
# Matern families (the alternative correlation Sec. 2 names), pinned by the
# Bessel-function definition of the Matern correlation (SciPy's K_nu), which
# shares nothing with the oracle's closed forms

MATERN = {"matern32": 1.5, "matern52": 2.5}


def _matern_bessel(h, nu):
    """2^(1-nu) / Gamma(nu) (sqrt(2 nu) h)^nu K_nu(sqrt(2 nu) h), 1 at h = 0."""
    from scipy.special import gamma, kv
    h = np.asarray(h, dtype=np.float64)
    z = np.sqrt(2 * nu) * h
    with np.errstate(invalid="ignore"):
        v = 2 ** (1 - nu) / gamma(nu) * z ** nu * kv(nu, z)
    return np.where(h == 0, 1.0, v)


def _matern_R(X, theta, nu, delta):
    diff = np.abs(X[:, None, :] - X[None, :, :])
    R = np.prod(_matern_bessel(theta[None, None, :] * diff, nu), axis=2)
    return R + delta * np.eye(X.shape[0])


@pytest.mark.parametrize("family", sorted(MATERN))
@pytest.mark.parametrize("extended", [False, True])
def test_matern_entries_match_the_bessel_definition(family, extended):
    rng = np.random.default_rng(300)
    X = rng.random((9, 3))
    th = np.array([0.7, 3.0, 12.0])
    R = oracle.corr(X, th, 2.0, 1e-6, extended=extended, family=family)
    ref = _matern_R(X, th, MATERN[family], 1e-6)
    np.testing.assert_allclose(R, ref, rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("family", sorted(MATERN))
@pytest.mark.parametrize("delta", [0.0, 1e-6, 0.1])
def test_matern_n2_closed_form(family, delta):
    X = np.array([[0.1, 0.7], [0.45, 0.2]])
    y = np.array([1.3, -0.4])
    th = np.array([2.0, 0.5])
    rho = float(np.prod(_matern_bessel(th * np.abs(X[0] - X[1]), MATERN[family])))
    r = oracle.nll_batch(X, y, th[None], 9.9, delta, extended=True, family=family)
    e = 1 + delta
    assert abs(r.logdet[0] - np.log(e * e - rho * rho)) <= 1e-13
    assert abs(r.mu[0] - 0.5 * (y[0] + y[1])) <= 1e-14
    s2 = (y[0] - y[1]) ** 2 / (4 * (e - rho))
    assert abs(r.sigma2[0] - s2) <= 1e-13 * s2


@pytest.mark.parametrize("family", sorted(MATERN))
def test_matern_likelihood_against_dense_linear_algebra(family):
    """n = 40: log|R| = sum ln eig(R), mu and sigma2 from dense solves, all on
    the Bessel-defined R."""
    rng = np.random.default_rng(301)
    n, d = 40, 3
    X = inputs.lhs_design(n, d, rng)
    y = inputs.sine_response(X, rng)
    th = np.array([1.5, 4.0, 0.8])
    R = _matern_R(X, th, MATERN[family], 1e-6)
    ld = np.sum(np.log(np.linalg.eigvalsh(R)))
    one = np.ones(n)
    mu = (one @ np.linalg.solve(R, y)) / (one @ np.linalg.solve(R, one))
    s2 = (y - mu) @ np.linalg.solve(R, y - mu) / n
    r = oracle.nll_batch(X, y, th[None], 2.0, 1e-6, family=family)
    assert abs(r.logdet[0] - ld) <= 1e-9 * max(1.0, abs(ld))
    assert abs(r.mu[0] - mu) <= 1e-9 * np.std(y)
    assert abs(r.sigma2[0] - s2) <= 1e-9 * s2


@pytest.mark.parametrize("family", sorted(MATERN))
def test_matern_gradient_matches_finite_differences(family):
    rng = np.random.default_rng(302)
    n, d = 60, 3
    X = inputs.lhs_design(n, d, rng)
    y = inputs.sine_response(X, rng)
    th = inputs.log_uniform_theta(2, d, 0.5, 10, rng)
    _, g = oracle.grad_batch(X, y, th, 2.0, 1e-6, family=family)
    for t in range(2):
        for k in range(d):
            h = 1e-6 * th[t, k]
            tp = th[t].copy(); tp[k] += h
            tm = th[t].copy(); tm[k] -= h
            fp = oracle.nll_batch(X, y, tp[None], 2.0, 1e-6, extended=True, family=family).nll[0]
            fm = oracle.nll_batch(X, y, tm[None], 2.0, 1e-6, extended=True, family=family).nll[0]
            fd = (fp - fm) / (2 * h)
            assert abs(g[t, k] - fd) <= 1e-5 * max(1.0, abs(fd)), (t, k, g[t, k], fd)


@pytest.mark.parametrize("family", sorted(MATERN))
def test_matern_prediction_interpolates_and_limits(family):
    """delta = 0: the predictor returns y at design points with zero mse; far
    from the data the mean tends to mu; theta -> infinity gives R = I."""
    rng = np.random.default_rng(303)
    n, d = 30, 2
    X = inputs.lhs_design(n, d, rng)
    y = inputs.sine_response(X, rng)
    th = np.array([3.0, 5.0])
    mean, mse, fit = oracle.predict(X, y, th, 2.0, 0.0, X[[2, 17]], family=family)
    np.testing.assert_allclose(mean, y[[2, 17]], rtol=0, atol=1e-9)
    assert np.all(np.abs(mse) <= 1e-9 * fit.sigma2[0])
    far, _, fit2 = oracle.predict(X, y, th, 2.0, 1e-6, np.array([[1e3, -1e3]]), family=family)
    assert abs(far[0] - fit2.mu[0]) <= 1e-12
    r = oracle.nll_batch(X, y, np.array([[1e9, 1e9]]), 2.0, 1e-6, family=family)
    assert abs(r.logdet[0] - n * np.log1p(1e-6)) <= 1e-12


def test_family_argument_checked():
    X = np.random.default_rng(0).random((5, 2))
    with pytest.raises(ValueError):
        oracle.corr(X, np.ones(2), 2.0, 0.0, family="gauss")
    # the power exponent is checked only for the power-exponential family
    with pytest.raises(ValueError):
        oracle.corr(X, np.ones(2), 2.5, 0.0)
    oracle.corr(X, np.ones(2), 2.5, 0.0, family="matern52")
