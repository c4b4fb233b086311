"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bar: every output within max(1e-10, 10 x the FP64 rounding spread for that
theta) of the 80-bit oracle, the spread being the larger error of two
independent FP64 codes (the oracle's FP64 build and LAPACK); integer status
(info) bit-exact.  Sizes span several 64/128/256 tiles with ragged tails, plus the
full-size workload on sampled thetas (expected values written by
tests/golden/make_expected.py, which calls only the oracle).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_1203_1269_amd import inputs
from parity_util import compare, lapack_fp64, scales, to_host, tolerances

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


def run_gpu(gp, X, y, theta, p, delta):
    ds = gp.Dataset(X, y, p, delta)
    res = gp.nll_batch(ds, theta)
    torch.cuda.synchronize()
    return to_host(res)


def check_against_oracle(gp, X, y, theta, p, delta, label):
    print(f"[parity] {label}: n={X.shape[0]} d={X.shape[1]} B={theta.shape[0]} p={p} delta={delta}",
          flush=True)
    got = run_gpu(gp, X, y, theta, p, delta)
    r64 = oracle.nll_batch(X, y, theta, p, delta)
    r80 = oracle.nll_batch(X, y, theta, p, delta, extended=True)
    tol = tolerances(r64, r80, y, lapack_fp64(X, y, theta, p, delta))
    return compare(got, r80, tol, y, label)


# ---------------------------------------------------------------------------
# Correlation build, entrywise

@pytest.mark.parametrize("n,d,p", [(200, 2, 2.0), (300, 5, 1.95), (130, 3, 1.0), (77, 12, 1.5),
                                   (64, 20, 0.7)])
def test_corr_build_entrywise(gp, n, d, p):
    rng = np.random.default_rng(1000 + n)
    X = inputs.lhs_design(n, d, rng)
    th = inputs.log_uniform_theta(3, d, 0.05, 20, rng)
    delta = 1e-6
    ds = gp.Dataset(X, np.zeros(n), p, delta)
    R, info = gp.corr_build(ds, th)
    torch.cuda.synchronize()
    R = R.cpu().numpy()
    assert np.all(info.cpu().numpy() == 0)
    np_ = gp.pad64(n)
    for b in range(3):
        G = R[b].T                       # column-major storage -> row-major view
        ref = oracle.corr(X, th[b], p, delta, extended=True)
        low = np.tril(np.ones((n, n), dtype=bool))
        err = np.abs(G[:n, :n] - ref)[low]
        # ulp bar from the arithmetic: the exponent s = sum_k theta_k |dx_k|^p
        # carries at most (d + 4) u s of rounding (pow within 2 ulp, the
        # product and d - 1 additions of positive terms within half an ulp
        # each, with slack), and exp(-s) adds 2 ulp; relative to R_ij that
        # is ((d + 4) s + 2) u, u = 2^-53 (entries below 1e-300: absolute)
        r = ref[low]
        s_ = -np.log(np.maximum(r, 1e-300))
        bar = ((d + 4) * s_ + 2) * 2.0 ** -53 * r + 1e-300
        assert np.all(err <= bar), (err / np.maximum(bar, 1e-300)).max()
        print(f"corr n={n} d={d} p={p}: worst error / ulp bar {(err / bar).max():.3f}")
        assert np.all(np.diag(G)[:n] == 1.0 + delta)
        # padding is the identity
        assert np.all(G[n:, :n] == 0.0)
        pad = G[n:np_, n:np_]
        assert np.array_equal(np.tril(pad), np.eye(np_ - n))


def test_corr_build_flags_invalid_theta(gp):
    X = np.random.default_rng(5).random((40, 2))
    ds = gp.Dataset(X, np.zeros(40), 2.0, 0.0)
    th = np.array([[1.0, 2.0], [-1.0, 2.0], [np.inf, 1.0], [0.0, 0.0]])
    _, info = gp.corr_build(ds, th)
    assert list(info.cpu().numpy()) == [0, -3, -3, 0]


# ---------------------------------------------------------------------------
# Blocked Cholesky and log-determinant on oracle-built matrices

@pytest.mark.parametrize("n", [64, 100, 257, 600, 1000])
def test_cholesky_factor_entrywise(gp, n):
    print(f"[parity] cholesky n={n}", flush=True)
    rng = np.random.default_rng(2000 + n)
    X = inputs.lhs_design(n, 3, rng)
    ths = inputs.log_uniform_theta(2, 3, 5.0, 40.0, rng)
    delta = 1e-3
    lda = gp.pad64(n) + 64
    A = torch.zeros((2, lda, lda), dtype=torch.float64)
    refs = []
    for b in range(2):
        R = oracle.corr(X, ths[b], 1.95, delta)
        A[b, :n, :n] = torch.from_numpy(R)      # symmetric: row/column-major agree
        A[b, n:, :] = float("nan")              # padding must be overwritten
        A[b, :, n:] = float("nan")
        refs.append(oracle.cholesky(R, extended=True))
    A = A.cuda()
    info, logdet = gp.cholesky_batch(A, n)
    torch.cuda.synchronize()
    A = A.cpu().numpy()
    info = info.cpu().numpy()
    logdet = logdet.cpu().numpy()
    for b in range(2):
        Lref, iref = refs[b]
        assert info[b] == iref == 0
        L = np.tril(A[b].T[:n, :n])
        colmax = np.max(np.abs(Lref), axis=0)
        err = np.max(np.abs(L - Lref) / colmax[None, :])
        assert err <= 1e-12, err
        ld_ref = 2 * np.sum(np.log(np.diag(Lref)))
        assert abs(logdet[b] - ld_ref) <= 1e-12 * max(1.0, abs(ld_ref))
        # the strict upper triangle of every diagonal 64-tile is zero
        np_ = gp.pad64(n)
        for t in range(0, np_, 64):
            blk = A[b].T[t:t + 64, t:t + 64]
            assert np.all(np.triu(blk, 1) == 0.0)


def test_cholesky_reports_first_bad_pivot(gp):
    # an all-ones matrix: the second pivot is exactly zero
    n = 150
    lda = gp.pad64(n)
    A = torch.ones((1, lda, lda), dtype=torch.float64, device="cuda")
    info, _ = gp.cholesky_batch(A, n)
    assert int(info.cpu()[0]) == 2
    # a pivot failing in a later tile (indefinite at row 131)
    R = np.eye(n)
    R[130, 130] = -1.0
    A = torch.zeros((1, lda, lda), dtype=torch.float64)
    A[0, :n, :n] = torch.from_numpy(R)
    A = A.cuda()
    info, _ = gp.cholesky_batch(A, n)
    assert int(info.cpu()[0]) == 131


# ---------------------------------------------------------------------------
# End to end

def test_small_2d_workload(gp):
    """n=200, d=2, p=2, nugget 1e-8, 64 thetas in [0.1, 10]^2."""
    w = inputs.small_2d()
    worst = check_against_oracle(gp, w.X, w.y, w.theta, w.p, w.delta, "fp64_n200_d2")
    print("worst rel err", worst)


@pytest.mark.parametrize("n,d,p,delta,B", [
    (2, 1, 2.0, 1e-6, 3),        # minimum n
    (63, 2, 1.95, 1e-6, 4),
    (64, 3, 2.0, 1e-6, 4),       # exactly one tile
    (65, 3, 2.0, 1e-6, 4),       # one tile + 1
    (255, 4, 1.5, 1e-6, 3),
    (257, 4, 1.95, 1e-6, 3),     # one outer panel + 1
    (777, 6, 1.95, 1e-6, 5),     # several panels, ragged tail
    (1500, 8, 1.95, 1e-6, 3),
    (300, 12, 2.0, 1e-6, 3),     # d > 8
    (130, 20, 1.0, 1e-4, 2),     # d > 16
])
def test_end_to_end_shapes(gp, n, d, p, delta, B):
    rng = np.random.default_rng(3000 + n + d)
    X = inputs.lhs_design(n, d, rng)
    y = inputs.sine_response(X, rng)
    th = inputs.log_uniform_theta(B, d, 0.05, 20, rng)
    check_against_oracle(gp, X, y, th, p, delta, f"n{n}_d{d}")


def test_edge_cases(gp):
    rng = np.random.default_rng(4000)
    n = 90
    X = rng.random((n, 2))
    y = rng.standard_normal(n)
    th = np.array([[60.0, 80.0], [-1.0, 1.0], [np.nan, 1.0], [0.0, 0.0], [1e9, 1e9], [1.0, 2.0]])
    got = run_gpu(gp, X, y, th, 2.0, 0.0)
    r80 = oracle.nll_batch(X, y, th, 2.0, 0.0, extended=True)
    assert list(got["info"][:5]) == list(r80.info[:5]) == [0, -3, -3, 2, 0]
    # numerically singular without a nugget: which pivot fails first depends on
    # rounding, so only the failure itself is compared
    assert r80.info[5] > 0 and got["info"][5] > 0
    for k in ("logdet", "mu", "sigma2", "nll"):
        assert np.all(np.isnan(got[k][1:4])) and np.isnan(got[k][5])
    assert abs(got["nll"][0] - r80.nll[0]) <= 1e-9 * abs(r80.nll[0])
    # theta -> infinity: R = I
    assert got["logdet"][4] == 0.0
    assert abs(got["mu"][4] - y.mean()) <= 1e-12
    assert abs(got["sigma2"][4] - np.mean((y - y.mean()) ** 2)) <= 1e-12 * np.var(y)
    # constant response: mu = c, sigma2 ~ 0
    c = 2.5
    got = run_gpu(gp, X, np.full(n, c), np.array([[3.0, 4.0]]), 2.0, 1e-6)
    assert abs(got["mu"][0] - c) <= 1e-10 * c
    assert got["sigma2"][0] <= 1e-20 * c * c
    assert got["info"][0] in (0, -1)


def test_single_theta_entry_point(gp):
    w = inputs.small_2d(B=4)
    ds = gp.Dataset(w.X, w.y, w.p, w.delta)
    single = to_host(gp.nll(ds, w.theta[2]))
    batch = to_host(gp.nll_batch(ds, w.theta))
    for k in ("logdet", "mu", "sigma2", "nll"):
        assert single[k][0] == batch[k][2]


def test_batch_independence_and_determinism(gp):
    """Each theta's result is bitwise the same alone, in a batch, and on a
    repeated call."""
    rng = np.random.default_rng(5000)
    n, d = 700, 5
    X = inputs.lhs_design(n, d, rng)
    y = inputs.sine_response(X, rng)
    th = inputs.log_uniform_theta(9, d, 0.05, 20, rng)
    ds = gp.Dataset(X, y, 1.95, 1e-6)
    a = to_host(gp.nll_batch(ds, th))
    b = to_host(gp.nll_batch(ds, th))
    c = to_host(gp.nll_batch(ds, th[4:5]))
    for k in ("logdet", "mu", "sigma2", "nll"):
        assert np.array_equal(a[k], b[k])
        assert a[k][4] == c[k][0]


# ---------------------------------------------------------------------------
# Full-size workloads, sampled thetas (expected values from the oracle only)

def _expected(name):
    path = os.path.join(HERE, "golden", f"{name}_expected.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    return json.load(open(path))


def test_fullsize_fp64_n4096_d8_sampled(gp):
    """The benchmarked launch: n=4096, d=8, p=1.95, nugget 1e-6, 128 thetas,
    one gp_nll_batch call; sampled thetas against the stored oracle values."""
    exp = _expected("fp64_n4096_d8")
    w = inputs.fp64_at_scale()
    assert w.X.shape == (4096, 8) and w.B == 128
    print("[parity] fullsize fp64 n=4096 d=8 B=128", flush=True)
    got = run_gpu(gp, w.X, w.y, w.theta, w.p, w.delta)
    assert np.all(got["info"] == 0)
    sc = scales(w.y)
    for rec in exp["samples"]:
        t = rec["index"]
        for k in ("logdet", "mu", "sigma2", "nll"):
            ref = rec["f80"][k]
            err = abs(got[k][t] - ref) / max(abs(ref), sc[k])
            tol = max(1e-10, 10 * max(rec["err64"][k], rec["err64_lapack"][k]))
            assert err <= tol, (t, k, got[k][t], ref, err, tol)
    # properties at every theta: Hadamard bound, finite outputs, sigma2 > 0
    assert np.all(got["logdet"] <= w.n * math.log1p(w.delta) + 1e-9)
    assert np.all(got["sigma2"] > 0) and np.all(np.isfinite(got["nll"]))


# ---------------------------------------------------------------------------
# Mixed precision (FP32-MFMA trailing updates): errors are reported against
# the oracle; they are bounded only loosely because they scale with the
# conditioning of R.

def test_mixed_fast_single_panel_factor_is_fp64(gp):
    """Without a trailing update (n <= 512, one outer panel) the mixed mode factors
    with the FP64 kernels only: log|R| is bitwise the FP64 one, and the
    refined mu and sigma2 stay within the FP64 tolerance."""
    w = inputs.small_2d()
    ds = gp.Dataset(w.X, w.y, w.p, w.delta)
    a = to_host(gp.nll_batch(ds, w.theta, prec="fp64"))
    b = to_host(gp.nll_batch(ds, w.theta, prec="mixed_fast"))
    assert np.array_equal(a["logdet"], b["logdet"])
    r64 = oracle.nll_batch(w.X, w.y, w.theta, w.p, w.delta)
    r80 = oracle.nll_batch(w.X, w.y, w.theta, w.p, w.delta, extended=True)
    tol = tolerances(r64, r80, w.y, lapack_fp64(w.X, w.y, w.theta, w.p, w.delta))
    sc = scales(w.y)
    for k in ("mu", "sigma2", "nll"):
        e = oracle.rel(b[k], getattr(r80, k), sc[k])
        assert np.all(e <= 100 * tol[k]), (k, e.max())


@pytest.mark.parametrize("n,d,p", [(1500, 8, 1.95), (2048, 6, 2.0)])
def test_mixed_fast_errors_reported(gp, n, d, p):
    """Mixed results are either refined (ir_iters == 2, mu and sigma2 at the
    FP64 level) or, where the FP32 updates broke positive definiteness or the
    refinement stalled, recomputed in FP64 inside the same call
    (ir_iters == -1): those must be bitwise the FP64 path's results."""
    rng = np.random.default_rng(6000 + n)
    X = inputs.lhs_design(n, d, rng)
    y = inputs.sine_response(X, rng)
    th = inputs.log_uniform_theta(6, d, 0.05, 20, rng)
    print(f"[parity] mixed_fast n={n} d={d}", flush=True)
    ds = gp.Dataset(X, y, p, 1e-6)
    got = to_host(gp.nll_batch(ds, th, prec="mixed_fast"))
    ref64 = to_host(gp.nll_batch(ds, th, prec="fp64"))
    r80 = oracle.nll_batch(X, y, th, p, 1e-6, extended=True)
    assert np.all(got["info"] == 0) and np.all(r80.info == 0), got["info"]
    assert np.all(np.isin(got["ir_iters"], [2, -1])), got["ir_iters"]
    fb = got["ir_iters"] == -1
    for k in ("logdet", "mu", "sigma2", "nll"):
        assert np.array_equal(got[k][fb], ref64[k][fb]), k
    sc = scales(y)
    errs = {k: oracle.rel(got[k], getattr(r80, k), sc[k]) for k in ("logdet", "mu", "sigma2", "nll")}
    print("mixed_fast max rel err vs 80-bit oracle:", {k: float(v.max()) for k, v in errs.items()},
          "refinement sweeps", got["ir_iters"], flush=True)
    for k in ("logdet", "nll"):
        assert np.all(errs[k] <= 1e-3), (k, errs[k])
    # the refined solves bring mu and sigma2 to the FP64 level (the FP64
    # rounding spread of the oracle and LAPACK, with a wider multiple)
    r64 = oracle.nll_batch(X, y, th, p, 1e-6)
    tol = tolerances(r64, r80, y, lapack_fp64(X, y, th, p, 1e-6))
    for k in ("mu", "sigma2"):
        assert np.all(errs[k] <= 100 * tol[k]), (k, errs[k], tol[k])


def test_mixed_fast_fallback_whole_batch(gp):
    """theta = 0 makes R = 1 1^T + delta I, whose FP32-updated factor is not
    positive definite at small delta; every such theta is recomputed in FP64
    and matches the FP64 path bitwise, while an invalid theta stays -3."""
    rng = np.random.default_rng(77)
    n, d = 600, 3
    X = inputs.lhs_design(n, d, rng)
    y = inputs.sine_response(X, rng)
    th = np.vstack([np.full((3, d), 1e-4), inputs.log_uniform_theta(2, d, 0.5, 5, rng),
                    np.array([[1.0, -1.0, 1.0]])])
    print("[parity] mixed_fast fallback n=600", flush=True)
    ds = gp.Dataset(X, y, 2.0, 1e-7)
    got = to_host(gp.nll_batch(ds, th, prec="mixed_fast"))
    ref64 = to_host(gp.nll_batch(ds, th, prec="fp64"))
    assert got["info"][-1] == -3 and ref64["info"][-1] == -3
    np.testing.assert_array_equal(got["info"], ref64["info"])
    fb = got["ir_iters"] == -1
    assert fb[:3].all(), got["ir_iters"]
    for k in ("logdet", "mu", "sigma2", "nll"):
        assert np.array_equal(got[k][fb], ref64[k][fb]), k
    ok = ref64["info"] == 0
    r80 = oracle.nll_batch(X, y, th[ok], 2.0, 1e-7, extended=True)
    e = oracle.rel(got["nll"][ok], r80.nll, 1.0)
    assert np.all(e[got["ir_iters"][ok] == -1] <= 1e-6), e
