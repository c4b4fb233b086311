"""Genetic-algorithm fits driven by gp_nll_batch (one launch sequence per
generation) against the same driver fed by the FP64 oracle.

The operators are host code tested on the CPU (test_ga.py); here every
objective value the GPU fit used is checked against the oracle at the same
theta, and the whole trajectory (every generation's thetas, the best theta)
must be the one the oracle-driven fit takes."""
import numpy as np
import pytest

import oracle
from paper_1203_1269_amd import ga, inputs
from parity_util import FP64_TOL, lapack_fp64, scales, tolerances

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1203_1269_amd import binding
    binding.lib()
    return binding


def _oracle_objective(w):
    def f(theta):
        r = oracle.nll_batch(w.X, w.y, theta, w.p, w.delta)
        return np.where(r.info == 0, r.nll, np.inf)
    return f


def _first_near_tie(values, eps=1e-10):
    """Index of the first generation whose values lie within eps (relative)
    of another distinct value evaluated so far; len(values) if none.  Up to
    that generation every ranking the GA made is decided by gaps far above
    the FP64 rounding of either code."""
    seen = np.empty(0)
    for gen, v in enumerate(values):
        u = np.unique(np.concatenate([seen, v[np.isfinite(v)]]))
        if u.size > 1 and np.min(np.diff(u) / np.maximum(np.abs(u[1:]), 1.0)) < eps:
            return gen
        seen = u
    return len(values)


@pytest.mark.parametrize("n,d,delta", [(150, 2, 1e-6), (300, 6, 1e-6)])
def test_ga_trajectory_matches_the_oracle_driven_fit(gp, n, d, delta):
    w = inputs.ga_workload(n, d, seed=20 + n, N=10, delta=delta)
    print(f"[parity] GA n={n} d={d} delta={delta} pop=100 gens=20", flush=True)
    ds = gp.Dataset(w.X, w.y, w.p, w.delta)
    g = ga.fit_ga(ds, seed=3, keep_history=True)
    f = _oracle_objective(w)
    c = ga.ga_minimise(f, d, seed=3, keep_history=True)
    assert g.evaluations == c.evaluations == 2000
    # the thetas of generation gstar still come from tie-free decisions
    gstar = _first_near_tie(c.all_values)
    for gen in range(min(gstar + 1, len(c.all_theta))):
        assert np.array_equal(g.all_theta[gen], c.all_theta[gen]), f"parted at generation {gen}"
    if gstar == len(c.all_theta):
        assert np.array_equal(g.theta, c.theta)
        assert abs(g.nll - c.nll) <= 1e-9 * max(1.0, abs(c.nll))
    # every value the GPU fit used, against the oracle at the same theta
    sc = scales(w.y)["nll"]
    nfar = 0
    for gen, (tg, vg) in enumerate(zip(g.all_theta, g.all_values)):
        vc = c.all_values[gen] if gen <= gstar else f(tg)
        ok = np.isfinite(vc)
        assert np.array_equal(ok, np.isfinite(vg)), gen
        e = oracle.rel(vg[ok], vc[ok], sc)
        far = np.nonzero(ok)[0][e > FP64_TOL]
        if far.size:
            # beyond 1e-10 of the FP64 oracle: hold those thetas to the FP64
            # bar (10 x the rounding spread of two FP64 codes, 80-bit reference)
            th = tg[far]
            r64 = oracle.nll_batch(w.X, w.y, th, w.p, w.delta)
            r80 = oracle.nll_batch(w.X, w.y, th, w.p, w.delta, extended=True)
            tol = tolerances(r64, r80, w.y, lapack_fp64(w.X, w.y, th, w.p, w.delta))
            e80 = oracle.rel(vg[far], r80.nll, sc)
            assert np.all(e80 <= tol["nll"]), (gen, far, e80, tol["nll"])
        nfar += far.size
    print("GA best -2logL GPU / oracle-driven:", g.nll, c.nll, "identical through generation",
          gstar, "values beyond 1e-10 of the FP64 oracle:", nfar, flush=True)


def test_ga_fit_at_the_paper_shape(gp):
    """d = 6, n = 1024, no nugget (the paper's Example 2 shape and budget):
    2000 evaluations, the best value is the oracle's at the best theta, and
    a prediction with it scores below the response's spread."""
    w = inputs.ga_workload(1024, 6, seed=31)
    print("[parity] GA fit n=1024 d=6 delta=0", flush=True)
    ds = gp.Dataset(w.X, w.y, w.p, w.delta)
    r = ga.fit_ga(ds, seed=1)
    assert r.evaluations == 2000 and np.isfinite(r.nll)
    ref = oracle.nll_batch(w.X, w.y, r.theta[None, :], w.p, w.delta)
    assert ref.info[0] == 0
    assert oracle.rel(np.array([r.nll]), ref.nll, 1.0)[0] <= 1e-8
    fit, mean, mse = gp.predict(ds, r.theta[None, :], w.Xs)
    sspe = float(((mean[0].cpu().numpy() - w.ys) ** 2).sum())
    assert sspe < 0.01 * float(((w.ys - w.ys.mean()) ** 2).sum()), sspe
